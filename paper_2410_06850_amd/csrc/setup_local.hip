// Level-1 set-up: the local spectral problem of eq. (spepb) on every coarse
// cell, batched in one persistent launch.
//
// For coarse cell i with owned free nodes F_i:
//   K_i Phi = lambda M_i Phi,
//   K_i = sum of k_e K0_e over elements whose 8 nodes are owned by i,
//   M_i = diag of the k-weighted lumped mass of the same elements,
// keep the Lc smallest pairs, M_i-normalised (Phi^T M_i Phi = I).
//
// Solver: Chebyshev-filtered subspace iteration (Zhou & Saad, 2007) on the
// standard form B = M^-1/2 K M^-1/2, whose spectrum lies in [0, 8 lmax(K0)/V]
// for any conductivities.  Each workgroup owns one cell at a time (work queue),
// keeps the cell's conductivities, mass and one block of vectors in LDS and
// the subspace blocks in registers; Rayleigh-Ritz and orthonormalisation use
// a parallel Jacobi eigensolver on the small projected matrices.  Cells with
// at most 16 free nodes are solved densely.
#include "eig_common.h"
#include "setup.h"

namespace msmg {

constexpr int DENSE_MAX = 16;
constexpr int RED_SLOTS = 640;  // block reductions of up to 136 values over 4 waves

struct LocalArgs {
  Geo g;
  Stencil st;
  Hier h;
  Material mat;
  const void* rho;
  int rho_dt;
  const uint32_t* bits;
  double lam_bound;
  int degree;
  int maxit;
  double tol;
  int nl_max;   // LDS capacity in nodes
  int warm;     // start from the basis in Rc64 (previous set-up)
  double* Rc64;
  double* evals;
  int* status;
  unsigned* work;
};

// cos-product start vector j (shell order of (a,b,c) by a^2+b^2+c^2)
MSMG_DEV void shell_index(int j, int& a, int& b, int& c) {
  // the first 20 triples ordered by a^2 + b^2 + c^2, ties by (c, b, a)
  const signed char T[20][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1},
                                {1, 1, 1}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {2, 1, 0}, {1, 2, 0}, {2, 0, 1},
                                {0, 2, 1}, {1, 0, 2}, {0, 1, 2}, {2, 1, 1}, {1, 2, 1}, {1, 1, 2}};
  const int q = j % 20;
  a = T[q][0];
  b = T[q][1];
  c = T[q][2];
}

MSMG_DEV double hash01(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return double(x) * (1.0 / 4294967296.0) - 0.5;
}

template <int M, int BS, int NPT>
__global__ __launch_bounds__(BS) void k_local_eigen(LocalArgs A) {
  extern __shared__ double lds[];
  const int NL = A.nl_max;
  double* V = lds;                  // M * NL : M^-1/2-scaled block for neighbour access
  double* kl = V + M * NL;          // NL : conductivities of internal elements
  double* isq = kl + NL;            // NL : 1/sqrt(m) on free nodes, 0 on fixed
  double* Gm = isq + NL;            // small matrices (16*16 each)
  double* Vm = Gm + 256;
  double* Bm = Vm + 256;
  double* Vs = Bm + 256;
  double* ev = Vs + 256;            // 16
  double* red = ev + 16;            // RED_SLOTS
  int* perm = reinterpret_cast<int*>(red + RED_SLOTS);   // 16
  int* ired = perm + 16;                          // 16
  int* fidx = ired + 16;                          // NL (dense path: free index of a node)
  int* flist = fidx + NL;                         // DENSE_MAX
  __shared__ int s_cell;

  const int tid = threadIdx.x;
  const Geo& g = A.g;
  const Hier& h = A.h;
  const double b_hi = A.lam_bound * 1.0001;
  const double dk = A.mat.kmax - A.mat.kmin;

  while (true) {
    if (tid == 0) s_cell = int(atomicAdd(A.work, 1u));
    __syncthreads();
    const int cell = s_cell;
    __syncthreads();
    if (cell >= h.ncells) break;
    const int cx = cell % h.ncx, cy = (cell / h.ncx) % h.ncy, cz = cell / (h.ncx * h.ncy);
    const int x0 = cell_begin(cx, h.H), x1 = cell_end(cx, h.H, h.ncx, g.nnx);
    const int y0 = cell_begin(cy, h.H), y1 = cell_end(cy, h.H, h.ncy, g.nny);
    const int z0 = cell_begin(cz, h.H), z1 = cell_end(cz, h.H, h.ncz, g.nnz);
    const int nlx = x1 - x0, nly = y1 - y0, nlz = z1 - z0;
    const int nloc = nlx * nly * nlz;
    const int nex = nlx - 1, ney = nly - 1, nez = nlz - 1;
    const int nel = nex * ney * nez;
    // conductivities of the internal elements
    for (int e = tid; e < nel; e += BS) {
      const int ex = e % nex, ey = (e / nex) % ney, ez = e / (nex * ney);
      const long long ge = elem_id(g, x0 + ex, y0 + ey, z0 + ez);
      const double r = (A.rho_dt == DT_F64) ? ((const double*)A.rho)[ge] : double(((const float*)A.rho)[ge]);
      kl[e] = conductivity<double>(r, A.mat.kmin, dk, A.mat.p);
    }
    __syncthreads();
    // lumped mass over internal elements; 1/sqrt on free nodes
    double nfree_d = 0.0, msum = 0.0;
    for (int ln = tid; ln < nloc; ln += BS) {
      const int lx = ln % nlx, ly = (ln / nlx) % nly, lz = ln / (nlx * nly);
      const long long gn = node_id(g, x0 + lx, y0 + ly, z0 + lz);
      double m = 0.0;
      for (int c = 0; c < 8; ++c) {
        const int ex = lx - 1 + (c & 1), ey = ly - 1 + ((c >> 1) & 1), ez = lz - 1 + ((c >> 2) & 1);
        if (ex >= 0 && ex < nex && ey >= 0 && ey < ney && ez >= 0 && ez < nez) m += kl[(ez * ney + ey) * nex + ex];
      }
      m *= g.vol / 8.0;
      const bool fixed = mask_bit(A.bits, gn);
      isq[ln] = (fixed || !(m > 0.0)) ? 0.0 : 1.0 / sqrt(m);
      if (!fixed && m > 0.0) {
        nfree_d += 1.0;
        msum += m;
      }
    }
    nfree_d = block_allsum(nfree_d, red);
    msum = block_allsum(msum, red);
    const int nfree = int(nfree_d + 0.5);
    const int L = min(h.Lc, nfree);

    double X[NPT][M];  // Ritz block (standard form), rows = own nodes
#pragma unroll
    for (int q = 0; q < NPT; ++q)
#pragma unroll
      for (int j = 0; j < M; ++j) X[q][j] = 0.0;
    int status = 0;
    bool tie = false;

    if (nfree == 0) {
      // nothing to solve: zero basis
    } else if (nfree <= DENSE_MAX) {
      // ---- dense path: assemble B on the free nodes and diagonalise it
      if (tid == 0) {
        int k = 0;
        for (int ln = 0; ln < nloc; ++ln) {
          if (isq[ln] > 0.0) {
            flist[k] = ln;
            fidx[ln] = k++;
          } else {
            fidx[ln] = -1;
          }
        }
      }
      __syncthreads();
      const int nf = nfree;
      for (int e = tid; e < nf * nf; e += BS) {
        const int ia = flist[e / nf], ib = flist[e % nf];
        const int ax = ia % nlx, ay = (ia / nlx) % nly, az = ia / (nlx * nly);
        const int bx = ib % nlx, by = (ib / nlx) % nly, bz = ib / (nlx * nly);
        const int dx = bx - ax, dy = by - ay, dz = bz - az;
        double kab = 0.0;
        if (abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) {
          double kk[8];
          for (int c = 0; c < 8; ++c) {
            const int ex = ax - 1 + (c & 1), ey = ay - 1 + ((c >> 1) & 1), ez = az - 1 + ((c >> 2) & 1);
            kk[c] = (ex >= 0 && ex < nex && ey >= 0 && ey < ney && ez >= 0 && ez < nez) ? kl[(ez * ney + ey) * nex + ex] : 0.0;
          }
          double w[27];
          stencil27(A.st, kk, w);
          kab = w[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)];
        }
        Gm[e] = isq[ia] * kab * isq[ib];
      }
      __syncthreads();
      block_jacobi(Gm, Vm, Bm, Vs, ev, perm, nf, red);
#pragma unroll
      for (int q = 0; q < NPT; ++q) {
        const int ln = tid + q * BS;
        if (ln < nloc && isq[ln] > 0.0) {
          const int f = fidx[ln];
#pragma unroll
          for (int j = 0; j < M; ++j) X[q][j] = (j < nf) ? Vs[f * nf + j] : 0.0;
        }
      }
      if (L < nf && ev[L] - ev[L - 1] < 1e-8 * b_hi) tie = true;
      __syncthreads();
    } else {
      // ---- Chebyshev-filtered subspace iteration
      double Y[NPT][M], Z[NPT][M];
      // precompute this thread's stencil weights (node-local, reused for every product)
      auto apply_B = [&](double (&in)[NPT][M], double (&out)[NPT][M]) {
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
          const int ln = tid + q * BS;
          if (ln < nloc) {
#pragma unroll
            for (int j = 0; j < M; ++j) V[j * NL + ln] = isq[ln] * in[q][j];
          }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
          const int ln = tid + q * BS;
#pragma unroll
          for (int j = 0; j < M; ++j) out[q][j] = 0.0;
          if (ln < nloc && isq[ln] > 0.0) {
            const int lx = ln % nlx, ly = (ln / nlx) % nly, lz = ln / (nlx * nly);
            double kk[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
              const int ex = lx - 1 + (c & 1), ey = ly - 1 + ((c >> 1) & 1), ez = lz - 1 + ((c >> 2) & 1);
              kk[c] = (ex >= 0 && ex < nex && ey >= 0 && ey < ney && ez >= 0 && ez < nez) ? kl[(ez * ney + ey) * nex + ex] : 0.0;
            }
            double w[27];
            stencil27(A.st, kk, w);
            // difference form: (K v)_n = sum_{o != 0} w_o (v_{n+o} - v_n)
            double v0[M];
#pragma unroll
            for (int j = 0; j < M; ++j) v0[j] = V[j * NL + ln];
#pragma unroll
            for (int o = 0; o < 27; ++o) {
              if (o == 13) continue;
              const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
              const int nx_ = lx + ox, ny_ = ly + oy, nz_ = lz + oz;
              const bool ok = nx_ >= 0 && nx_ < nlx && ny_ >= 0 && ny_ < nly && nz_ >= 0 && nz_ < nlz;
              const int nb = ok ? (nz_ * nly + ny_) * nlx + nx_ : ln;
              const double wo = ok ? w[o] : 0.0;
#pragma unroll
              for (int j = 0; j < M; ++j) out[q][j] += wo * (V[j * NL + nb] - v0[j]);
            }
            const double s = isq[ln];
#pragma unroll
            for (int j = 0; j < M; ++j) out[q][j] *= s;
          }
        }
        __syncthreads();
      };
      // Gram matrix of a block into Gm (full symmetric)
      auto gram = [&](double (&P)[NPT][M], double (&Q)[NPT][M]) {
        constexpr int NV = M * (M + 1) / 2;
        double s[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] = 0.0;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
          int k = 0;
#pragma unroll
          for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = i; j < M; ++j) s[k++] += P[q][i] * Q[q][j];
        }
        block_allsum_vec<NV>(s, red);
        if (tid == 0) {
          int k = 0;
          for (int i = 0; i < M; ++i)
            for (int j = i; j < M; ++j) {
              Gm[i * M + j] = s[k];
              Gm[j * M + i] = s[k];
              ++k;
            }
        }
        __syncthreads();
      };
      // P <- P C with C (M x M) in LDS
      auto transform = [&](double (&P)[NPT][M], const double* C) {
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
          double t[M];
#pragma unroll
          for (int j = 0; j < M; ++j) {
            double a = 0.0;
#pragma unroll
            for (int i = 0; i < M; ++i) a += P[q][i] * C[i * M + j];
            t[j] = a;
          }
#pragma unroll
          for (int j = 0; j < M; ++j) P[q][j] = t[j];
        }
      };
      // orthonormalise a block: G = P^T P = U S U^T, P <- P U S^-1/2
      auto orthonormalise = [&](double (&P)[NPT][M]) {
        gram(P, P);
        block_jacobi(Gm, Vm, Bm, Vs, ev, perm, M, red);
        for (int e = tid; e < M * M; e += BS) {
          const int k = e % M;
          const double sv = ev[k];
          Bm[e] = (sv > 1e-300) ? Vs[e] / sqrt(sv) : 0.0;
        }
        __syncthreads();
        transform(P, Bm);
        __syncthreads();
      };
      // Rayleigh-Ritz on an orthonormal block P: X = P V, Z = (B P) V, ev = Ritz values
      auto rayleigh_ritz = [&](double (&P)[NPT][M]) {
        apply_B(P, Z);
        gram(P, Z);
        block_jacobi(Gm, Vm, Bm, Vs, ev, perm, M, red);
        transform(P, Vs);
        transform(Z, Vs);
#pragma unroll
        for (int q = 0; q < NPT; ++q)
#pragma unroll
          for (int j = 0; j < M; ++j) X[q][j] = P[q][j];
        __syncthreads();
      };

      // start block: low-frequency cosines on the cell box, times sqrt(m)
#pragma unroll
      for (int q = 0; q < NPT; ++q) {
        const int ln = tid + q * BS;
        if (ln < nloc && isq[ln] > 0.0) {
          const int lx = ln % nlx, ly = (ln / nlx) % nly, lz = ln / (nlx * nly);
          const double sm = 1.0 / isq[ln];
#pragma unroll
          for (int j = 0; j < M; ++j) {
            int a, b, c;
            shell_index(j, a, b, c);
            const double v = cos(M_PI * a * lx / double(max(nlx - 1, 1))) * cos(M_PI * b * ly / double(max(nly - 1, 1))) *
                             cos(M_PI * c * lz / double(max(nlz - 1, 1)));
            Y[q][j] = sm * (v + 1e-2 * hash01(unsigned(ln * 131 + j * 7919 + 17)));
            if (A.warm && j < h.Lc) {
              // previous basis in standard form (Phi sqrt(m)), cosines kept as a small
              // admixture so that empty columns still span a direction
              const long long gn = node_id(g, x0 + lx, y0 + ly, z0 + lz);
              Y[q][j] = A.Rc64[gn * h.Lc + j] * sm + 1e-3 * Y[q][j];
            }
          }
        } else {
#pragma unroll
          for (int j = 0; j < M; ++j) Y[q][j] = 0.0;
        }
      }
      orthonormalise(Y);
      orthonormalise(Y);
      rayleigh_ritz(Y);
      double a_lo = ev[M - 1], a_min = ev[0];
      int it = 0;
      bool conv = false;
      while (true) {
        // residuals of the wanted pairs
        double rs[M];
#pragma unroll
        for (int j = 0; j < M; ++j) rs[j] = 0.0;
#pragma unroll
        for (int q = 0; q < NPT; ++q)
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const double r = Z[q][j] - ev[j] * X[q][j];
            rs[j] += r * r;
          }
        block_allsum_vec<M>(rs, red);
        double worst = 0.0;
        for (int j = 0; j < L; ++j) worst = fmax(worst, rs[j]);
        if (worst <= (A.tol * b_hi) * (A.tol * b_hi)) {
          conv = true;
          break;
        }
        if (it >= A.maxit) break;
        ++it;
        // Chebyshev filter damping [a_lo, b_hi], scaled by the lower end a_min
        double lo = a_lo;
        if (!(lo < 0.95 * b_hi)) lo = 0.95 * b_hi;
        const double e = 0.5 * (b_hi - lo), cc = 0.5 * (b_hi + lo);
        double amin = a_min;
        if (!(amin < lo - 1e-3 * e)) amin = lo - 1e-3 * e;
        // keep the amplification of the block below ~1e6 so its Gram matrix stays well conditioned
        const double xs = (cc - amin) / e;
        int deg = A.degree;
        if (xs > 1.0) {
          const int dmax = int(14.5 / acosh(xs));
          deg = max(2, min(deg, dmax));
        }
        double sigma = e / (amin - cc);
        const double tau = 2.0 / sigma;
        // Y <- (B X - c X) sigma / e   (X holds the Ritz block, Z = B X)
#pragma unroll
        for (int q = 0; q < NPT; ++q)
#pragma unroll
          for (int j = 0; j < M; ++j) Y[q][j] = (Z[q][j] - cc * X[q][j]) * (sigma / e);
        for (int d = 2; d <= deg; ++d) {
          const double sn = 1.0 / (tau - sigma);
          apply_B(Y, Z);
#pragma unroll
          for (int q = 0; q < NPT; ++q)
#pragma unroll
            for (int j = 0; j < M; ++j) {
              const double yn = (Z[q][j] - cc * Y[q][j]) * (2.0 * sn / e) - (sigma * sn) * X[q][j];
              X[q][j] = Y[q][j];
              Y[q][j] = yn;
            }
          sigma = sn;
        }
        orthonormalise(Y);
        orthonormalise(Y);
        rayleigh_ritz(Y);
        a_lo = ev[M - 1];
        a_min = ev[0];
      }
      status = min(it, 0xFFFFF) | (conv ? 0 : (1 << 28));
      if (L < M && ev[L] - ev[L - 1] < 1e-8 * b_hi) tie = true;
    }

    // ---- normalise the sign and write R_c (Phi = M^-1/2 w) and eigenvalues
    double sdot[M];
#pragma unroll
    for (int j = 0; j < M; ++j) sdot[j] = 0.0;
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int ln = tid + q * BS;
      if (ln < nloc && isq[ln] > 0.0) {
#pragma unroll
        for (int j = 0; j < M; ++j) sdot[j] += X[q][j] / isq[ln];  // sum_n m_n Phi_n
      }
    }
    block_allsum_vec<M>(sdot, red);
    double sgn[M];
    for (int j = 0; j < M; ++j) {
      if (j >= L) {
        sgn[j] = 0.0;
        continue;
      }
      if (fabs(sdot[j]) > 1e-8 * sqrt(msum)) {
        sgn[j] = sdot[j] > 0.0 ? 1.0 : -1.0;
      } else {
        double amax = 0.0;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
          const int ln = tid + q * BS;
          if (ln < nloc) amax = fmax(amax, fabs(X[q][j] * isq[ln]));
        }
        amax = block_allmax(amax, red);
        int first = 1 << 30;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
          const int ln = tid + q * BS;
          if (ln < nloc && fabs(X[q][j] * isq[ln]) >= (1.0 - 1e-8) * amax) first = min(first, ln);
        }
        first = block_allmin_int(first, ired);
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
          const int ln = tid + q * BS;
          if (ln == first) v = X[q][j];
        }
        v = block_allsum(v, red);
        sgn[j] = v > 0.0 ? 1.0 : -1.0;
      }
    }
    const int Lc = h.Lc;
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      const int ln = tid + q * BS;
      if (ln < nloc) {
        const int lx = ln % nlx, ly = (ln / nlx) % nly, lz = ln / (nlx * nly);
        const long long gn = node_id(g, x0 + lx, y0 + ly, z0 + lz);
        for (int l = 0; l < Lc; ++l) {
          double v = 0.0;
#pragma unroll
          for (int j = 0; j < M; ++j)
            if (j == l) v = X[q][j];
          A.Rc64[gn * Lc + l] = (l < L) ? sgn[l] * v * isq[ln] : 0.0;
        }
      }
    }
    if (tid == 0) {
      for (int l = 0; l < Lc; ++l) A.evals[(long long)cell * Lc + l] = (l < L) ? ev[l] : 0.0;
      // bits 0-19 outer iterations, 20-27 basis size, 28 not converged, 29 cutoff tie
      A.status[cell] = status | (L << 20) | (tie ? (1 << 29) : 0);
    }
    __syncthreads();
  }
}

// LDS bytes of one workgroup
static size_t local_lds_bytes(int M, int nl) {
  return sizeof(double) * (size_t(M) * nl + 2 * size_t(nl) + 4 * 256 + 16 + RED_SLOTS) + sizeof(int) * (16 + 16 + size_t(nl) + DENSE_MAX);
}

template <int M, int BS, int NPT>
static void launch_local_t(const LocalArgs& a, int blocks, hipStream_t s) {
  const size_t lds = local_lds_bytes(M, a.nl_max);
  (void)hipFuncSetAttribute((const void*)k_local_eigen<M, BS, NPT>, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  hipLaunchKernelGGL((k_local_eigen<M, BS, NPT>), dim3(blocks), dim3(BS), lds, s, a);
}

int launch_local_eigen(const Ctx& c, const SetupArgs& sa, SetupScratch* sc, int bs, int m, int degree, int blocks,
                       hipStream_t s) {
  LocalArgs a;
  a.g = c.g;
  a.st = c.st;
  a.h = c.h;
  a.mat = c.mat;
  a.rho = c.rho;
  a.rho_dt = c.rho_dt;
  a.bits = c.bits;
  a.lam_bound = sa.lam_bound;
  a.degree = degree;
  a.maxit = sa.opt->eig_maxit;
  a.tol = sa.opt->eig_tol;
  a.nl_max = sa.max_cell_nodes;
  a.warm = sa.warm;
  a.Rc64 = sa.Rc64;
  a.evals = sa.evals;
  a.status = sa.cell_status;
  a.work = sc->work;
  if (m < c.h.Lc + 1) return MSMG_EINVAL;
  if (local_lds_bytes(m, a.nl_max) > 160 * 1024) return MSMG_EINVAL;
  if (hipMemsetAsync(sc->work, 0, sizeof(unsigned), s) != hipSuccess) return MSMG_EHIP;
  const int npt = (a.nl_max + bs - 1) / bs;
#define LL(M_, BS_, NPT_)                               \
  if (m == M_ && bs == BS_ && npt <= NPT_) {            \
    launch_local_t<M_, BS_, NPT_>(a, blocks, s);        \
    return hipGetLastError() == hipSuccess ? MSMG_OK : MSMG_EHIP; \
  }
  LL(8, 256, 1)
  LL(8, 256, 2)
  LL(8, 256, 3)
  LL(8, 256, 4)
  LL(8, 512, 1)
  LL(8, 512, 2)
#undef LL
  return MSMG_EINVAL;
}

}  // namespace msmg
