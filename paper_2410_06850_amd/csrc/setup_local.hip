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
// for any conductivities.  Each workgroup owns one cell at a time (work queue)
// and keeps the cell's conductivities, mass and two blocks of vectors in LDS;
// the filter recurrence, the Gram matrices and the block rotations work node
// by node on those buffers, so registers only hold per-node temporaries.
// Rayleigh-Ritz and orthonormalisation use a parallel Jacobi eigensolver on
// the small projected matrices.  Cells with
// at most 16 free nodes are solved densely.
#include "eig_common.h"
#include "setup.h"

namespace msmg {

constexpr int DENSE_MAX = 16;
#ifndef MSMG_LOCAL_CHOLQR
#define MSMG_LOCAL_CHOLQR 1  // orthonormalise by Cholesky-QR (else always by the eigen-decomposition)
#endif
constexpr int RED_SLOTS = 256;  // block reductions of up to 16 values over 16 waves
// doubles of the second subspace block: it also holds the dense path's four
// DENSE_MAX^2 matrices and its node index lists
MSMG_HD constexpr size_t local_blk1_words(int M, int nl) {
  return (size_t(M) * nl > 4 * DENSE_MAX * DENSE_MAX + (size_t(nl) + DENSE_MAX + 1) / 2 + 1)
             ? size_t(M) * nl
             : 4 * DENSE_MAX * DENSE_MAX + (size_t(nl) + DENSE_MAX + 1) / 2 + 1;
}

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
  int nl_max;   // LDS capacity in nodes (the largest cell of the class)
  double lc_thr;  // > 0: keep the eigenpairs with lambda <= lc_thr (at least one)
  int warm;     // start from the basis in Rc64 (previous set-up)
  const int* cells;  // the class's cells: cells[0 .. ncells)
  int ncells;   // cells to solve
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

// NLC: the LDS capacity per vector as a compile-time constant (the common
// cell sizes), so that the vector strides become immediate offsets; 0 takes
// it from the arguments.  TP: the cell-centred two-point flux problem of the
// same equation (unknowns are the cells of the coarse cell, K_i the TPFA form
// of its internal faces, M_i = diag(k_K |K|)).
template <int M, int BS, int NLC, bool TP>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(BS <= 512 ? 2 * BS / 256 : 1)))
void k_local_eigen(LocalArgs A) {
  extern __shared__ double lds[];
  const int NL = NLC > 0 ? NLC : A.nl_max;
  // Both subspace blocks live in LDS (node-contiguous per vector); registers
  // only hold per-node temporaries, so the kernel runs without spilling.
  double* blk0 = lds;               // M * NL : block buffer
  double* blk1 = blk0 + M * NL;     // local_blk1_words : block buffer
  double* kl = blk1 + local_blk1_words(M, NL);  // NL : conductivities of internal elements
  double* isq = kl + NL;            // NL : 1/sqrt(m) on free nodes, 0 on fixed
  double* Gm = isq + NL;            // small matrices (M*M each)
  double* Vm = Gm + M * M;
  double* Bm = Vm + M * M;
  double* Vs = Bm + M * M;
  double* ev = Vs + M * M;          // 16
  double* red = ev + 16;            // RED_SLOTS
  int* perm = reinterpret_cast<int*>(red + RED_SLOTS);   // 16
  int* ired = perm + 16;                          // 16
  // the dense path (at most DENSE_MAX free nodes) works in the second block
  double* Gd = blk1;                              // DENSE_MAX^2 each
  double* Vd = Gd + DENSE_MAX * DENSE_MAX;
  double* Bd = Vd + DENSE_MAX * DENSE_MAX;
  double* Vsd = Bd + DENSE_MAX * DENSE_MAX;
  int* fidx = reinterpret_cast<int*>(Vsd + DENSE_MAX * DENSE_MAX);  // NL: free index of a node
  int* flist = fidx + NL;                         // DENSE_MAX
  __shared__ int s_cell;

  const int tid = threadIdx.x;
  const int wid = tid >> 6, lane = tid & 63;
  constexpr int NW = BS / 64;
  const Geo& g = A.g;
  const Hier& h = A.h;
  const double b_hi = A.lam_bound * 1.0001;
  const double dk = A.mat.kmax - A.mat.kmin;
  const double pat_ax[3] = {A.st.ax[0], A.st.ax[1], A.st.ax[2]};
  const double pat_fd[3] = {A.st.fd[0], A.st.fd[1], A.st.fd[2]};
  const double pat_bd = A.st.bd;
  // TP: face weights |F| / h_d
  const double tw[3] = {g.hy * g.hz / g.hx, g.hx * g.hz / g.hy, g.hx * g.hy / g.hz};

  while (true) {
    if (tid == 0) s_cell = int(atomicAdd(A.work, 1u));
    __syncthreads();
    const int wi = s_cell;
    __syncthreads();
    if (wi >= A.ncells) break;
    const int cell = A.cells[wi];
    const int cx = cell % h.ncx, cy = (cell / h.ncx) % h.ncy, cz = cell / (h.ncx * h.ncy);
    const int x0 = cell_begin(cx, h.H), x1 = cell_end(cx, h.H, h.ncx, g.nnx);
    const int y0 = cell_begin(cy, h.H), y1 = cell_end(cy, h.H, h.ncy, g.nny);
    const int z0 = cell_begin(cz, h.H), z1 = cell_end(cz, h.H, h.ncz, g.nnz);
    const int nlx = x1 - x0, nly = y1 - y0, nlz = z1 - z0;
    const int nloc = nlx * nly * nlz;
    const int nex = nlx - 1, ney = nly - 1, nez = nlz - 1;
    const int nel = TP ? nloc : nex * ney * nez;
    // conductivities of the internal elements (of the cells for TP)
    if (TP) {
      for (int e = tid; e < nloc; e += BS) {
        const int ex = e % nlx, ey = (e / nlx) % nly, ez = e / (nlx * nly);
        const long long gc = node_id(g, x0 + ex, y0 + ey, z0 + ez);
        const double r = (A.rho_dt == DT_F64) ? ((const double*)A.rho)[gc] : double(((const float*)A.rho)[gc]);
        kl[e] = conductivity<double>(r, A.mat.kmin, dk, A.mat.p);
      }
    } else for (int e = tid; e < nel; e += BS) {
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
      if (TP) {
        m = kl[ln] * g.vol;
        isq[ln] = m > 0.0 ? 1.0 / sqrt(m) : 0.0;
        if (m > 0.0) {
          nfree_d += 1.0;
          msum += m;
        }
        continue;
      }
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

    // X = the block holding the Ritz vectors at the end (standard form)
    double* X = blk0;
    double* Y = blk1;
    int status = 0;
    bool tie = false;

    // (B v)_n for all M vectors of block P at local node ln (standard form:
    // B = M^-1/2 K M^-1/2, K in difference form with per-offset weights)
    auto apply_node = [&](const double* P, int ln, double* out) {
      const int lx = ln % nlx, ly = (ln / nlx) % nly, lz = ln / (nlx * nly);
      if constexpr (TP) {
        // faces to the six neighbours inside the coarse cell: T = w_d 2 k k' / (k + k')
        const double s0 = isq[ln], k0 = kl[ln];
        double v0[M];
#pragma unroll
        for (int j = 0; j < M; ++j) {
          v0[j] = s0 * P[j * NL + ln];
          out[j] = 0.0;
        }
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          const int a = f / 2, sd = (f & 1) ? 1 : -1;
          const int p = (a == 0 ? lx : (a == 1 ? ly : lz)) + sd;
          const int na = a == 0 ? nlx : (a == 1 ? nly : nlz);
          const bool in = p >= 0 && p < na;
          const int step = a == 0 ? 1 : (a == 1 ? nlx : nlx * nly);
          const int nb = in ? ln + sd * step : ln;
          const double kn = kl[nb], sb = isq[nb];
          const double T = in ? tw[a] * (2.0 * k0 * kn / (k0 + kn)) : 0.0;
          double pv[M];
#pragma unroll
          for (int j = 0; j < M; ++j) pv[j] = P[j * NL + nb];
#pragma unroll
          for (int j = 0; j < M; ++j) out[j] += T * (v0[j] - sb * pv[j]);
        }
#pragma unroll
        for (int j = 0; j < M; ++j) out[j] *= s0;
        return;
      }
      double kk[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int ex = lx - 1 + (c & 1), ey = ly - 1 + ((c >> 1) & 1), ez = lz - 1 + ((c >> 2) & 1);
        kk[c] = (ex >= 0 && ex < nex && ey >= 0 && ey < ney && ez >= 0 && ez < nez) ? kl[(ez * ney + ey) * nex + ex] : 0.0;
      }
      const double s0 = isq[ln];
      double v0[M];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        v0[j] = s0 * P[j * NL + ln];
        out[j] = 0.0;
      }
#pragma unroll
      for (int o = 0; o < 27; ++o) {
        if (o == 13) continue;
        const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
        const int nd = (ox != 0) + (oy != 0) + (oz != 0);
        double pat;
        if (nd == 3) pat = pat_bd;
        else if (nd == 1) pat = pat_ax[ox != 0 ? 0 : (oy != 0 ? 1 : 2)];
        else pat = pat_fd[ox == 0 ? 0 : (oy == 0 ? 1 : 2)];
        if (nd == 1 && pat == 0.0) continue;  // axis neighbours vanish on cubes
        double ks = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int ccx = c & 1, ccy = (c >> 1) & 1, ccz = (c >> 2) & 1;
          const bool okx = (ox == 0) || (ox > 0 && ccx == 1) || (ox < 0 && ccx == 0);
          const bool oky = (oy == 0) || (oy > 0 && ccy == 1) || (oy < 0 && ccy == 0);
          const bool okz = (oz == 0) || (oz > 0 && ccz == 1) || (oz < 0 && ccz == 0);
          if (okx && oky && okz) ks += kk[c];
        }
        // a neighbour outside the cell box shares only absent elements with
        // the node (ks = 0): its clamped index reads some local node's finite
        // values, weighted by zero.  No branch, so the loads of consecutive
        // neighbours can be in flight together.
        const int nb = min(max(ln + (oz * nly + oy) * nlx + ox, 0), nloc - 1);
        const double wo = pat * ks, sb = isq[nb];
        double pv[M];
#pragma unroll
        for (int j = 0; j < M; ++j) pv[j] = P[j * NL + nb];
#pragma unroll
        for (int j = 0; j < M; ++j) out[j] += wo * (sb * pv[j] - v0[j]);
      }
#pragma unroll
      for (int j = 0; j < M; ++j) out[j] *= s0;
    };
    // Gram matrix P^T Q into Gm: each wave forms whole dot products (fixed order)
    auto gram = [&](const double* P, const double* Q) {
      constexpr int NV = M * (M + 1) / 2;
      for (int k = wid; k < NV; k += NW) {
        int i = 0, r = k;
        while (r >= M - i) {
          r -= M - i;
          ++i;
        }
        const int j = i + r;
        double acc = 0.0;
        for (int n = lane; n < nloc; n += 64) acc += P[i * NL + n] * Q[j * NL + n];
        acc = wave_sum(acc);
        if (lane == 0) {
          Gm[i * M + j] = acc;
          Gm[j * M + i] = acc;
        }
      }
      __syncthreads();
    };
    // P <- P C (C is M x M in LDS), node by node in place
    auto transform = [&](double* P, const double* C) {
      for (int ln = tid; ln < nloc; ln += BS) {
        // keeps the M x M coefficients in LDS instead of hoisting them into registers
        asm volatile("" ::: "memory");
        double t[M], u[M];
#pragma unroll
        for (int i = 0; i < M; ++i) t[i] = P[i * NL + ln];
#pragma unroll
        for (int j = 0; j < M; ++j) {
          double a = 0.0;
#pragma unroll
          for (int i = 0; i < M; ++i) a += t[i] * C[i * M + j];
          u[j] = a;
        }
#pragma unroll
        for (int j = 0; j < M; ++j) P[j * NL + ln] = u[j];
      }
      __syncthreads();
    };
    // eigen-decomposition of the M x M matrix in Gm -> ev (ascending), Vs
    auto small_eig = [&]() {
      if constexpr (M == 8) {
        if (wid == 0) wave_jacobi8(Gm, Vs, ev);
        __syncthreads();
      } else {
        block_jacobi(Gm, Vm, Bm, Vs, ev, perm, M, red, red + 32);
      }
    };
    // orthonormalise a block from G = P^T P: P <- P R^-1 with the Cholesky
    // factor R (two such passes make the block orthonormal to rounding for any
    // condition the filter leaves); where G is not safely positive definite,
    // the symmetric transform G = U S U^T, P <- P U S^-1/2, which drops null
    // directions
    __shared__ int s_chol;
    auto orthonormalise = [&](double* P) {
      gram(P, P);
      if constexpr (M == 8 && MSMG_LOCAL_CHOLQR) {
        if (wid == 0) {
          const bool ok = wave_cholinv8(Gm, Bm);
          if (lane == 0) s_chol = ok ? 1 : 0;
        }
        __syncthreads();
        if (s_chol) {
          transform(P, Bm);
          return;
        }
      }
      small_eig();
      for (int e = tid; e < M * M; e += BS) {
        const int k = e % M;
        const double sv = ev[k];
        Bm[e] = (sv > 1e-300) ? Vs[e] / sqrt(sv) : 0.0;
      }
      __syncthreads();
      transform(P, Bm);
    };
    // Rayleigh-Ritz on an orthonormal block P: Q = B P, then both rotated by
    // the eigenvectors of P^T Q; ev = Ritz values
    auto rayleigh_ritz = [&](double* P, double* Q) {
      for (int ln = tid; ln < nloc; ln += BS) {
        double z[M];
        apply_node(P, ln, z);
#pragma unroll
        for (int j = 0; j < M; ++j) Q[j * NL + ln] = z[j];
      }
      __syncthreads();
      gram(P, Q);
      small_eig();
      transform(P, Vs);
      transform(Q, Vs);
    };

    if (nfree == 0) {
      for (int e = tid; e < M * NL; e += BS) X[e] = 0.0;
      __syncthreads();
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
        if (TP) {
          const int ad = abs(dx) + abs(dy) + abs(dz);
          if (ad == 0) {
            // diagonal: the sum of the cell's internal face transmissibilities
            for (int f = 0; f < 6; ++f) {
              const int a = f / 2, sd = (f & 1) ? 1 : -1;
              const int p = (a == 0 ? ax : (a == 1 ? ay : az)) + sd;
              const int na = a == 0 ? nlx : (a == 1 ? nly : nlz);
              if (p < 0 || p >= na) continue;
              const int nb = ia + sd * (a == 0 ? 1 : (a == 1 ? nlx : nlx * nly));
              kab += tw[a] * (2.0 * kl[ia] * kl[nb] / (kl[ia] + kl[nb]));
            }
          } else if (ad == 1) {
            const int a = dx != 0 ? 0 : (dy != 0 ? 1 : 2);
            kab = -tw[a] * (2.0 * kl[ia] * kl[ib] / (kl[ia] + kl[ib]));
          }
        } else if (abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) {
          double kk[8];
          for (int c = 0; c < 8; ++c) {
            const int ex = ax - 1 + (c & 1), ey = ay - 1 + ((c >> 1) & 1), ez = az - 1 + ((c >> 2) & 1);
            kk[c] = (ex >= 0 && ex < nex && ey >= 0 && ey < ney && ez >= 0 && ez < nez) ? kl[(ez * ney + ey) * nex + ex] : 0.0;
          }
          double w[27];
          stencil27(A.st, kk, w);
          kab = w[(dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)];
        }
        Gd[e] = isq[ia] * kab * isq[ib];
      }
      __syncthreads();
      block_jacobi(Gd, Vd, Bd, Vsd, ev, perm, nf, red, red + 32);
      for (int e = tid; e < M * NL; e += BS) {
        const int j = e / NL, ln = e % NL;
        double v = 0.0;
        if (ln < nloc && isq[ln] > 0.0 && j < nf) v = Vsd[fidx[ln] * nf + j];
        X[e] = v;
      }
      if (L < nf && ev[L] - ev[L - 1] < 1e-8 * b_hi) tie = true;
      __syncthreads();
    } else {
      // ---- Chebyshev-filtered subspace iteration (two LDS blocks: X, Y)
      // start block: low-frequency cosines on the cell box, times sqrt(m), or
      // the previous set-up's basis (warm start)
      for (int ln = tid; ln < nloc; ln += BS) {
        const int lx = ln % nlx, ly = (ln / nlx) % nly, lz = ln / (nlx * nly);
        const bool fr = isq[ln] > 0.0;
        const double sm = fr ? 1.0 / isq[ln] : 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
          double y = 0.0;
          if (fr) {
            int a, b, c;
            shell_index(j, a, b, c);
            const double v = cos(M_PI * a * lx / double(max(nlx - 1, 1))) * cos(M_PI * b * ly / double(max(nly - 1, 1))) *
                             cos(M_PI * c * lz / double(max(nlz - 1, 1)));
            y = sm * (v + 1e-2 * hash01(unsigned(ln * 131 + j * 7919 + 17)));
            if (A.warm && j < h.Lc) {
              // previous basis in standard form (Phi sqrt(m)), cosines kept as a small
              // admixture so that empty columns still span a direction
              const long long gn = node_id(g, x0 + lx, y0 + ly, z0 + lz);
              y = A.Rc64[gn * h.Lc + j] * sm + 1e-3 * y;
            }
          }
          Y[j * NL + ln] = y;
        }
      }
      __syncthreads();
      orthonormalise(Y);
      orthonormalise(Y);
      rayleigh_ritz(Y, X);  // Ritz vectors in Y, B Y in X
      {
        double* t = X;
        X = Y;
        Y = t;  // X: Ritz vectors, Y: B X
      }
      double a_lo = ev[M - 1], a_min = ev[0];
      int it = 0;
      bool conv = false;
      while (true) {
        // residuals of the wanted pairs
        double rs[M];
#pragma unroll
        for (int j = 0; j < M; ++j) rs[j] = 0.0;
        for (int ln = tid; ln < nloc; ln += BS) {
#pragma unroll
          for (int j = 0; j < M; ++j) {
            const double r = Y[j * NL + ln] - ev[j] * X[j * NL + ln];
            rs[j] += r * r;
          }
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
        // Y1 = (B X - c X) sigma / e, written over B X
        for (int ln = tid; ln < nloc; ln += BS) {
#pragma unroll
          for (int j = 0; j < M; ++j) Y[j * NL + ln] = (Y[j * NL + ln] - cc * X[j * NL + ln]) * (sigma / e);
        }
        __syncthreads();
        // three-term recurrence Y_{d} = (2 sn / e)(B - c) Y_{d-1} - sigma sn Y_{d-2}; the
        // new block overwrites Y_{d-2} node by node (nothing else reads it)
        for (int d = 2; d <= deg; ++d) {
          const double sn = 1.0 / (tau - sigma);
          for (int ln = tid; ln < nloc; ln += BS) {
            double z[M];
            apply_node(Y, ln, z);
#pragma unroll
            for (int j = 0; j < M; ++j)
              X[j * NL + ln] = (z[j] - cc * Y[j * NL + ln]) * (2.0 * sn / e) - (sigma * sn) * X[j * NL + ln];
          }
          __syncthreads();
          double* t = X;
          X = Y;
          Y = t;  // Y: newest iterate, X: the previous one
          sigma = sn;
        }
        orthonormalise(Y);
        orthonormalise(Y);
        rayleigh_ritz(Y, X);
        {
          double* t = X;
          X = Y;
          Y = t;  // X: Ritz vectors, Y: B X
        }
        a_lo = ev[M - 1];
        a_min = ev[0];
      }
      status = min(it, 0xFFFFF) | (conv ? 0 : (1 << 28));
      if (L < M && ev[L] - ev[L - 1] < 1e-8 * b_hi) tie = true;
    }

    // adaptive basis size: the pairs at or below the threshold, at least one
    // (ev holds the computed pairs in ascending order)
    int Lk = L;
    if (A.lc_thr > 0.0 && L > 1) {
      int cnt = 0;
      for (int j = 0; j < L; ++j) cnt += ev[j] <= A.lc_thr ? 1 : 0;
      Lk = max(1, cnt);
      const int nev = nfree <= DENSE_MAX ? nfree : M;
      tie = Lk < nev && ev[Lk] - ev[Lk - 1] < 1e-8 * b_hi;
    }

    // ---- normalise the sign and write R_c (Phi = M^-1/2 w) and eigenvalues
    double sdot[M];
#pragma unroll
    for (int j = 0; j < M; ++j) sdot[j] = 0.0;
    for (int ln = tid; ln < nloc; ln += BS) {
      if (isq[ln] > 0.0) {
#pragma unroll
        for (int j = 0; j < M; ++j) sdot[j] += X[j * NL + ln] / isq[ln];  // sum_n m_n Phi_n
      }
    }
    block_allsum_vec<M>(sdot, red);
    double sgn[M];
    for (int j = 0; j < M; ++j) {
      if (j >= Lk) {
        sgn[j] = 0.0;
        continue;
      }
      if (fabs(sdot[j]) > 1e-8 * sqrt(msum)) {
        sgn[j] = sdot[j] > 0.0 ? 1.0 : -1.0;
      } else {
        double amax = 0.0;
        for (int ln = tid; ln < nloc; ln += BS) amax = fmax(amax, fabs(X[j * NL + ln] * isq[ln]));
        amax = block_allmax(amax, red);
        int first = 1 << 30;
        for (int ln = tid; ln < nloc; ln += BS)
          if (fabs(X[j * NL + ln] * isq[ln]) >= (1.0 - 1e-8) * amax) first = min(first, ln);
        first = block_allmin_int(first, ired);
        const double v = X[j * NL + first];
        sgn[j] = v > 0.0 ? 1.0 : -1.0;
      }
    }
    const int Lc = h.Lc;
    for (int ln = tid; ln < nloc; ln += BS) {
      const int lx = ln % nlx, ly = (ln / nlx) % nly, lz = ln / (nlx * nly);
      const long long gn = node_id(g, x0 + lx, y0 + ly, z0 + lz);
      for (int l = 0; l < Lc; ++l) A.Rc64[gn * Lc + l] = (l < Lk) ? sgn[l] * X[l * NL + ln] * isq[ln] : 0.0;
    }
    if (tid == 0) {
      for (int l = 0; l < Lc; ++l) A.evals[(long long)cell * Lc + l] = (l < Lk) ? ev[l] : 0.0;
      // bits 0-19 outer iterations, 20-27 basis size, 28 not converged, 29 cutoff tie
      A.status[cell] = status | (Lk << 20) | (tie ? (1 << 29) : 0);
    }
    __syncthreads();
  }
}

// LDS bytes of one workgroup
size_t local_lds_bytes(int M, int nl) {
  return sizeof(double) * (size_t(M) * nl + local_blk1_words(M, nl) + 2 * size_t(nl) + 4 * size_t(M) * M + 16 +
                           RED_SLOTS) +
         sizeof(int) * (16 + 16);
}

template <int M, int BS, int NLC, bool TP>
static void launch_local_t(const LocalArgs& a, int blocks, hipStream_t s) {
  const size_t lds = local_lds_bytes(M, a.nl_max);
  (void)hipFuncSetAttribute((const void*)k_local_eigen<M, BS, NLC, TP>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            int(lds));
  hipLaunchKernelGGL((k_local_eigen<M, BS, NLC, TP>), dim3(blocks), dim3(BS), lds, s, a);
}

int launch_local_eigen(const Ctx& c, const SetupArgs& sa, SetupScratch* sc, int bs, int m, int degree, int blocks,
                       hipStream_t s, int first, int count, int nl) {
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
  a.nl_max = nl;
  a.warm = sa.warm;
  {
    const double hmax = std::max(c.g.hx, std::max(c.g.hy, c.g.hz));
    const double lref = (M_PI / (c.h.H * hmax)) * (M_PI / (c.h.H * hmax));
    a.lc_thr = sa.opt->lc_threshold > 0.0 ? sa.opt->lc_threshold * lref : 0.0;
  }
  if (first < 0 || count < 0 || first + count > c.h.ncells || nl < 1 || nl > sa.max_cell_nodes) return MSMG_EINVAL;
  a.cells = sc->cells + first;
  a.ncells = count;
  if (count == 0) return MSMG_OK;
  a.Rc64 = sa.Rc64;
  a.evals = sa.evals;
  a.status = sa.cell_status;
  a.work = sc->work;
  if (m < c.h.Lc + 1) return MSMG_EINVAL;
  if (local_lds_bytes(m, a.nl_max) > 160 * 1024) return MSMG_EINVAL;
  if (hipMemsetAsync(sc->work, 0, sizeof(unsigned), s) != hipSuccess) return MSMG_EHIP;
  // compile-time capacities: 8^3-node cells (H = 8) and 9^3 (the last cells
  // of a mesh of 8 k elements per axis)
#define LL(M_, BS_, NLC_)                                              \
  if (!c.tpfa && m == M_ && bs == BS_ && (NLC_ == 0 || a.nl_max == NLC_)) { \
    launch_local_t<M_, BS_, NLC_, false>(a, blocks, s);                \
    return hipGetLastError() == hipSuccess ? MSMG_OK : MSMG_EHIP;      \
  }
#define LT(M_, BS_, NLC_)                                              \
  if (c.tpfa && m == M_ && bs == BS_ && (NLC_ == 0 || a.nl_max == NLC_)) { \
    launch_local_t<M_, BS_, NLC_, true>(a, blocks, s);                 \
    return hipGetLastError() == hipSuccess ? MSMG_OK : MSMG_EHIP;      \
  }
  LT(8, 256, 512)
  LT(8, 512, 512)
  LT(8, 256, 0)
  LT(8, 512, 0)
  LT(8, 768, 0)
  LT(8, 1024, 0)
  LL(8, 256, 512)
  LL(8, 512, 512)
  LL(8, 512, 729)
  LL(8, 768, 729)
  LL(8, 1024, 729)
  LL(8, 256, 0)
  LL(8, 512, 0)
  LL(8, 768, 0)
  LL(8, 1024, 0)
#undef LL
#undef LT
  return MSMG_EINVAL;
}

}  // namespace msmg
