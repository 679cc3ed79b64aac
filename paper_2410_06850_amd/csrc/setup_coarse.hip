// Coarse set-up kernels (paper section 3):
//   * Galerkin blocks A_c = R_c A R_c^T (and the coarse-coarse stiffness
//     R_c K^cc R_c^T that keeps only elements inside one coarse-coarse cell),
//     computed by colouring the coarse cells modulo 3 so that one pass per
//     colour class yields one neighbour block of every cell;
//   * diagonal-block inverses of A_c for block Gauss-Seidel;
//   * a batched Chebyshev-filtered subspace iteration for the standard
//     coarse-coarse eigenproblems of eq. (spectral cc), vectors in HBM;
//   * A_cc = R_cc A_c R_cc^T and its in-place Gauss-Jordan inverse (SPD, no
//     pivoting) used as the direct coarse-coarse solve.
#include "eig_common.h"
#include "setup.h"

#include <algorithm>
#include <vector>

namespace msmg {


// ---------------------------------------------------------------------------
// Galerkin blocks.  For colour class q = (qx,qy,qz) in {0,1,2}^3 every cell j
// has exactly one neighbour cell i (offset in {-1,0,1}^3) with i = q mod 3; the
// pass computes  out[j][block(j->i)][a][b] = sum_{n in j} R[n][a] (A phi_i^b)(n)
// where phi_i^b is basis vector b of cell i.  With drop_cc, elements whose
// nodes belong to two coarse-coarse cells are left out of A.
template <typename BT, int LT>
__global__ void k_galerkin(Geo g, Stencil st, Hier h, int CX, const void* rho, int rho_dt, Material mat,
                           const BT* __restrict__ R, int qx, int qy, int qz, int drop_cc, double* __restrict__ out) {
  extern __shared__ double smem[];
  const long long tile = xcd_tile(blockIdx.x, gridDim.x);
  const Tile t = tile_of_thread(g, h, CX, tile);
  const int H = h.H;
  double acc[LT][LT];
#pragma unroll
  for (int a = 0; a < LT; ++a)
#pragma unroll
    for (int b = 0; b < LT; ++b) acc[a][b] = 0.0;
  const double dk = mat.kmax - mat.kmin;
  int bidx = 13;
  if (t.active) {
    auto off3 = [](int c, int q) {
      const int d = ((q - c) % 3 + 3) % 3;
      return d == 0 ? 0 : (d == 1 ? 1 : -1);
    };
    const int ox = off3(t.cx, qx), oy = off3(t.cy, qy), oz = off3(t.cz, qz);
    bidx = (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1);
    const int icx = t.cx + ox, icy = t.cy + oy, icz = t.cz + oz;
    const bool exists = icx >= 0 && icx < h.ncx && icy >= 0 && icy < h.ncy && icz >= 0 && icz < h.ncz;
    if (exists) {
      // towards a neighbour cell only the cell's boundary layer on that side
      // has stencil partners there
      int xs = t.xs, xe = t.xe, ys = t.ys, ye = t.ye, zs = t.zs, ze = t.ze;
      if (ox > 0) xs = max(xs, cell_end(t.cx, H, h.ncx, g.nnx) - 1);
      if (ox < 0) xe = min(xe, cell_begin(t.cx, H) + 1);
      if (oy > 0) ys = max(ys, cell_end(t.cy, H, h.ncy, g.nny) - 1);
      if (oy < 0) ye = min(ye, cell_begin(t.cy, H) + 1);
      if (oz > 0) zs = max(zs, cell_end(t.cz, H, h.ncz, g.nnz) - 1);
      if (oz < 0) ze = min(ze, cell_begin(t.cz, H) + 1);
      // node ranges of the neighbour cell (its nodes are the stencil partners
      // counted), and the cc-cell boundaries an element of this cell's
      // neighbourhood can straddle: the first node of this cell and of the
      // next one along each axis, where that node starts a new cc cell
      const int nbx0 = cell_begin(icx, H), nbx1 = cell_end(icx, H, h.ncx, g.nnx);
      const int nby0 = cell_begin(icy, H), nby1 = cell_end(icy, H, h.ncy, g.nny);
      const int nbz0 = cell_begin(icz, H), nbz1 = cell_end(icz, H, h.ncz, g.nnz);
      auto starts_cc = [&](int c, int nc, int ng) {
        return c >= 1 && c <= nc - 1 && c % h.sd == 0 && c / h.sd <= ng - 1;
      };
      const int sbx0 = starts_cc(t.cx, h.ncx, h.nccx) ? cell_begin(t.cx, H) : -1;
      const int sbx1 = starts_cc(t.cx + 1, h.ncx, h.nccx) ? cell_begin(t.cx + 1, H) : -1;
      const int sby0 = starts_cc(t.cy, h.ncy, h.nccy) ? cell_begin(t.cy, H) : -1;
      const int sby1 = starts_cc(t.cy + 1, h.ncy, h.nccy) ? cell_begin(t.cy + 1, H) : -1;
      const int sbz0 = starts_cc(t.cz, h.ncz, h.nccz) ? cell_begin(t.cz, H) : -1;
      const int sbz1 = starts_cc(t.cz + 1, h.ncz, h.nccz) ? cell_begin(t.cz + 1, H) : -1;
      for (int k = zs; k < ze; ++k)
        for (int j = ys; j < ye; ++j)
          for (int i = xs; i < xe; ++i) {
            const long long n = node_id(g, i, j, k);
            double kk[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
              const int ei = i - 1 + (c & 1), ej = j - 1 + ((c >> 1) & 1), ek = k - 1 + ((c >> 2) & 1);
              bool in = ei >= 0 && ei < g.nx && ej >= 0 && ej < g.ny && ek >= 0 && ek < g.nz;
              if (in && drop_cc) {
                // the element's upper node starts a new cc cell on some axis
                const bool sx = (ei + 1 == sbx0) || (ei + 1 == sbx1);
                const bool sy = (ej + 1 == sby0) || (ej + 1 == sby1);
                const bool sz = (ek + 1 == sbz0) || (ek + 1 == sbz1);
                in = !(sx || sy || sz);
              }
              if (in) {
                const long long e = elem_id(g, ei, ej, ek);
                const double r = rho_dt == DT_F64 ? ((const double*)rho)[e] : double(((const float*)rho)[e]);
                kk[c] = conductivity<double>(r, mat.kmin, dk, mat.p);
              } else {
                kk[c] = 0.0;
              }
            }
            double w[27];
            stencil27(st, kk, w);
            double wb[LT];
#pragma unroll
            for (int b = 0; b < LT; ++b) wb[b] = 0.0;
#pragma unroll
            for (int o = 0; o < 27; ++o) {
              const int mx = i + o % 3 - 1, my = j + (o / 3) % 3 - 1, mz = k + o / 9 - 1;
              if (mx < 0 || mx >= g.nnx || my < 0 || my >= g.nny || mz < 0 || mz >= g.nnz) continue;
              if (mx < nbx0 || mx >= nbx1 || my < nby0 || my >= nby1 || mz < nbz0 || mz >= nbz1) continue;
              const long long m = node_id(g, mx, my, mz);
#pragma unroll
              for (int b = 0; b < LT; ++b) wb[b] += w[o] * ld<double, BT>(R, m * LT + b);
            }
#pragma unroll
            for (int a = 0; a < LT; ++a) {
              const double ra = ld<double, BT>(R, n * LT + a);
#pragma unroll
              for (int b = 0; b < LT; ++b) acc[a][b] += ra * wb[b];
            }
          }
    }
  }
  // per-cell sums in a fixed order, four (a, b) entries at a time: the H
  // x-threads of each cell and row first, then the rows
  const int nthr = blockDim.x * blockDim.y;
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;
  const int bx = blockDim.x, by = blockDim.y;
  double* part = smem + nthr * 4;  // [by][CX][4]
  const int ntx = (h.ncx + CX - 1) / CX;
  const int tx = int(tile % ntx), ty = int((tile / ntx) % h.ncy), tz = int(tile / ((long long)ntx * h.ncy));
  for (int g0 = 0; g0 < LT * LT; g0 += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      double v = 0.0;
#pragma unroll
      for (int aa = 0; aa < LT; ++aa)
#pragma unroll
        for (int bb = 0; bb < LT; ++bb)
          if (aa * LT + bb == g0 + u) v = acc[aa][bb];
      smem[tid * 4 + u] = v;
    }
    __syncthreads();
    for (int w = tid; w < by * CX * 4; w += nthr) {
      const int u = w % 4, c = (w / 4) % CX, ly = w / (4 * CX);
      double s = 0.0;
      for (int x = 0; x < H; ++x) s += smem[(ly * bx + c * H + x) * 4 + u];
      part[(ly * CX + c) * 4 + u] = s;
    }
    __syncthreads();
    if (tid < CX * 4) {
      const int u = tid % 4, c = tid / 4;
      const int cx = tx * CX + c;
      if (cx < h.ncx && tz < h.ncz && g0 + u < LT * LT) {
        double s = 0.0;
        for (int ly = 0; ly < by; ++ly) s += part[(ly * CX + c) * 4 + u];
        const long long cell = ((long long)tz * h.ncy + ty) * h.ncx + cx;
        // the cell's colour offset, from its own coordinates
        const int ox = (((qx - cx) % 3 + 3) % 3), oy = (((qy - ty) % 3 + 3) % 3), oz = (((qz - tz) % 3 + 3) % 3);
        const int bxo = ox == 0 ? 1 : (ox == 1 ? 2 : 0), byo = oy == 0 ? 1 : (oy == 1 ? 2 : 0), bzo = oz == 0 ? 1 : (oz == 1 ? 2 : 0);
        const int bi = bzo * 9 + byo * 3 + bxo;
        out[(cell * 27 + bi) * LT * LT + g0 + u] = s;
      }
    }
    __syncthreads();
  }
  (void)bidx;
}

// Diagonal-block inverses of A_c.  Padded basis slots (zero rows) get a unit
// diagonal first so every block is invertible; they stay decoupled.
__global__ void k_block_inverse(int ncells, int L, double* __restrict__ Ac, double* __restrict__ Dinv) {
  const long long cell = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (cell >= ncells) return;
  double a[LC_MAX][2 * LC_MAX];
  double* blk = Ac + (cell * 27 + 13) * L * L;
  for (int r = 0; r < L; ++r) {
    bool zero = true;
    for (int c = 0; c < L; ++c) zero = zero && (blk[r * L + c] == 0.0);
    if (zero) blk[r * L + r] = 1.0;
  }
  for (int r = 0; r < L; ++r)
    for (int c = 0; c < 2 * L; ++c) a[r][c] = (c < L) ? blk[r * L + c] : (c - L == r ? 1.0 : 0.0);
  // Gauss-Jordan without pivoting (the block is SPD)
  for (int k = 0; k < L; ++k) {
    const double piv = 1.0 / a[k][k];
    for (int c = 0; c < 2 * L; ++c) a[k][c] *= piv;
    for (int r = 0; r < L; ++r) {
      if (r == k) continue;
      const double f = a[r][k];
      for (int c = 0; c < 2 * L; ++c) a[r][c] -= f * a[k][c];
    }
  }
  for (int r = 0; r < L; ++r)
    for (int c = 0; c < L; ++c) Dinv[(cell * L + r) * L + c] = a[r][L + c];
}

// ---------------------------------------------------------------------------
// Coarse-coarse subspace iteration.  Per cc cell J the operator is the block
// of G = R_c K^cc R_c^T on J's coarse dofs; vectors of J are stored as
// [mcc][nd_J] at offset mcc * cc_ptr[J].  Padded coarse dofs (beyond a cell's
// basis size) are kept at zero, which restricts the problem to real dofs.

struct CCArgs {
  Hier h;
  int J0, nJ;            // the group of cc cells being solved: J0 .. J0 + nJ - 1
  int m;                 // block size
  const double* G;       // [ncells][27][Lc][Lc]
  const int* cc_ptr;
  const int* cc_dofs;
  const int* dof_cc;
  const int* dof_loc;
  const int* cell_status;  // basis size of each cell in bits 20-27
};

MSMG_DEV bool dof_valid(const CCArgs& a, long long d) {
  const int L = a.h.Lc;
  const int cell = int(d / L), l = int(d % L);
  return l < ((a.cell_status[cell] >> 20) & 0xff);
}

// start block: cos products over the cc cell (evaluated at coarse-cell centres)
// on basis slot 0 plus a small deterministic perturbation on all valid slots
__global__ void k_cc_start(CCArgs a, double* __restrict__ Y) {
  const long long d = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const Hier& h = a.h;
  if (d >= (long long)h.ncells * h.Lc) return;
  const int J = a.dof_cc[d], loc = a.dof_loc[d];
  if (J < a.J0 || J >= a.J0 + a.nJ) return;
  const int d0 = a.cc_ptr[J], nd = a.cc_ptr[J + 1] - d0;
  const int cell = int(d / h.Lc), l = int(d % h.Lc);
  const int cx = cell % h.ncx, cy = (cell / h.ncx) % h.ncy, cz = cell / (h.ncx * h.ncy);
  const int jx = J % h.nccx, jy = (J / h.nccx) % h.nccy, jz = J / (h.nccx * h.nccy);
  const int gx0 = group_begin(jx, h.sd), gx1 = group_end(jx, h.sd, h.nccx, h.ncx);
  const int gy0 = group_begin(jy, h.sd), gy1 = group_end(jy, h.sd, h.nccy, h.ncy);
  const int gz0 = group_begin(jz, h.sd), gz1 = group_end(jz, h.sd, h.nccz, h.ncz);
  const double ux = (cx - gx0 + 0.5) / (gx1 - gx0), uy = (cy - gy0 + 0.5) / (gy1 - gy0), uz = (cz - gz0 + 0.5) / (gz1 - gz0);
  const bool ok = dof_valid(a, d);
  for (int j = 0; j < a.m; ++j) {
    // shells of (p, q, r) frequencies
    const int pq[20][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1},
                           {1, 1, 1}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {2, 1, 0}, {1, 2, 0}, {2, 0, 1},
                           {0, 2, 1}, {1, 0, 2}, {0, 1, 2}, {2, 1, 1}, {1, 2, 1}, {1, 1, 2}};
    const int s = j % 20;
    double v = cos(M_PI * pq[s][0] * ux) * cos(M_PI * pq[s][1] * uy) * cos(M_PI * pq[s][2] * uz);
    v = (l == 0 ? v : 0.0);
    unsigned x = unsigned(d) * 2654435761u + unsigned(j) * 40503u + 12345u;
    x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
    v += 0.05 * (double(x) * (1.0 / 4294967296.0) - 0.5);
    Y[(long long)a.m * d0 + (long long)j * nd + loc] = ok ? v : 0.0;
  }
}

// Z = G Y on the active cc cells.  Grid (ceil(cells / 64), ncc, m / 8): a
// thread owns one coarse cell of cc cell J and eight vectors, so each 27 x L x L
// block row of G is read once per eight vectors; the L entries of a
// neighbour cell are contiguous in every vector.  Invalid (padded) dofs get 0.
template <int L>
__global__ __launch_bounds__(64) void k_cc_spmm(CCArgs a, const double* __restrict__ Y, double* __restrict__ Z,
                                                const int* __restrict__ flag) {
  const int J = a.J0 + blockIdx.y;
  if (flag && flag[J] >= 0) return;
  const Hier& h = a.h;
  const int m = a.m;
  const int d0 = a.cc_ptr[J], nd = a.cc_ptr[J + 1] - d0;
  const int lc = blockIdx.x * 64 + threadIdx.x;
  if (lc * L >= nd) return;
  const int j0 = blockIdx.z * 8;
  const int cell = a.cc_dofs[d0 + lc * L] / L;
  const int cx = cell % h.ncx, cy = (cell / h.ncx) % h.ncy, cz = cell / (h.ncx * h.ncy);
  const double* YJ = Y + (long long)m * d0;
  double acc[8][L];
#pragma unroll
  for (int jj = 0; jj < 8; ++jj)
#pragma unroll
    for (int l = 0; l < L; ++l) acc[jj][l] = 0.0;
  const double* Gr = a.G + (long long)cell * 27 * L * L;
  for (int b = 0; b < 27; ++b) {
    const int x = cx + b % 3 - 1, y = cy + (b / 3) % 3 - 1, z = cz + b / 9 - 1;
    if (x < 0 || x >= h.ncx || y < 0 || y >= h.ncy || z < 0 || z >= h.ncz) continue;
    const long long nc = ((long long)z * h.ncy + y) * h.ncx + x;
    if (a.dof_cc[nc * L] != J) continue;
    const int nloc0 = a.dof_loc[nc * L];
    double g[L][L];
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
      for (int q = 0; q < L; ++q) g[l][q] = Gr[(b * L + l) * L + q];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      if (j0 + jj >= m) break;
      const double* yv = YJ + (long long)(j0 + jj) * nd + nloc0;
      double yq[L];
#pragma unroll
      for (int q = 0; q < L; ++q) yq[q] = yv[q];
#pragma unroll
      for (int l = 0; l < L; ++l)
#pragma unroll
        for (int q = 0; q < L; ++q) acc[jj][l] += g[l][q] * yq[q];
    }
  }
  double* ZJ = Z + (long long)m * d0;
#pragma unroll
  for (int jj = 0; jj < 8; ++jj) {
    if (j0 + jj >= m) break;
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const long long d = (long long)cell * L + l;
      ZJ[(long long)(j0 + jj) * nd + lc * L + l] = dof_valid(a, d) ? acc[jj][l] : 0.0;
    }
  }
}

// S_J = P_J^T Q_J (m x m per cc cell, m <= 32), in CC_KS slices of the dofs:
// workgroup (J, ks) sums the 64-dof chunks ks, ks + CC_KS, ... of cell J into
// part[(J - J0) * CC_KS + ks] (upper triangle mirrored); k_cc_gram_sum adds
// the slices in a fixed order into small[J][which].  Chunks of both blocks
// are staged in LDS and each thread accumulates a 2 x 2 patch.
constexpr int CC_KS = CC_GRAM_SLICES;
__global__ __launch_bounds__(256) void k_cc_gram(CCArgs a, const double* __restrict__ P, const double* __restrict__ Q,
                                                 double* __restrict__ part, const int* __restrict__ flag) {
  __shared__ double Ps[32 * 65], Qs[32 * 65];
  const int J = a.J0 + blockIdx.x, ks = blockIdx.y;
  if (flag && flag[J] >= 0) return;
  const int m = a.m;
  const int d0 = a.cc_ptr[J], nd = a.cc_ptr[J + 1] - d0;
  const double* PJ = P + (long long)m * d0;
  const double* QJ = Q + (long long)m * d0;
  const int tid = threadIdx.x;
  const int ti = (tid >> 4) * 2, tj = (tid & 15) * 2;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int k0 = ks * 64; k0 < nd; k0 += 64 * CC_KS) {
    __syncthreads();
    for (int e = tid; e < 32 * 64; e += 256) {
      const int i = e >> 6, kk = e & 63;
      const bool ok = i < m && k0 + kk < nd;
      Ps[i * 65 + kk] = ok ? PJ[(long long)i * nd + k0 + kk] : 0.0;
      Qs[i * 65 + kk] = ok ? QJ[(long long)i * nd + k0 + kk] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 64; ++kk) {
      const double p0 = Ps[ti * 65 + kk], p1 = Ps[(ti + 1) * 65 + kk];
      const double q0 = Qs[tj * 65 + kk], q1 = Qs[(tj + 1) * 65 + kk];
      acc[0][0] += p0 * q0;
      acc[0][1] += p0 * q1;
      acc[1][0] += p1 * q0;
      acc[1][1] += p1 * q1;
    }
  }
  double* S = part + ((long long)(J - a.J0) * CC_KS + ks) * m * m;
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const int i = ti + u, j = tj + v;
      if (i < m && j < m && j >= i) {
        S[i * m + j] = acc[u][v];
        S[j * m + i] = acc[u][v];
      }
    }
}

__global__ __launch_bounds__(256) void k_cc_gram_sum(CCArgs a, const double* __restrict__ part,
                                                     double* __restrict__ small, int which,
                                                     const int* __restrict__ flag) {
  const int J = a.J0 + blockIdx.x;
  if (flag && flag[J] >= 0) return;
  const int m = a.m;
  const double* Pt = part + (long long)(J - a.J0) * CC_KS * m * m;
  double* S = small + ((long long)J * 4 + which) * m * m;
  for (int e = threadIdx.x; e < m * m; e += 256) {
    double v = 0.0;
#pragma unroll
    for (int ks = 0; ks < CC_KS; ++ks) v += Pt[(long long)ks * m * m + e];
    S[e] = v;
  }
}

// Per cc cell: eigen-decomposition of small[J][which] (m x m).
//   kind 0 (orthonormalise): C = U S^-1/2 -> small[J][2]
//   kind 1 (Rayleigh-Ritz):  C = U (ascending) -> small[J][2], Ritz values -> ritz[J][:]
//   only (kind 0): when not null, only the cells whose Cholesky factorisation
//   failed (only[J] != 0)
__global__ void k_cc_small_eig(CCArgs a, double* __restrict__ small, int which, int kind, double* __restrict__ ritz,
                               const int* __restrict__ flag, const int* __restrict__ only) {
  extern __shared__ double sm[];
  const int J = a.J0 + blockIdx.x;
  if (flag && flag[J] >= 0) return;
  if (only && !only[J]) return;
  const int m = a.m;
  double* A = sm;
  double* V = A + m * m;
  double* B = V + m * m;
  double* Vs = B + m * m;
  double* ev = Vs + m * m;
  double* red = ev + m;
  double* cs = red + 64;
  int* perm = reinterpret_cast<int*>(cs + 2 * m);
  const double* S = small + ((long long)J * 4 + which) * m * m;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) A[e] = S[e];
  __syncthreads();
  block_jacobi(A, V, B, Vs, ev, perm, m, red, cs);
  double* C = small + ((long long)J * 4 + 2) * m * m;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
    const int k = e % m;
    if (kind == 0) C[e] = ev[k] > 1e-300 ? Vs[e] / sqrt(ev[k]) : 0.0;
    else C[e] = Vs[e];
  }
  if (kind == 1)
    for (int k = threadIdx.x; k < m; k += blockDim.x) ritz[(long long)J * m + k] = ev[k];
}

// Orthonormalising transform of a cc cell's block from its Gram matrix
// S = small[J][which] (m x m, m <= 32) by one wave: the Cholesky factor
// S = L L^T and C = L^-T (upper triangular) -> small[J][2], so that P C has
// orthonormal columns (the block orthonormalised in column order, as
// Gram-Schmidt would).  A pivot below 1e-14 of its diagonal entry (a block
// of condition above ~1e7) or not positive sets failed[J] = 1 and leaves C
// unwritten; the eigen-decomposition then takes that cell.
__global__ __launch_bounds__(64) void k_cc_cholinv(CCArgs a, double* __restrict__ small, int which,
                                                   const int* __restrict__ flag, int* __restrict__ failed) {
  __shared__ double Ls[32 * 33];
  __shared__ double Xs[32 * 33];
  const int J = a.J0 + blockIdx.x;
  if (flag && flag[J] >= 0) return;
  const int m = a.m;
  const int lane = threadIdx.x;
  const double* S = small + ((long long)J * 4 + which) * m * m;
  for (int e = lane; e < m * m; e += 64) Ls[(e / m) * 33 + e % m] = S[e];
  __syncthreads();
  bool ok = true;
  for (int k = 0; k < m && ok; ++k) {
    const double d = Ls[k * 33 + k];
    const double s0 = S[k * m + k];
    ok = (d > 1e-14 * s0) && (d > 1e-300);
    if (!ok) break;
    const double rd = 1.0 / sqrt(d);
    __syncthreads();
    // column k of L (rows k .. m-1)
    for (int i = k + lane; i < m; i += 64) Ls[i * 33 + k] *= rd;
    __syncthreads();
    // trailing lower triangle: S_ij -= L_ik L_jk for k < j <= i
    const int t = m - k - 1;
    for (int e = lane; e < t * t; e += 64) {
      const int i = k + 1 + e / t, j = k + 1 + e % t;
      if (j <= i) Ls[i * 33 + j] -= Ls[i * 33 + k] * Ls[j * 33 + k];
    }
    __syncthreads();
  }
  if (!ok) {
    if (lane == 0) failed[J] = 1;
    return;
  }
  // X = L^-1 by forward substitution, column j in lane j
  if (lane < m) {
    const int j = lane;
    for (int i = 0; i < m; ++i) {
      double acc = (i == j) ? 1.0 : 0.0;
      for (int k = j; k < i; ++k) acc -= Ls[i * 33 + k] * Xs[k * 33 + j];
      Xs[i * 33 + j] = (i >= j) ? acc / Ls[i * 33 + i] : 0.0;
    }
  }
  __syncthreads();
  // C = X^T
  double* C = small + ((long long)J * 4 + 2) * m * m;
  for (int e = lane; e < m * m; e += 64) {
    const int i = e / m, j = e % m;
    C[e] = Xs[j * 33 + i];
  }
  if (lane == 0) failed[J] = 0;
}

// Q = P C per cc cell (C = small[J][2], m <= 32).  Grid (ceil(nd / 256), ncc):
// a thread owns one dof of cc cell J and all m vectors, C sits in LDS.
__global__ __launch_bounds__(256) void k_cc_transform(CCArgs a, const double* __restrict__ P, double* __restrict__ Q,
                                                      const double* __restrict__ small, const int* __restrict__ flag) {
  __shared__ double Cs[32 * 32];
  const int J = a.J0 + blockIdx.y;
  if (flag && flag[J] >= 0) return;
  const int m = a.m;
  const int d0 = a.cc_ptr[J], nd = a.cc_ptr[J + 1] - d0;
  const double* C = small + ((long long)J * 4 + 2) * m * m;
  for (int e = threadIdx.x; e < 32 * 32; e += 256) {
    const int i = e >> 5, j = e & 31;
    Cs[e] = (i < m && j < m) ? C[i * m + j] : 0.0;
  }
  __syncthreads();
  const int loc = blockIdx.x * 256 + threadIdx.x;
  if (loc >= nd) return;
  const double* PJ = P + (long long)m * d0;
  double t[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) t[i] = i < m ? PJ[(long long)i * nd + loc] : 0.0;
  double* QJ = Q + (long long)m * d0;
#pragma unroll 4
  for (int j = 0; j < 32; ++j) {
    if (j >= m) break;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 32; ++i) s += t[i] * Cs[i * 32 + j];
    QJ[(long long)j * nd + loc] = s;
  }
}

// Residual check per cc cell (one block per J).  X Ritz block, Z = G X, ritz
// values.  Converged when every wanted residual ||Z_j - theta_j X_j|| <=
// tol * bound.  Sets flag[J] = iteration when done, -2 - iteration when the
// last iteration ends unconverged.
__global__ void k_cc_check(CCArgs a, const double* __restrict__ X, const double* __restrict__ Z,
                           const double* __restrict__ ritz, int* __restrict__ flag, const double* __restrict__ bound,
                           int Lwant, double tol, int iter, int last) {
  __shared__ double red[64];
  __shared__ double worst_s;
  const int J = a.J0 + blockIdx.x;
  if (flag[J] >= 0) return;
  const int m = a.m;
  const int d0 = a.cc_ptr[J], nd = a.cc_ptr[J + 1] - d0;
  const int lw = min(Lwant, nd);
  const double* XJ = X + (long long)m * d0;
  const double* ZJ = Z + (long long)m * d0;
  const double* th = ritz + (long long)J * m;
  if (threadIdx.x == 0) worst_s = 0.0;
  __syncthreads();
  for (int j = 0; j < lw; ++j) {
    double s = 0.0;
    for (int d = threadIdx.x; d < nd; d += blockDim.x) {
      const double r = ZJ[(long long)j * nd + d] - th[j] * XJ[(long long)j * nd + d];
      s += r * r;
    }
    s = block_allsum(s, red);
    if (threadIdx.x == 0) worst_s = fmax(worst_s, s);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double b = bound[J];
  if (worst_s <= (tol * b) * (tol * b)) flag[J] = iter;
  else if (last) flag[J] = -2 - iter;  // not converged (kept as is)
}

// Gershgorin bound of each cc operator (max over rows of sum |G_ij|)
__global__ void k_cc_bound(CCArgs a, double* __restrict__ bound) {
  __shared__ double red[64];
  const int J = a.J0 + blockIdx.x;
  const Hier& h = a.h;
  const int L = h.Lc;
  const int d0 = a.cc_ptr[J], nd = a.cc_ptr[J + 1] - d0;
  double mx = 0.0;
  for (int q = threadIdx.x; q < nd; q += blockDim.x) {
    const long long d = a.cc_dofs[d0 + q];
    if (!dof_valid(a, d)) continue;
    const int cell = int(d / L), l = int(d % L);
    const int cx = cell % h.ncx, cy = (cell / h.ncx) % h.ncy, cz = cell / (h.ncx * h.ncy);
    double s = 0.0;
    for (int b = 0; b < 27; ++b) {
      const int x = cx + b % 3 - 1, y = cy + (b / 3) % 3 - 1, z = cz + b / 9 - 1;
      if (x < 0 || x >= h.ncx || y < 0 || y >= h.ncy || z < 0 || z >= h.ncz) continue;
      for (int m = 0; m < L; ++m) s += fabs(a.G[(((long long)cell * 27 + b) * L + l) * L + m]);
    }
    mx = fmax(mx, s);
  }
  mx = block_allmax(mx, red);
  if (threadIdx.x == 0) bound[J] = mx * 1.0001 + 1e-300;
}

// Final R_cc rows: sign-normalised Ritz vectors 0..Lcc-1 of each cc cell.
// Rcc layout: [J][b][nd_J] at offset Lcc * cc_ptr[J].  Sign: sum of entries > 0,
// else the first entry of largest magnitude positive.
__global__ void k_cc_finish(CCArgs a, const double* __restrict__ X, const double* __restrict__ ritz, double* __restrict__ Rcc,
                            double* __restrict__ cc_evals, int Lcc) {
  __shared__ double red[64];
  __shared__ int ired[16];
  const int J = a.J0 + blockIdx.x;
  const int m = a.m;
  const int d0 = a.cc_ptr[J], nd = a.cc_ptr[J + 1] - d0;
  const double* XJ = X + (long long)m * d0;
  for (int b = 0; b < Lcc; ++b) {
    const bool have = b < nd && b < m;
    double s = 0.0, ss = 0.0;
    if (have)
      for (int d = threadIdx.x; d < nd; d += blockDim.x) s += XJ[(long long)b * nd + d];
    s = block_allsum(s, red);
    (void)ss;
    double sgn = s > 0.0 ? 1.0 : -1.0;
    if (have && !(fabs(s) > 1e-8 * sqrt(double(nd)))) {
      double amax = 0.0;
      for (int d = threadIdx.x; d < nd; d += blockDim.x) amax = fmax(amax, fabs(XJ[(long long)b * nd + d]));
      amax = block_allmax(amax, red);
      int first = 1 << 30;
      for (int d = threadIdx.x; d < nd; d += blockDim.x)
        if (fabs(XJ[(long long)b * nd + d]) >= (1.0 - 1e-8) * amax) first = min(first, d);
      first = block_allmin_int(first, ired);
      sgn = XJ[(long long)b * nd + first] > 0.0 ? 1.0 : -1.0;
    }
    for (int d = threadIdx.x; d < nd; d += blockDim.x)
      Rcc[(long long)Lcc * d0 + (long long)b * nd + d] = have ? sgn * XJ[(long long)b * nd + d] : 0.0;
    if (threadIdx.x == 0) cc_evals[(long long)J * Lcc + b] = have ? ritz[(long long)J * m + b] : 0.0;
    __syncthreads();
  }
}

// Small coarse-coarse cells (nd <= 32): assemble G_J densely and diagonalise it.
// Padded dofs get a huge decoupled diagonal so they sort last.  Writes the
// Ritz block X (first min(m, nd) rows) and values, and marks the cell done.
constexpr int CC_DENSE = 32;
__global__ void k_cc_dense(CCArgs a, double* __restrict__ X, double* __restrict__ ritz, int* __restrict__ flag) {
  extern __shared__ double sm[];
  const int J = a.J0 + blockIdx.x;
  const Hier& h = a.h;
  const int L = h.Lc;
  const int d0 = a.cc_ptr[J], nd = a.cc_ptr[J + 1] - d0;
  if (nd > CC_DENSE) return;
  double* A = sm;
  double* V = A + nd * nd;
  double* B = V + nd * nd;
  double* Vs = B + nd * nd;
  double* ev = Vs + nd * nd;
  double* red = ev + nd;
  double* cs = red + 64;
  int* perm = reinterpret_cast<int*>(cs + 2 * nd);
  for (int e = threadIdx.x; e < nd * nd; e += blockDim.x) {
    const int p = e / nd, q = e % nd;
    const long long dp = a.cc_dofs[d0 + p], dq = a.cc_dofs[d0 + q];
    double v = 0.0;
    if (!dof_valid(a, dp) || !dof_valid(a, dq)) {
      v = (p == q) ? 1e300 : 0.0;
    } else {
      const int cp = int(dp / L), lp = int(dp % L), cq = int(dq / L), lq = int(dq % L);
      const int px = cp % h.ncx, py = (cp / h.ncx) % h.ncy, pz = cp / (h.ncx * h.ncy);
      const int qx = cq % h.ncx, qy = (cq / h.ncx) % h.ncy, qz = cq / (h.ncx * h.ncy);
      const int ox = qx - px, oy = qy - py, oz = qz - pz;
      if (abs(ox) <= 1 && abs(oy) <= 1 && abs(oz) <= 1) {
        const int b = (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1);
        v = a.G[(((long long)cp * 27 + b) * L + lp) * L + lq];
      }
    }
    A[e] = v;
  }
  __syncthreads();
  // symmetrise
  for (int e = threadIdx.x; e < nd * nd; e += blockDim.x) {
    const int p = e / nd, q = e % nd;
    if (p < q) {
      const double v = 0.5 * (A[p * nd + q] + A[q * nd + p]);
      B[e] = v;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nd * nd; e += blockDim.x) {
    const int p = e / nd, q = e % nd;
    if (p < q) A[e] = B[e];
    else if (p > q) A[e] = B[q * nd + p];
  }
  __syncthreads();
  block_jacobi(A, V, B, Vs, ev, perm, nd, red, cs);
  const int m = a.m;
  for (int e = threadIdx.x; e < m * nd; e += blockDim.x) {
    const int k = e / nd, d = e % nd;
    X[(long long)m * d0 + (long long)k * nd + d] = (k < nd) ? Vs[d * nd + k] : 0.0;
  }
  for (int k = threadIdx.x; k < m; k += blockDim.x) ritz[(long long)J * m + k] = (k < nd) ? ev[k] : 0.0;
  if (threadIdx.x == 0) flag[J] = 0;
}

// ---------------------------------------------------------------------------
// A_cc = R_cc A_c R_cc^T by colouring cc cells modulo 3: for class Q and
// vector b, u = A_c v with v = sum over cc cells J of class Q of R_cc[J][b],
// then A_cc[(I, a), (J(Q, I), b)] = R_cc[I][a] . u.

// One launch pair per class Q takes the columns b0 .. b0 + 31 at once: u
// holds column b at u + (b - b0) * ustride, each thread one coarse dof.
constexpr int ACC_B = 32;
template <typename AT, typename VT, int L>
__global__ __launch_bounds__(256) void k_acc_apply_cols(Hier h, const AT* __restrict__ Ac, const VT* __restrict__ Rcc,
                                                        const int* __restrict__ cc_ptr, const int* __restrict__ dof_cc,
                                                        const int* __restrict__ dof_loc, int qx, int qy, int qz, int b0,
                                                        double* __restrict__ u, long long ustride) {
  const long long d = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (d >= (long long)h.ncells * L) return;
  const int nb = min(ACC_B, h.Lcc - b0);
  const int cell = int(d / L), l = int(d % L);
  const int cx = cell % h.ncx, cy = (cell / h.ncx) % h.ncy, cz = cell / (h.ncx * h.ncy);
  const AT* A = Ac + (long long)cell * 27 * L * L;
  double s[ACC_B];
#pragma unroll
  for (int b = 0; b < ACC_B; ++b) s[b] = 0.0;
  for (int bb = 0; bb < 27; ++bb) {
    const int x = cx + bb % 3 - 1, y = cy + (bb / 3) % 3 - 1, z = cz + bb / 9 - 1;
    if (x < 0 || x >= h.ncx || y < 0 || y >= h.ncy || z < 0 || z >= h.ncz) continue;
    const long long nc = ((long long)z * h.ncy + y) * h.ncx + x;
    const int J = dof_cc[nc * L];
    const int jx = J % h.nccx, jy = (J / h.nccx) % h.nccy, jz = J / (h.nccx * h.nccy);
    if (jx % 3 != qx || jy % 3 != qy || jz % 3 != qz) continue;
    const int d0 = cc_ptr[J], nd = cc_ptr[J + 1] - d0;
    const int bend = min(min(h.Lcc, nd) - b0, nb);
    const int loc0 = dof_loc[nc * L];
    double a[L];
#pragma unroll
    for (int m = 0; m < L; ++m) a[m] = double(ld<double, AT>(A, (bb * L + l) * L + m));
    const VT* R = Rcc + (long long)h.Lcc * d0 + (long long)b0 * nd + loc0;
#pragma unroll
    for (int b = 0; b < ACC_B; ++b) {
      if (b < bend) {
#pragma unroll
        for (int m = 0; m < L; ++m) s[b] += a[m] * double(R[(long long)b * nd + m]);
      }
    }
  }
#pragma unroll
  for (int b = 0; b < ACC_B; ++b)
    if (b < nb) u[(long long)b * ustride + d] = s[b];
}

template <typename VT>
__global__ void k_acc_dot_cols(Hier h, const VT* __restrict__ Rcc, const int* __restrict__ cc_ptr,
                               const int* __restrict__ cc_dofs, const double* __restrict__ u, long long ustride, int qx,
                               int qy, int qz, int b0, int n_cc, double* __restrict__ Acc) {
  const long long w = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int nb = min(ACC_B, h.Lcc - b0);
  if (w >= (long long)h.ncc * h.Lcc * nb) return;
  const int bl = int(w % nb), a = int((w / nb) % h.Lcc), I = int(w / ((long long)nb * h.Lcc));
  const int b = b0 + bl;
  const int ix = I % h.nccx, iy = (I / h.nccx) % h.nccy, iz = I / (h.nccx * h.nccy);
  auto off3 = [](int c, int q) {
    const int dd = ((q - c) % 3 + 3) % 3;
    return dd == 0 ? 0 : (dd == 1 ? 1 : -1);
  };
  const int jx = ix + off3(ix, qx), jy = iy + off3(iy, qy), jz = iz + off3(iz, qz);
  if (jx < 0 || jx >= h.nccx || jy < 0 || jy >= h.nccy || jz < 0 || jz >= h.nccz) return;
  const int J = (jz * h.nccy + jy) * h.nccx + jx;
  const int d0 = cc_ptr[I], nd = cc_ptr[I + 1] - d0;
  const int ndJ = cc_ptr[J + 1] - cc_ptr[J];
  if (a >= min(h.Lcc, nd) || b >= min(h.Lcc, ndJ)) return;
  const VT* R = Rcc + (long long)h.Lcc * d0 + (long long)a * nd;
  const double* ub = u + (long long)bl * ustride;
  double s = 0.0;
  for (int d = lane; d < nd; d += 64) s += double(R[d]) * ub[cc_dofs[d0 + d]];
  s = wave_sum(s);
  if (lane == 0) Acc[(long long)(I * h.Lcc + a) * n_cc + (J * h.Lcc + b)] = s;
}

// unused cc slots (cells with fewer than Lcc dofs) get a unit diagonal
__global__ void k_acc_pad(Hier h, const int* __restrict__ cc_ptr, int n_cc, double* __restrict__ Acc) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= n_cc) return;
  const int I = w / h.Lcc, a = w % h.Lcc;
  const int nd = cc_ptr[I + 1] - cc_ptr[I];
  if (a >= nd) Acc[(long long)w * n_cc + w] = 1.0;
}

// ---------------------------------------------------------------------------
// In-place Gauss-Jordan inverse of a batch of SPD matrices (n x n each, stride
// n*n, batch index blockIdx.z) by pivot blocks of NB:
//   P = A_kk^-1;  A_kJ <- P A_kJ;  A_IJ -= A_Ik A_kJ;  A_Ik <- -A_Ik P;  A_kk <- P.
// No pivoting is needed for SPD matrices.
// Symmetric in-place inversion of SPD matrices by block sweeps (the sweep
// operator of Goodnight, 1979): sweeping pivot block K with P = A_KK^-1 gives
//   A_KK <- -P,  A_KJ <- P A_KJ,  A_IK <- A_IK P,  A_IJ <- A_IJ - A_IK P A_KJ,
// which keeps the matrix symmetric; after all blocks it holds -A^-1.  Only the
// lower triangle (i >= j) is read and kept up to date, halving the trailing
// updates; a last pass negates and mirrors it into the full inverse.
//
// Pivot block: invert the current A_KK (SPD, read from the lower triangle) by
// unblocked Gauss-Jordan, keep P, store -P; 1024 threads, each holding the
// entries of a full block in registers (a partial last block in LDS); the
// pivot row and column of each step pass through LDS (dynamic LDS,
// GJ_PIVOT_LDS).
constexpr int GJ_PLD = GJ_NB + 1;
constexpr size_t GJ_PIVOT_LDS = sizeof(double) * (2 * GJ_NB + GJ_NB * GJ_PLD);
__global__ __launch_bounds__(1024) void k_gj_pivot(int n, double* __restrict__ Ab, int k0, int nb,
                                                   double* __restrict__ Pb) {
  extern __shared__ double gjp_lds[];
  constexpr int NQ = (GJ_NB * GJ_NB + 1023) / 1024;
  double* A = Ab + (long long)blockIdx.z * n * n;
  double* P = Pb + (long long)blockIdx.z * GJ_NB * GJ_NB;
  const int tid = threadIdx.x;
  const int ne = nb * nb;
  double* rowk = gjp_lds;
  double* colk = rowk + GJ_NB;
  if (nb == GJ_NB) {
    // full block: the thread holds column c = tid % nb of rows r0 + 8 q in
    // registers; each step the owners publish the pivot row and column
    static_assert(GJ_NB * 8 == 1024, "a full pivot block is 8 rows per pass of 1024 threads");
    const int c = tid & (GJ_NB - 1), r0 = tid >> 7;
    double v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int r = r0 + 8 * q;
      v[q] = A[(long long)(k0 + max(r, c)) * n + (k0 + min(r, c))];
    }
    for (int k = 0; k < nb; ++k) {
      if (r0 == (k & 7)) {
        double w = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) w = (q == (k >> 3)) ? v[q] : w;
        rowk[c] = w;
      }
      if (c == k) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) colk[r0 + 8 * q] = v[q];
      }
      __syncthreads();
      const double piv = 1.0 / rowk[k];
      const double rc = rowk[c];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int r = r0 + 8 * q;
        if (r == k && c == k) v[q] = piv;
        else if (r == k) v[q] = rc * piv;
        else if (c == k) v[q] = -colk[r] * piv;
        else v[q] = v[q] - colk[r] * rc * piv;
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int r = r0 + 8 * q;
      P[r * nb + c] = v[q];
      A[(long long)(k0 + r) * n + (k0 + c)] = -v[q];
    }
    return;
  }
  // the last, partial block: the entries tid + 1024 q in LDS
  double* blk = colk + GJ_NB;
  auto a = [&](int r, int c) -> double& { return blk[r * GJ_PLD + c]; };
  int rq[NQ], cq[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int e = tid + 1024 * q;
    rq[q] = e < ne ? e / nb : -1;
    cq[q] = e < ne ? e % nb : 0;
    if (rq[q] >= 0) a(rq[q], cq[q]) = A[(long long)(k0 + max(rq[q], cq[q])) * n + (k0 + min(rq[q], cq[q]))];
  }
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    if (tid < nb) {
      rowk[tid] = a(k, tid);
      colk[tid] = a(tid, k);
    }
    __syncthreads();
    const double piv = 1.0 / rowk[k];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int r = rq[q], c = cq[q];
      if (r < 0) continue;
      if (r == k && c == k) a(r, c) = piv;
      else if (r == k) a(r, c) = rowk[c] * piv;
      else if (c == k) a(r, c) = -colk[r] * piv;
      else a(r, c) = a(r, c) - colk[r] * rowk[c] * piv;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int r = rq[q], c = cq[q];
    if (r < 0) continue;
    P[r * nb + c] = a(r, c);
    A[(long long)(k0 + r) * n + (k0 + c)] = -a(r, c);
  }
}

// The two products of a sweep step on 64 x 64 output tiles, computed by FP64
// matrix cores (inner dimension: the nb <= GJ_NB pivot columns, staged in
// 64-deep halves), reading A through its lower triangle (A_xy = A[max][min]):
//   GJ_ROW:    Rb[r][j]  =  sum_t P[r][t] A[k0+t][j]     (j outside the pivot block)
//   GJ_UPDATE: A[i][j]  -=  sum_t A[i][k0+t] Rb[t][j]    (i >= j tiles, both outside it)
// Each wave owns a 32 x 32 quarter of the tile as 2 x 2 blocks of
// v_mfma_f64_16x16x4 (A operand: lane holds row lane % 16, k lane / 16; B
// operand: column lane % 16, k lane / 16; result register v: column
// lane % 16, row lane / 16 + 4 v, as measured on gfx950).  Both operands are
// staged in LDS with row strides chosen so that the operand reads of 32 lanes
// hit distinct banks; every thread issues all its global loads of a half (and,
// for the update, its part of the output tile) before the first LDS store, so
// the loads of a tile are in flight together.  Operand entries beyond nb are
// zero.  A pass over the lower triangle per step is what bounds the update, so
// the wider pivot block halves the passes for the same arithmetic.
typedef double gj_v4d __attribute__((ext_vector_type(4)));
constexpr int GJ_LDA = 66, GJ_LDB = 80;
constexpr int GJ_HALVES = GJ_NB / 64;
static_assert(GJ_NB % 64 == 0, "pivot blocks of whole 64-deep halves");
constexpr size_t GJ_TILE_LDS = sizeof(double) * (64 * GJ_LDA + 64 * GJ_LDB);
constexpr long long GJ_WORKGROUPS = 2048;  // persistent tile loops: a few rounds of resident workgroups
enum { GJ_ROW = 0, GJ_UPDATE = 2 };

template <int MODE>
__global__ __launch_bounds__(256) void k_gj_tile(int n, double* __restrict__ Ab, int k0, int nb,
                                                 const double* __restrict__ Pb, double* __restrict__ Rbb, int batch) {
  extern __shared__ double gj_lds[];
  double* As = gj_lds;                 // As[r][t], 64 x GJ_LDA
  double* Bs = gj_lds + 64 * GJ_LDA;   // Bs[t][c], 64 x GJ_LDB
  // tiles per matrix: the row panel's GJ_HALVES x nt tiles (tile row = 64
  // pivot rows), or the nt (nt + 1) / 2 tiles of the lower triangle;
  // workgroups loop over (matrix, tile) pairs
  const int nt = (n + 63) / 64;
  const long long per = MODE == GJ_ROW ? (long long)GJ_HALVES * nt : (long long)nt * (nt + 1) / 2;
  const long long total = per * batch;
  for (long long wk = blockIdx.x; wk < total; wk += gridDim.x) {
    const long long z = wk / per, tl = wk % per;
    int ti = 0, tj = int(tl);
    if (MODE == GJ_UPDATE) {
      // tl = ti (ti + 1) / 2 + tj with 0 <= tj <= ti
      ti = int((sqrt(8.0 * double(tl) + 1.0) - 1.0) * 0.5);
      while ((long long)(ti + 1) * (ti + 2) / 2 <= tl) ++ti;
      while ((long long)ti * (ti + 1) / 2 > tl) --ti;
      tj = int(tl - (long long)ti * (ti + 1) / 2);
    } else {
      ti = int(tl / nt);  // tile row of the panel: pivot rows 64 ti ..
      tj = int(tl % nt);
    }
    const int i0 = ti * 64, j0 = tj * 64;
    const bool ipiv_tile = i0 >= k0 && i0 + 64 <= k0 + nb, jpiv_tile = j0 >= k0 && j0 + 64 <= k0 + nb;
    if (MODE == GJ_UPDATE && (ipiv_tile || jpiv_tile)) continue;  // pivot rows/columns: write-back
    if (MODE == GJ_ROW && (jpiv_tile || i0 >= nb)) continue;
    double* A = Ab + z * n * n;
    const double* P = Pb + z * GJ_NB * GJ_NB;
    double* Rb = Rbb + z * GJ_NB * n;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w & 1) * 32, wc = (w >> 1) * 32;
    const int l16 = lane & 15, lk = lane >> 4;
    // entry (i, j) of the symmetric matrix from its lower triangle
    auto sym = [&](int i, int j) { return A[(long long)max(i, j) * n + min(i, j)]; };
    auto a_elem = [&](int r, int t) -> double {  // A operand [r][t] (t: pivot column)
      if (t >= nb) return 0.0;
      if (MODE == GJ_ROW) return i0 + r < nb ? P[(i0 + r) * nb + t] : 0.0;
      const int i = i0 + r;
      return i < n ? sym(i, k0 + t) : 0.0;
    };
    auto b_elem = [&](int t, int c) -> double {  // B operand [t][c]
      if (t >= nb) return 0.0;
      const int j = j0 + c;
      if (j >= n) return 0.0;
      return MODE == GJ_ROW ? sym(k0 + t, j) : Rb[(long long)t * n + j];
    };
    auto out_ok = [&](int i, int j) {
      const bool iok = i < n && !(i >= k0 && i < k0 + nb), jok = j < n && !(j >= k0 && j < k0 + nb);
      if (MODE == GJ_UPDATE) return iok && jok;
      return i < nb && jok;
    };
    // panels read through the upper triangle's mirror (rows above or columns
    // right of the pivot block) are contiguous along the other index: let
    // consecutive lanes run along it so the loads stay coalesced
    const bool a_tr = MODE == GJ_UPDATE && i0 < k0;
    const bool b_tr = MODE == GJ_ROW && j0 >= k0 + nb;
    auto a_rt = [&](int e, int& r, int& t) {
      r = a_tr ? (e & 63) : (e >> 6);
      t = a_tr ? (e >> 6) : (e & 63);
    };
    auto b_tc = [&](int e, int& t, int& c) {
      t = b_tr ? (e & 63) : (e >> 6);
      c = b_tr ? (e >> 6) : (e & 63);
    };
    double ra[16], rb[16];
    auto load_half = [&](int t0) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int e = tid + 256 * q;
        int r, t, c;
        a_rt(e, r, t);
        ra[q] = a_elem(r, t0 + t);
        b_tc(e, t, c);
        rb[q] = b_elem(t0 + t, c);
      }
    };
    gj_v4d cv[2][2];
    if (MODE == GJ_UPDATE) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = i0 + wr + bi * 16 + lk + 4 * v, j = j0 + wc + bj * 16 + l16;
            cv[bi][bj][v] = out_ok(i, j) ? A[(long long)i * n + j] : 0.0;
          }
    }
    gj_v4d acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = gj_v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int hf = 0; hf < GJ_HALVES; ++hf) {
      const int t0 = hf * 64;
      if (t0 >= nb) break;  // uniform over the workgroup
      load_half(t0);
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int e = tid + 256 * q;
        int r, t, c;
        a_rt(e, r, t);
        As[r * GJ_LDA + t] = ra[q];
        b_tc(e, t, c);
        Bs[t * GJ_LDB + c] = rb[q];
      }
      __syncthreads();
      const int ksteps = (min(64, nb - t0) + 3) / 4;
#pragma unroll 4
      for (int ks = 0; ks < ksteps; ++ks) {
        const int kk = ks * 4 + lk;
        const double a0 = As[(wr + l16) * GJ_LDA + kk];
        const double a1 = As[(wr + 16 + l16) * GJ_LDA + kk];
        const double b0 = Bs[kk * GJ_LDB + wc + l16];
        const double b1 = Bs[kk * GJ_LDB + wc + 16 + l16];
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
      }
      __syncthreads();  // the next half (or tile) overwrites the staged operands
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + wr + bi * 16 + lk + 4 * v, j = j0 + wc + bj * 16 + l16;
          if (!out_ok(i, j)) continue;
          if (MODE == GJ_UPDATE) A[(long long)i * n + j] = cv[bi][bj][v] - acc[bi][bj][v];
          else Rb[(long long)i * n + j] = acc[bi][bj][v];
        }
  }
}

// New pivot row panel P A_KJ into the lower triangle (row K left of the
// block, column K below it); by symmetry it is also the column panel.
__global__ void k_gj_writeback(int n, double* __restrict__ Ab, int k0, int nb, const double* __restrict__ Rbb,
                               int batch) {
  const long long per = (long long)nb * n, total = per * batch;
  for (long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x; gid < total;
       gid += (long long)gridDim.x * blockDim.x) {
    const long long z = gid / per, e = gid % per;
    double* A = Ab + z * n * n;
    const double* Rb = Rbb + z * GJ_NB * n;
    const int r = int(e / n), j = int(e % n);
    if (j < k0) A[(long long)(k0 + r) * n + j] = Rb[(long long)r * n + j];
    else if (j >= k0 + nb) A[(long long)j * n + k0 + r] = Rb[(long long)r * n + j];
  }
}

// -A (lower triangle, after the last sweep) -> the full symmetric inverse:
// one 64 x 64 tile pair (i0 >= j0) per workgroup through LDS.
__global__ __launch_bounds__(256) void k_gj_finish(int n, double* __restrict__ Ab) {
  __shared__ double t[64][65];
  const int ti = blockIdx.y, tj = blockIdx.x;
  if (tj > ti) return;
  double* A = Ab + (long long)blockIdx.z * n * n;
  const int i0 = ti * 64, j0 = tj * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const int i = i0 + r, j = j0 + c;
    double v = 0.0;
    if (i < n && j < n) v = -A[(long long)max(i, j) * n + min(i, j)];
    t[r][c] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    if (i0 + r < n && j0 + c < n) A[(long long)(i0 + r) * n + j0 + c] = t[r][c];
    if (ti != tj && j0 + r < n && i0 + c < n) A[(long long)(j0 + r) * n + i0 + c] = t[c][r];
  }
}

// ---------------------------------------------------------------------------
// Coarse-coarse shift-invert operator: dense G_J + sigma_J I per cc cell
// (nd_max x nd_max, padded slots and invalid dofs decoupled with a large
// diagonal), inverted by the batched Gauss-Jordan sweep.

// sigma_J = 1e-6 * mean valid diagonal (stored in par[J*8 + 7])
__global__ void k_ccd_shift(CCArgs a, double* __restrict__ par) {
  __shared__ double red[64];
  const int J = a.J0 + blockIdx.x;
  const Hier& h = a.h;
  const int L = h.Lc;
  const int d0 = a.cc_ptr[J], nd = a.cc_ptr[J + 1] - d0;
  double s = 0.0, cnt = 0.0;
  for (int q = threadIdx.x; q < nd; q += blockDim.x) {
    const long long d = a.cc_dofs[d0 + q];
    if (!dof_valid(a, d)) continue;
    const int cell = int(d / L), l = int(d % L);
    s += a.G[(((long long)cell * 27 + 13) * L + l) * L + l];
    cnt += 1.0;
  }
  s = block_allsum(s, red);
  cnt = block_allsum(cnt, red);
  if (threadIdx.x == 0) par[J * 8 + 7] = 1e-6 * (cnt > 0 ? s / cnt : 1.0) + 1e-300;
}

__global__ void k_ccd_assemble(CCArgs a, int ndm, const double* __restrict__ par, double* __restrict__ Gd) {
  const int J = a.J0 + blockIdx.y;
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= (long long)ndm * ndm) return;
  const Hier& h = a.h;
  const int L = h.Lc;
  const int d0 = a.cc_ptr[J], nd = a.cc_ptr[J + 1] - d0;
  const int p = int(e / ndm), q = int(e % ndm);
  double v = 0.0;
  const double big = 1e30;
  if (p >= nd || q >= nd) {
    v = (p == q) ? 1.0 : 0.0;
  } else {
    const long long dp = a.cc_dofs[d0 + p], dq = a.cc_dofs[d0 + q];
    if (!dof_valid(a, dp) || !dof_valid(a, dq)) {
      v = (p == q) ? big : 0.0;
    } else {
      const int cp = int(dp / L), lp = int(dp % L), cq = int(dq / L), lq = int(dq % L);
      const int px = cp % h.ncx, py = (cp / h.ncx) % h.ncy, pz = cp / (h.ncx * h.ncy);
      const int qx = cq % h.ncx, qy = (cq / h.ncx) % h.ncy, qz = cq / (h.ncx * h.ncy);
      const int ox = qx - px, oy = qy - py, oz = qz - pz;
      if (abs(ox) <= 1 && abs(oy) <= 1 && abs(oz) <= 1) {
        const int b = (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1);
        const int bt = (1 - oz) * 9 + (1 - oy) * 3 + (1 - ox);
        // symmetrised entry
        v = 0.5 * (a.G[(((long long)cp * 27 + b) * L + lp) * L + lq] + a.G[(((long long)cq * 27 + bt) * L + lq) * L + lp]);
      }
      if (p == q) v += par[J * 8 + 7];
    }
  }
  Gd[(long long)(J - a.J0) * ndm * ndm + e] = v;
}

// Y = (G + sigma I)^-1 X per active cc cell (the inverse is symmetric: row q of
// it is column q).  A workgroup computes 512 rows x 32 vectors: wave w owns
// rows (w & 1) * 256 + lane + 64 k (k < 4) and vectors (w >> 1) * 16 .. +16,
// so each inverse entry loaded from HBM feeds 16 FMAs and each vector entry
// read from LDS (a broadcast) feeds 4.  Vectors are staged in chunks of 64
// entries, transposed, with rows beyond nd and vectors beyond m zero.
constexpr int CCD_ROWS = 512, CCD_QC = 64, CCD_XS = 34;

__global__ __launch_bounds__(256) void k_ccd_apply(CCArgs a, int ndm, const double* __restrict__ Gi,
                                                   const double* __restrict__ X, double* __restrict__ Y,
                                                   const int* __restrict__ flag) {
  __shared__ __align__(16) double Xs[CCD_QC * CCD_XS];
  const int J = a.J0 + blockIdx.y;
  if (flag[J] >= 0) return;
  const int m = a.m;
  const int d0 = a.cc_ptr[J], nd = a.cc_ptr[J + 1] - d0;
  const int rbase = blockIdx.x * CCD_ROWS;
  if (rbase >= nd) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r0 = rbase + (w & 1) * 256 + lane;
  const int c0 = (w >> 1) * 16;
  const double* G = Gi + (long long)(J - a.J0) * ndm * ndm;
  const double* XJ = X + (long long)m * d0;
  int rc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) rc[k] = min(r0 + 64 * k, ndm - 1);  // clamped: in bounds, result unused
  double acc[4][16];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[k][c] = 0.0;
  for (int q0 = 0; q0 < nd; q0 += CCD_QC) {
    __syncthreads();
    for (int e = tid; e < CCD_QC * 32; e += 256) {
      const int qq = e % CCD_QC, j = e / CCD_QC;
      const int q = q0 + qq;
      Xs[qq * CCD_XS + j] = (j < m && q < nd) ? XJ[(long long)j * nd + q] : 0.0;
    }
    __syncthreads();
    const int qn = min(CCD_QC, nd - q0);
#pragma unroll 2
    for (int qq = 0; qq < qn; ++qq) {
      const double* Gq = G + (long long)(q0 + qq) * ndm;
      double g[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) g[k] = Gq[rc[k]];
      const double2* xs = reinterpret_cast<const double2*>(Xs + qq * CCD_XS + c0);
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const double2 x = xs[c];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          acc[k][2 * c] += g[k] * x.x;
          acc[k][2 * c + 1] += g[k] * x.y;
        }
      }
    }
  }
  double* YJ = Y + (long long)m * d0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int r = r0 + 64 * k;
    if (r >= nd) continue;
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c0 + c < m) YJ[(long long)(c0 + c) * nd + r] = acc[k][c];
  }
}

// ---------------------------------------------------------------------------
// Host launchers

int launch_galerkin(const Ctx& c, const void* R, int b_dt, int drop_cc, double* out, hipStream_t s) {
  const dim3 gr((unsigned)(((c.ntiles + 7) / 8) * 8)), bl(c.CX * c.h.H, c.h.H);
  const size_t sh = (size_t(bl.x) * bl.y * 4 + size_t(bl.y) * c.CX * 4) * sizeof(double);
  const int L = c.h.Lc;
  for (int q = 0; q < 27; ++q) {
    const int qx = q % 3, qy = (q / 3) % 3, qz = q / 9;
#define GL(BT, LT) hipLaunchKernelGGL((k_galerkin<BT, LT>), gr, bl, sh, s, c.g, c.st, c.h, c.CX, c.rho, c.rho_dt, c.mat, (const BT*)R, qx, qy, qz, drop_cc, out)
#define GLL(BT)                                    \
  switch (L) {                                     \
    case 1: GL(BT, 1); break;                      \
    case 2: GL(BT, 2); break;                      \
    case 3: GL(BT, 3); break;                      \
    case 4: GL(BT, 4); break;                      \
    case 5: GL(BT, 5); break;                      \
    case 6: GL(BT, 6); break;                      \
    case 7: GL(BT, 7); break;                      \
    default: GL(BT, 8); break;                     \
  }
    if (b_dt == DT_F64) { GLL(double) }
    else if (b_dt == DT_F32) { GLL(float) }
    else { GLL(bf16) }
#undef GLL
#undef GL
  }
  return hipGetLastError() == hipSuccess ? MSMG_OK : MSMG_EHIP;
}

void launch_block_inverse(const Ctx& c, double* Ac, double* Dinv, hipStream_t s) {
  hipLaunchKernelGGL(k_block_inverse, dim3((c.h.ncells + 63) / 64), dim3(64), 0, s, c.h.ncells, c.h.Lc, Ac, Dinv);
}

// One group of cc cells (J0 .. J0 + nJ - 1): start block, dense path for small
// cells, shift-invert subspace iteration with Rayleigh-Ritz on G, R_cc rows.
static int run_cc_group(const Ctx& c, const SetupArgs& sa, SetupScratch* sc, CCArgs a, SetupReport* rep,
                        hipStream_t s) {
  const Hier& h = c.h;
  const int m = a.m, nJ = a.nJ, J0 = a.J0;
  const long long ndof = (long long)h.ncells * h.Lc;
  const dim3 gt((unsigned)((sa.max_cc_dofs + 255) / 256), nJ), bt(256);
  const dim3 gs((unsigned)((h.max_cc_cells + 63) / 64), nJ, (unsigned)((m + 7) / 8)), bs(64);
  double* Y = sc->Y;
  double* Xp = sc->Yp;
  double* Z = sc->Z;
  double* small = sc->small;
  double* par = sc->ccpar;
  double* ritz = par + (size_t)h.ncc * 8;
  double* bound = ritz + (size_t)h.ncc * m;
  int* flag = sc->ccflag;
  const int small_threads = std::min(1024, std::max(64, ((m * m + 63) / 64) * 64));
  const size_t small_lds = sizeof(double) * (4 * m * m + 3 * m + 64) + sizeof(int) * m;
  int* chol_failed = sc->ccflag + h.ncc;
  hipLaunchKernelGGL(k_cc_bound, dim3(nJ), dim3(256), 0, s, a, bound);
  hipLaunchKernelGGL(k_cc_start, dim3((unsigned)((ndof + 255) / 256)), dim3(256), 0, s, a, Y);
  if (hipMemsetAsync(flag + J0, 0xff, sizeof(int) * nJ, s) != hipSuccess) return MSMG_EHIP;  // -1: active
  {
    const size_t lds = sizeof(double) * (4 * CC_DENSE * CC_DENSE + 3 * CC_DENSE + 64) + sizeof(int) * CC_DENSE;
    hipLaunchKernelGGL(k_cc_dense, dim3(nJ), dim3(1024), lds, s, a, Xp, ritz, flag);
  }
  auto orth = [&](double* P, double* tmp) {
    hipLaunchKernelGGL(k_cc_gram, dim3(nJ, CC_KS), dim3(256), 0, s, a, P, P, sc->gpart, flag);
    hipLaunchKernelGGL(k_cc_gram_sum, dim3(nJ), dim3(256), 0, s, a, sc->gpart, small, 0, flag);
    hipLaunchKernelGGL(k_cc_cholinv, dim3(nJ), dim3(64), 0, s, a, small, 0, flag, chol_failed);
    hipLaunchKernelGGL(k_cc_small_eig, dim3(nJ), dim3(small_threads), small_lds, s, a, small, 0, 0, ritz, flag,
                       (const int*)chol_failed);
    hipLaunchKernelGGL(k_cc_transform, gt, bt, 0, s, a, P, tmp, small, flag);
  };
  auto spmm = [&](const double* P, double* Q) {
    switch (h.Lc) {
#define SPMM_L(L_) case L_: hipLaunchKernelGGL(k_cc_spmm<L_>, gs, bs, 0, s, a, P, Q, flag); break;
      SPMM_L(1) SPMM_L(2) SPMM_L(3) SPMM_L(4) SPMM_L(5) SPMM_L(6) SPMM_L(7) SPMM_L(8)
#undef SPMM_L
    }
  };
  // orthonormalise twice (Y -> Xp -> Y), Rayleigh-Ritz (Z = G Y; X = Y C; Z = Z C)
  auto rr = [&]() {
    orth(Y, Xp);
    orth(Xp, Y);
    spmm(Y, Z);
    hipLaunchKernelGGL(k_cc_gram, dim3(nJ, CC_KS), dim3(256), 0, s, a, Y, Z, sc->gpart, flag);
    hipLaunchKernelGGL(k_cc_gram_sum, dim3(nJ), dim3(256), 0, s, a, sc->gpart, small, 0, flag);
    hipLaunchKernelGGL(k_cc_small_eig, dim3(nJ), dim3(small_threads), small_lds, s, a, small, 0, 1, ritz, flag,
                       (const int*)nullptr);
    hipLaunchKernelGGL(k_cc_transform, gt, bt, 0, s, a, Y, Xp, small, flag);  // Xp = Ritz vectors
    hipLaunchKernelGGL(k_cc_transform, gt, bt, 0, s, a, Z, Y, small, flag);   // Y = G * Ritz vectors
    std::swap(Y, Z);                                                            // Z = G X, Y free
  };
  rr();
  const int maxit = sa.opt->cc_maxit;
  const double tol = sa.opt->eig_tol;
  // shift-invert operator (G_J + sigma_J I)^-1 for every cc cell of the group
  const int ndm = sa.max_cc_dofs;
  hipLaunchKernelGGL(k_ccd_shift, dim3(nJ), dim3(256), 0, s, a, par);
  hipLaunchKernelGGL(k_ccd_assemble, dim3((unsigned)(((long long)ndm * ndm + 255) / 256), nJ), dim3(256), 0, s, a,
                     ndm, par, sc->Gd);
  {
    const int r = timed_gj_inverse(sa, rep, ndm, nJ, sc->Gd, sc->gj, s);
    if (r != MSMG_OK) return r;
  }
  const dim3 ga((ndm + CCD_ROWS - 1) / CCD_ROWS, nJ), ba(256);
  std::vector<int> hf(nJ);
  for (int it = 0; it <= maxit; ++it) {
    hipLaunchKernelGGL(k_cc_check, dim3(nJ), dim3(256), 0, s, a, Xp, Z, ritz, flag, bound, h.Lcc, tol, it,
                       it == maxit ? 1 : 0);
    if (it == maxit) break;
    if (it % 4 == 3) {
      if (hipMemcpyAsync(hf.data(), flag + J0, sizeof(int) * nJ, hipMemcpyDeviceToHost, s) != hipSuccess)
        return MSMG_EHIP;
      if (hipStreamSynchronize(s) != hipSuccess) return MSMG_EHIP;
      bool all = true;
      for (int v : hf) all = all && v >= 0;
      if (all) break;
    }
    // Y = (G + sigma I)^-1 X, then orthonormalise and Rayleigh-Ritz with G
    hipLaunchKernelGGL(k_ccd_apply, ga, ba, 0, s, a, ndm, sc->Gd, Xp, Y, flag);
    rr();
  }
  // X (Ritz vectors) in Xp
  hipLaunchKernelGGL(k_cc_finish, dim3(nJ), dim3(256), 0, s, a, Xp, ritz, sa.Rcc64, sa.cc_evals, h.Lcc);
  return hipGetLastError() == hipSuccess ? MSMG_OK : MSMG_EHIP;
}

int run_cc_eigen(const Ctx& c, const SetupArgs& sa, SetupScratch* sc, const double* G, int* n_unconv, SetupReport* rep,
                 hipStream_t s) {
  const Hier& h = c.h;
  CCArgs a;
  a.h = h;
  a.m = sc->mcc;
  a.G = G;
  a.cc_ptr = sa.cc_ptr;
  a.cc_dofs = sa.cc_dofs;
  a.dof_cc = sa.dof_cc;
  a.dof_loc = sa.dof_loc;
  a.cell_status = sa.cell_status;
  if (a.m > 32 || sc->cc_group < 1) return MSMG_EINVAL;
  // the dense shifted matrices of one group at a time fit the scratch
  for (int J0 = 0; J0 < h.ncc; J0 += sc->cc_group) {
    a.J0 = J0;
    a.nJ = std::min(sc->cc_group, h.ncc - J0);
    const int r = run_cc_group(c, sa, sc, a, rep, s);
    if (r != MSMG_OK) return r;
  }
  int* flag = sc->ccflag;
  std::vector<int> hf(h.ncc);
  if (hipMemcpyAsync(hf.data(), flag, sizeof(int) * h.ncc, hipMemcpyDeviceToHost, s) != hipSuccess) return MSMG_EHIP;
  if (hipMemcpyAsync(sa.cc_status, flag, sizeof(int) * h.ncc, hipMemcpyDeviceToDevice, s) != hipSuccess) return MSMG_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return MSMG_EHIP;
  int nu = 0;
  for (int v : hf) nu += (v < 0);
  *n_unconv = nu;
  return hipGetLastError() == hipSuccess ? MSMG_OK : MSMG_EHIP;
}

int build_acc(const Ctx& c, const SetupArgs& sa, double* u, hipStream_t s) {
  // A_cc = R_cc A_c R_cc^T from the FP64 masters (the cycle may hold an FP32 copy of A_c)
  const Hier& h = c.h;
  const int n = sa.n_cc;
  if (hipMemsetAsync(sa.Acc, 0, sizeof(double) * (size_t)n * n, s) != hipSuccess) return MSMG_EHIP;
  const long long ndof = (long long)h.ncells * h.Lc;
  const dim3 gu((unsigned)((ndof + 255) / 256)), bu(256);
  const long long nw = (long long)h.ncc * h.Lcc;
  const dim3 gd((unsigned)((nw * 64 + 255) / 256)), bd(256);
  // u holds up to ACC_B columns of ndof values (the scratch block has m > Lcc)
  for (int q = 0; q < 27; ++q) {
    const int qx = q % 3, qy = (q / 3) % 3, qz = q / 9;
    if (qx >= h.nccx || qy >= h.nccy || qz >= h.nccz) continue;
    for (int b0 = 0; b0 < h.Lcc; b0 += ACC_B) {
      const int nb = std::min(ACC_B, h.Lcc - b0);
      switch (h.Lc) {
#define ACA(L_) case L_: hipLaunchKernelGGL((k_acc_apply_cols<double, double, L_>), gu, bu, 0, s, h, (const double*)sa.Ac64, (const double*)sa.Rccv, sa.cc_ptr, sa.dof_cc, sa.dof_loc, qx, qy, qz, b0, u, ndof); break;
        ACA(1) ACA(2) ACA(3) ACA(4) ACA(5) ACA(6) ACA(7) ACA(8)
#undef ACA
      }
      const dim3 gdc((unsigned)((nw * nb * 64 + 255) / 256));
      hipLaunchKernelGGL((k_acc_dot_cols<double>), gdc, bd, 0, s, h, (const double*)sa.Rccv, sa.cc_ptr, sa.cc_dofs, u, ndof, qx, qy, qz, b0, n, sa.Acc);
    }
  }
  hipLaunchKernelGGL(k_acc_pad, dim3((n + 255) / 256), dim3(256), 0, s, h, sa.cc_ptr, n, sa.Acc);
  return hipGetLastError() == hipSuccess ? MSMG_OK : MSMG_EHIP;
}

int gj_inverse(int n, int batch, double* A, double* work, hipStream_t s) {
  double* P = work;
  double* Rb = P + (size_t)batch * GJ_NB * GJ_NB;
  for (const void* f : {(const void*)k_gj_tile<GJ_ROW>, (const void*)k_gj_tile<GJ_UPDATE>})
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(GJ_TILE_LDS)) != hipSuccess)
      return MSMG_EHIP;
  if (hipFuncSetAttribute((const void*)k_gj_pivot, hipFuncAttributeMaxDynamicSharedMemorySize, int(GJ_PIVOT_LDS)) !=
      hipSuccess)
    return MSMG_EHIP;
  const unsigned nt = unsigned((n + 63) / 64);
  for (int k0 = 0; k0 < n; k0 += GJ_NB) {
    const int nb = std::min(GJ_NB, n - k0);
    hipLaunchKernelGGL(k_gj_pivot, dim3(1, 1, batch), dim3(1024), GJ_PIVOT_LDS, s, n, A, k0, nb, P);
    // the row panel tiles run along j (GJ_NB / 64 tile rows); the update covers
    // the lower triangle; both loop over (matrix, tile) pairs on at most
    // GJ_WORKGROUPS workgroups
    const long long nrow = (long long)GJ_HALVES * nt * batch, nupd = (long long)nt * (nt + 1) / 2 * batch;
    hipLaunchKernelGGL(k_gj_tile<GJ_ROW>, dim3((unsigned)std::min<long long>(nrow, GJ_WORKGROUPS)), dim3(256),
                       GJ_TILE_LDS, s, n, A, k0, nb, P, Rb, batch);
    hipLaunchKernelGGL(k_gj_tile<GJ_UPDATE>, dim3((unsigned)std::min<long long>(nupd, GJ_WORKGROUPS)), dim3(256),
                       GJ_TILE_LDS, s, n, A, k0, nb, P, Rb, batch);
    const long long rn = (long long)nb * n * batch;
    hipLaunchKernelGGL(k_gj_writeback, dim3((unsigned)std::min<long long>((rn + 255) / 256, 8192)), dim3(256), 0, s,
                       n, A, k0, nb, Rb, batch);
  }
  hipLaunchKernelGGL(k_gj_finish, dim3(nt, nt, batch), dim3(256), 0, s, n, A);
  return hipGetLastError() == hipSuccess ? MSMG_OK : MSMG_EHIP;
}

}  // namespace msmg
