// Coarse levels of the three-grid cycle (Algorithm 1): block Gauss-Seidel
// smoothing on A_c, residuals on level 1, restriction / prolongation with
// R_cc, and the direct coarse-coarse solve (explicit FP64 inverse of A_cc
// applied as a matrix-vector product).
#include "internal.h"

namespace msmg {

// Neighbour block index b = (oz+1)*9 + (oy+1)*3 + (ox+1), 13 = the cell itself.
MSMG_DEV long long nb_cell(const Hier& h, int cx, int cy, int cz, int b, bool& ok) {
  const int ox = b % 3 - 1, oy = (b / 3) % 3 - 1, oz = b / 9 - 1;
  const int x = cx + ox, y = cy + oy, z = cz + oz;
  ok = x >= 0 && x < h.ncx && y >= 0 && y < h.ncy && z >= 0 && z < h.ncz;
  return ((long long)z * h.ncy + y) * h.ncx + x;
}

// One colour of one block Gauss-Seidel sweep started from a zero guess:
//   x_i = D_i^-1 (b_i - sum_{j earlier in the sweep} A_ij x_j)
// for every cell i of the colour (colour = parity of the cell indices).  Cells
// of one colour are never neighbours; cells of later colours are still zero,
// so only earlier colours are read and x needs no clearing.  The forward sweep
// (colours 0..7) is S_c^-1 = (D + L)^-1, the backward sweep (7..0) its
// transpose.
// LP * 8 lanes per cell (LP = power of two >= Lc): lane = (row l, slot q); slot q
// sums the neighbour blocks b = q, q + 8, q + 16, q + 24 of row l; the 8 slots
// of a row are then combined by shuffles (fixed order), so the 27-block
// products of a cell run in parallel.  L is a compile-time constant so that
// every load of a lane (its row of up to four blocks, the matching entries of
// x, b_i and the row of D_i^-1) is issued before the first product.
constexpr int ROW_SLOTS = 8;
constexpr int SLOT_BLOCKS = (27 + ROW_SLOTS - 1) / ROW_SLOTS;

template <int L>
constexpr int lanes_pow2() {
  return L <= 1 ? 1 : L <= 2 ? 2 : L <= 4 ? 4 : 8;
}

// Row l, slot q of one cell: the blocks b = q + 8 k it uses (use[k]) with
// their neighbour cells, loaded with the matching entries of x; part = the
// sum of A_ib x_b over them in the order of b then m (unused blocks add 0).
template <typename VT, typename AT, int L, typename Use>
MSMG_DEV VT row_products(const Hier& h, const AT* __restrict__ A, const VT* __restrict__ x, int cx, int cy, int cz,
                         int l, int q, bool row, Use use_block) {
  bool use[SLOT_BLOCKS];
  long long nc[SLOT_BLOCKS];
#pragma unroll
  for (int k = 0; k < SLOT_BLOCKS; ++k) {
    const int bb = q + ROW_SLOTS * k;
    bool ok = false;
    nc[k] = 0;
    if (row && bb < 27) nc[k] = nb_cell(h, cx, cy, cz, bb, ok);
    use[k] = ok && use_block(bb);
  }
  VT part = VT(0);
  if constexpr (L <= 4) {
    VT av[SLOT_BLOCKS][L], xv[SLOT_BLOCKS][L];
#pragma unroll
    for (int k = 0; k < SLOT_BLOCKS; ++k)
#pragma unroll
      for (int m = 0; m < L; ++m) {
        av[k][m] = use[k] ? ld<VT, AT>(A, ((q + ROW_SLOTS * k) * L + l) * L + m) : VT(0);
        xv[k][m] = use[k] ? x[nc[k] * L + m] : VT(0);
      }
#pragma unroll
    for (int k = 0; k < SLOT_BLOCKS; ++k)
#pragma unroll
      for (int m = 0; m < L; ++m) part += av[k][m] * xv[k][m];
  } else {
    // larger rows: the staged copies would spill; products as the loads land
#pragma unroll
    for (int k = 0; k < SLOT_BLOCKS; ++k)
      if (use[k])
#pragma unroll
        for (int m = 0; m < L; ++m) part += ld<VT, AT>(A, ((q + ROW_SLOTS * k) * L + l) * L + m) * x[nc[k] * L + m];
  }
  return part;
}

template <typename VT, typename AT, int L>
__global__ void k_gs_colour(Hier h, int colour, int forward, const AT* __restrict__ Ac,
                            const AT* __restrict__ Dinv, const VT* __restrict__ b, VT* __restrict__ x,
                            const Scalars* sc) {
  if (sc && sc->done) return;
  constexpr int CL = lanes_pow2<L>() * ROW_SLOTS;
  const long long gtid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int lane = int(gtid % CL);
  const int l = lane / ROW_SLOTS, q = lane % ROW_SLOTS;
  const long long ci = gtid / CL;
  const int px = colour & 1, py = (colour >> 1) & 1, pz = (colour >> 2) & 1;
  const int nx = (h.ncx - px + 1) / 2, ny = (h.ncy - py + 1) / 2, nz = (h.ncz - pz + 1) / 2;
  const bool valid = ci < (long long)nx * ny * nz;
  const bool row = valid && l < L;
  long long cell = 0;
  int cx = 0, cy = 0, cz = 0;
  if (valid) {
    cx = 2 * int(ci % nx) + px;
    cy = 2 * int((ci / nx) % ny) + py;
    cz = 2 * int(ci / ((long long)nx * ny)) + pz;
    cell = ((long long)cz * h.ncy + cy) * h.ncx + cx;
  }
  const VT bi = row ? b[cell * L + l] : VT(0);
  VT dv[L];
#pragma unroll
  for (int m = 0; m < L; ++m) dv[m] = row ? ld<VT, AT>(Dinv, (cell * L + l) * L + m) : VT(0);
  VT part = row_products<VT, AT, L>(h, Ac + cell * 27 * L * L, x, cx, cy, cz, l, q, row, [&](int bb) {
    const int ox = bb % 3 - 1, oy = (bb / 3) % 3 - 1, oz = bb / 9 - 1;
    const int ncol = ((px + ox) & 1) + 2 * ((py + oy) & 1) + 4 * ((pz + oz) & 1);
    return forward ? (ncol < colour) : (ncol > colour);
  });
  // row sums over the 8 slots (xor within aligned groups of 8 lanes)
#pragma unroll
  for (int off = 1; off < ROW_SLOTS; off <<= 1) part += __shfl_xor(part, off, 64);
  const VT t = row ? bi - part : VT(0);
  // x_i = D_i^-1 t: lane (l, 0) of each row computes row l
  const int base = (threadIdx.x / CL) * CL;
  VT upd = VT(0);
#pragma unroll
  for (int m = 0; m < L; ++m) {
    const VT tm = __shfl(t, base + m * ROW_SLOTS, 64);
    if (row) upd += dv[m] * tm;
  }
  if (row && q == 0) x[cell * L + l] = upd;
}

// t = b - A_c x on every cell (lanes per cell as in the sweep).
template <typename VT, typename AT, int L>
__global__ void k_ac_residual(Hier h, const AT* __restrict__ Ac, const VT* __restrict__ b,
                              const VT* __restrict__ x, VT* __restrict__ t, const Scalars* sc) {
  if (sc && sc->done) return;
  constexpr int CL = lanes_pow2<L>() * ROW_SLOTS;
  const long long gtid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int lane = int(gtid % CL);
  const int l = lane / ROW_SLOTS, q = lane % ROW_SLOTS;
  const long long cell = gtid / CL;
  const bool row = cell < h.ncells && l < L;
  int cx = 0, cy = 0, cz = 0;
  if (row) {
    cx = int(cell % h.ncx);
    cy = int((cell / h.ncx) % h.ncy);
    cz = int(cell / ((long long)h.ncx * h.ncy));
  }
  const VT bi = row ? b[cell * L + l] : VT(0);
  VT part = row_products<VT, AT, L>(h, Ac + (row ? cell : 0) * 27 * L * L, x, cx, cy, cz, l, q, row,
                                    [](int) { return true; });
#pragma unroll
  for (int off = 1; off < ROW_SLOTS; off <<= 1) part += __shfl_xor(part, off, 64);
  if (row && q == 0) t[cell * L + l] = bi - part;
}

// r_cc[J*Lcc + b] = sum_d R_cc[J][b][d] t[cc_dofs[d]]: one wave per output entry.
template <typename VT>
__global__ void k_cc_restrict(Hier h, const VT* __restrict__ Rcc, const int* __restrict__ cc_ptr,
                              const int* __restrict__ cc_dofs, const VT* __restrict__ t, double* __restrict__ rcc,
                              const Scalars* sc) {
  if (sc && sc->done) return;
  const long long w = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (w >= (long long)h.ncc * h.Lcc) return;
  const int J = int(w / h.Lcc), bidx = int(w % h.Lcc);
  const int d0 = cc_ptr[J], nd = cc_ptr[J + 1] - d0;
  const VT* R = Rcc + (long long)h.Lcc * d0 + (long long)bidx * nd;
  double s = 0.0;
  for (int d = lane; d < nd; d += 64) s += double(R[d]) * double(t[cc_dofs[d0 + d]]);
  s = wave_sum(s);
  if (lane == 0) rcc[w] = s;
}

// e = AccInv r (dense symmetric FP64): one wave per row.
__global__ void k_acc_solve(int n, const double* __restrict__ Ainv, const double* __restrict__ r,
                            double* __restrict__ e, const Scalars* sc) {
  if (sc && sc->done) return;
  const long long row = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const double* a = Ainv + row * (long long)n;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += a[j] * r[j];
  s = wave_sum(s);
  if (lane == 0) e[row] = s;
}

// out[d] = base[d] + sum_b R_cc[J][b][loc(d)] e[J*Lcc + b]
template <typename VT>
__global__ void k_cc_prolong(Hier h, int n_c, const VT* __restrict__ Rcc, const int* __restrict__ cc_ptr,
                             const int* __restrict__ dof_cc, const int* __restrict__ dof_loc,
                             const VT* __restrict__ base, const double* __restrict__ e, VT* __restrict__ out,
                             const Scalars* sc) {
  if (sc && sc->done) return;
  const long long d = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (d >= n_c) return;
  const int J = dof_cc[d], loc = dof_loc[d];
  const int d0 = cc_ptr[J], nd = cc_ptr[J + 1] - d0;
  const VT* R = Rcc + (long long)h.Lcc * d0;
  double s = base ? double(base[d]) : 0.0;
  for (int b = 0; b < h.Lcc; ++b) s += double(R[(long long)b * nd + loc]) * e[(long long)J * h.Lcc + b];
  out[d] = VT(s);
}

// ---------------------------------------------------------------------------
// dispatch over the number of basis vectors per cell (1 .. LC_MAX)
#define COARSE_L_DISPATCH(Lrt, ...)                          \
  do {                                                       \
    switch (Lrt) {                                           \
      case 1: { constexpr int LL = 1; __VA_ARGS__; } break;  \
      case 2: { constexpr int LL = 2; __VA_ARGS__; } break;  \
      case 3: { constexpr int LL = 3; __VA_ARGS__; } break;  \
      case 4: { constexpr int LL = 4; __VA_ARGS__; } break;  \
      case 5: { constexpr int LL = 5; __VA_ARGS__; } break;  \
      case 6: { constexpr int LL = 6; __VA_ARGS__; } break;  \
      case 7: { constexpr int LL = 7; __VA_ARGS__; } break;  \
      default: { constexpr int LL = 8; __VA_ARGS__; } break; \
    }                                                        \
  } while (0)
static_assert(LC_MAX == 8, "COARSE_L_DISPATCH covers 1 .. 8");

static inline int lanes_per_cell(int L) {
  int lp = 1;
  while (lp < L) lp <<= 1;
  return lp;
}

void launch_gs_sweep(const Ctx& c, const void* b, void* x, bool forward, hipStream_t s) {
  const Hier& h = c.h;
  const int LP = lanes_per_cell(h.Lc);
  for (int q = 0; q < 8; ++q) {
    const int colour = forward ? q : 7 - q;
    const int px = colour & 1, py = (colour >> 1) & 1, pz = (colour >> 2) & 1;
    const long long ncol = (long long)((h.ncx - px + 1) / 2) * ((h.ncy - py + 1) / 2) * ((h.ncz - pz + 1) / 2);
    if (ncol == 0) continue;
    const long long nthreads = ncol * LP * ROW_SLOTS;
    const dim3 gr((unsigned)((nthreads + 255) / 256)), bl(256);
#define GS(VT, AT) COARSE_L_DISPATCH(h.Lc, hipLaunchKernelGGL((k_gs_colour<VT, AT, LL>), gr, bl, 0, s, h, colour, forward ? 1 : 0, (const AT*)c.cc.Ac, (const AT*)c.cc.AcDinv, (const VT*)b, (VT*)x, c.sc))
    if (c.cc.a_dt == DT_F64) GS(double, double);
    else GS(double, float);
#undef GS
  }
}

void launch_ac_residual(const Ctx& c, const void* b, const void* x, void* t, hipStream_t s) {
  const int LP = lanes_per_cell(c.h.Lc);
  const long long n = (long long)c.h.ncells * LP * ROW_SLOTS;
  const dim3 gr((unsigned)((n + 255) / 256)), bl(256);
#define AR(VT, AT) COARSE_L_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_ac_residual<VT, AT, LL>), gr, bl, 0, s, c.h, (const AT*)c.cc.Ac, (const VT*)b, (const VT*)x, (VT*)t, c.sc))
  if (c.cc.a_dt == DT_F64) AR(double, double);
  else AR(double, float);
#undef AR
}

void launch_cc_restrict(const Ctx& c, const void* t, double* rcc, hipStream_t s) {
  const long long nw = (long long)c.h.ncc * c.h.Lcc;
  const dim3 gr((unsigned)((nw * 64 + 255) / 256)), bl(256);
  hipLaunchKernelGGL((k_cc_restrict<double>), gr, bl, 0, s, c.h, (const double*)c.cc.Rcc, c.cc.cc_ptr, c.cc.cc_dofs, (const double*)t, rcc, c.sc);
}

void launch_acc_solve(const Ctx& c, const double* rcc, double* ecc, hipStream_t s) {
  const long long n = c.cc.n_cc;
  const dim3 gr((unsigned)((n * 64 + 255) / 256)), bl(256);
  hipLaunchKernelGGL(k_acc_solve, gr, bl, 0, s, c.cc.n_cc, c.cc.AccInv, rcc, ecc, c.sc);
}

void launch_cc_prolong(const Ctx& c, const void* base, const double* ecc, void* out, hipStream_t s) {
  const long long n = c.cc.n_c;
  const dim3 gr((unsigned)((n + 255) / 256)), bl(256);
  hipLaunchKernelGGL((k_cc_prolong<double>), gr, bl, 0, s, c.h, c.cc.n_c, (const double*)c.cc.Rcc, c.cc.cc_ptr, c.cc.dof_cc, c.cc.dof_loc, (const double*)base, ecc, (double*)out, c.sc);
}

}  // namespace msmg
