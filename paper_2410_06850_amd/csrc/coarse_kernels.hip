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
  // eight entries per lane in flight (the index loads, then the values they
  // address), summed in the order d = lane, lane + 64, ...
  for (int db = lane; db < nd; db += 8 * 64) {
    int idx[8];
    double rv[8], tv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int d = db + 64 * u < nd ? db + 64 * u : 0;
      idx[u] = cc_dofs[d0 + d];
      rv[u] = double(R[d]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) tv[u] = double(t[idx[u]]);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (db + 64 * u < nd) s += rv[u] * tv[u];
  }
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
  // eight entries per lane in flight, summed in the order j = lane, lane + 64, ...
  for (int jb = lane; jb < n; jb += 8 * 64) {
    double av[8], rv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = jb + 64 * u < n ? jb + 64 * u : 0;
      av[u] = a[j];
      rv[u] = r[j];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (jb + 64 * u < n) s += av[u] * rv[u];
  }
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
// Levels 1 and 2 of Algorithm 1 in one grid-synchronised launch.
//
// The coarse work between the restriction and the prolongation is about twenty
// dependent steps (eight colours of the forward sweep, the residual, the
// coarse-coarse restriction, the direct solve with its prolongation, eight
// colours of the backward sweep), each far too small to fill the GPU; as
// separate launches they cost more in launch gaps than in work.  Here one
// workgroup per compute unit runs every step, with a grid-wide barrier
// between steps.  The grid never exceeds the number of workgroups the device
// keeps resident at once, so all of them run together; each barrier wait is
// bounded (spin_limit polls): a workgroup that exceeds it stops waiting, and
// the solve reports MSMG_ETIMEOUT instead of hanging.
//
// Values one step writes and a later step reads on another workgroup (the
// coarse iterate, the residual, r_cc) go through agent-scope atomic exchanges
// and loads, which are performed at the device's coherence point: the compute
// units of different XCDs do not share an L2.  A workgroup waits for the
// results of its exchanges before it arrives at a barrier, so its values are in
// place when the last arrival releases the others.  Read-only data (A_c, the
// block inverses, R_cc, A_cc^-1, the restricted residual written by the
// previous kernel) use ordinary loads.
//
// Backward sweep: Algorithm 1 sets e_c = x1 + S_c^-T (r_c - A_c x1).  One
// Gauss-Seidel sweep over the colours 7..0 on A_c e = r_c started from x1,
// updating x in place from all 27 neighbour blocks, computes exactly this
// (the update of a cell sees x1 on colours not yet swept and the new values on
// the swept ones, which is the transposed sweep applied to the residual), so
// the residual step before it and the separate correction vector disappear.
// Per right-hand side (one or two, see NS): rc, x, t, rcc, sc.  With two
// sides the lanes of one cell's two sides sit in one wave, so their loads of
// A_c, R_cc and A_cc^-1 are the same addresses and coalesce.
struct Level1Args {
  Hier h;
  const double* Ac;          // [ncells][27][L][L]
  const double* Dinv;        // [ncells][L][L] inverses of the diagonal blocks
  Two<const double*> rc;     // R_c (r0 - A r1), from the previous kernel
  Two<double*> x;            // coarse iterate: x0, then x1, then e_c
  Two<double*> t;            // r_c - A_c x0
  Two<double*> rcc;          // R_cc t
  const double* Rcc;         // per cc cell J: [Lcc][nd_J]
  const int* cc_ptr;
  const int* cc_dofs;
  const double* AccInv;      // [n_cc][n_cc]
  int n_cc;
  unsigned* bar;             // barrier words (level1_barrier_words(), zero between launches)
  Two<Scalars*> sc;
  unsigned spin_limit;
};

MSMG_DEV double coh_load(const double* p) {
  return __longlong_as_double((long long)__hip_atomic_load(reinterpret_cast<unsigned long long*>(const_cast<double*>(p)),
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
MSMG_DEV unsigned long long coh_store(double* p, double v) {
  return __hip_atomic_exchange(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier words (each on its own 128-byte line): arrivals of the 8 workgroup
// groups (workgroup b belongs to group b % 8, the XCD the hardware deals it
// to), arrivals of the groups, the release word each group polls, the exits.
constexpr int L1B_GROUPS = 8, L1B_LINE = 32;
constexpr int L1B_GLOBAL = L1B_GROUPS * L1B_LINE, L1B_RELEASE = L1B_GLOBAL + L1B_LINE;
constexpr int L1B_EXIT = L1B_RELEASE + L1B_GROUPS * L1B_LINE;
constexpr int L1B_WORDS = L1B_EXIT + 1;

// Grid-wide barrier number `k` (1, 2, ...), two-level so that no counter
// serialises more than a few dozen atomics: a workgroup counts itself in its
// group; the group's last arrival counts the group globally; the last group
// publishes k in every group's release word, which the group polls.  Counters
// only grow within a launch (each workgroup arrives once per barrier), so
// arrival number k * size - 1 is the last one of barrier k.  Returns false
// (and stops waiting at later barriers) when a wait exceeded the spin limit.
MSMG_DEV bool l1_barrier(const Level1Args& a, unsigned k, unsigned long long seen, int* ok_sh) {
  asm volatile("" ::"v"(seen) : "memory");  // this thread's exchanges have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = *ok_sh;
    const unsigned ng = gridDim.x < L1B_GROUPS ? gridDim.x : L1B_GROUPS;
    const unsigned g = blockIdx.x % L1B_GROUPS;
    const unsigned gsize = (gridDim.x - g + L1B_GROUPS - 1) / L1B_GROUPS;
    unsigned* rel = a.bar + L1B_RELEASE + g * L1B_LINE;
    const unsigned t = __hip_atomic_fetch_add(a.bar + g * L1B_LINE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (t == k * gsize - 1) {
      const unsigned tg = __hip_atomic_fetch_add(a.bar + L1B_GLOBAL, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (tg == k * ng - 1)
        for (unsigned q = 0; q < ng; ++q)
          __hip_atomic_store(a.bar + L1B_RELEASE + q * L1B_LINE, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (ok) {
      unsigned n = 0;
      while (__hip_atomic_load(rel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k) {
        __builtin_amdgcn_s_sleep(1);
        if (++n >= a.spin_limit) {
          ok = 0;
          break;
        }
      }
    }
    *ok_sh = ok;
  }
  __syncthreads();
  return *ok_sh != 0;
}

// sum over the lane's neighbour blocks k (ok[k]) of A_{i,bb} x_{nc[k]} for row
// l of the cell's 27 blocks A (bb = q + ROW_SLOTS k), with every load of A and
// of x issued before the first product (the coherent loads of x would
// otherwise go one block at a time); nc[k] of a skipped block is any valid
// cell, its loads are not used.  Products in the order k, then m.
template <int L>
MSMG_DEV double l1_block_products(const double* A, const double* x, int l, int q, const bool (&ok)[SLOT_BLOCKS],
                                  const long long (&nc)[SLOT_BLOCKS]) {
  double av[SLOT_BLOCKS][L], xv[SLOT_BLOCKS][L];
#pragma unroll
  for (int k = 0; k < SLOT_BLOCKS; ++k) {
    const int bb = ok[k] ? q + ROW_SLOTS * k : 0;
#pragma unroll
    for (int m = 0; m < L; ++m) {
      av[k][m] = A[(bb * L + l) * L + m];
      xv[k][m] = coh_load(x + nc[k] * L + m);
    }
  }
  double part = 0.0;
#pragma unroll
  for (int k = 0; k < SLOT_BLOCKS; ++k)
    if (ok[k]) {
#pragma unroll
      for (int m = 0; m < L; ++m) part += av[k][m] * xv[k][m];
    }
  return part;
}

// One Gauss-Seidel colour of the grid-synchronised sweep.  forward: x_i =
// D_i^-1 (b_i - sum_{j of earlier colours} A_ij x_j) (zero start, colour 0
// first).  !forward: x_i += D_i^-1 (b_i - sum_{all 27 j} A_ij x_j) (in place).
template <int L, int NS>
MSMG_DEV unsigned long long l1_colour(const Level1Args& a, int colour, bool forward) {
  constexpr int CL = lanes_pow2<L>() * ROW_SLOTS;
  const Hier& h = a.h;
  const int px = colour & 1, py = (colour >> 1) & 1, pz = (colour >> 2) & 1;
  const int nx = (h.ncx - px + 1) / 2, ny = (h.ncy - py + 1) / 2, nz = (h.ncz - pz + 1) / 2;
  const long long total = (long long)nx * ny * nz * CL * NS;
  const long long stride = (long long)gridDim.x * blockDim.x;
  unsigned long long seen = 0;
  // the loop bound is uniform over a wave (base differs per wave by multiples of 64)
  for (long long base = (long long)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < total; base += stride) {
    const long long gtid = base + (threadIdx.x & 63);
    const int lane = int(gtid % CL);
    const int side = NS == 1 ? 0 : int((gtid / CL) % NS);
    const int l = lane / ROW_SLOTS, q = lane % ROW_SLOTS;
    const long long ci = gtid / (CL * NS);
    const bool valid = gtid < total;
    const bool row = valid && l < L;
    double* __restrict__ x = a.x[side];
    long long cell = 0;
    int cx = 0, cy = 0, cz = 0;
    if (valid) {
      cx = 2 * int(ci % nx) + px;
      cy = 2 * int((ci / nx) % ny) + py;
      cz = 2 * int(ci / ((long long)nx * ny)) + pz;
      cell = ((long long)cz * h.ncy + cy) * h.ncx + cx;
    }
    const double bi = row ? a.rc[side][cell * L + l] : 0.0;
    const double xi = (row && !forward) ? coh_load(x + cell * L + l) : 0.0;
    double dv[L];
#pragma unroll
    for (int m = 0; m < L; ++m) dv[m] = row ? a.Dinv[(cell * L + l) * L + m] : 0.0;
    // row_products with coherent loads of x
    bool okk[SLOT_BLOCKS];
    long long ncs[SLOT_BLOCKS];
#pragma unroll
    for (int k = 0; k < SLOT_BLOCKS; ++k) {
      const int bb = q + ROW_SLOTS * k;
      bool ok = false;
      long long nc = 0;
      if (row && bb < 27) nc = nb_cell(h, cx, cy, cz, bb, ok);
      if (ok && forward) {
        const int ox = bb % 3 - 1, oy = (bb / 3) % 3 - 1, oz = bb / 9 - 1;
        const int ncol = ((px + ox) & 1) + 2 * ((py + oy) & 1) + 4 * ((pz + oz) & 1);
        ok = ncol < colour;
      }
      okk[k] = ok;
      ncs[k] = ok ? nc : cell;
    }
    double part = l1_block_products<L>(a.Ac + cell * 27 * L * L, x, row ? l : 0, q, okk, ncs);
#pragma unroll
    for (int off = 1; off < ROW_SLOTS; off <<= 1) part += __shfl_xor(part, off, 64);
    const double tv = row ? bi - part : 0.0;
    const int gbase = (threadIdx.x & 63) / CL * CL;
    double upd = 0.0;
#pragma unroll
    for (int m = 0; m < L; ++m) {
      const double tm = __shfl(tv, gbase + m * ROW_SLOTS, 64);
      if (row) upd += dv[m] * tm;
    }
    if (row && q == 0) seen |= coh_store(x + cell * L + l, xi + upd);
  }
  return seen;
}

template <int L, int NS>
__global__ __launch_bounds__(512) void k_level1(Level1Args a) {
  bool all_done = true;
#pragma unroll
  for (int q = 0; q < NS; ++q) all_done = all_done && a.sc[q]->done;
  if (all_done) return;  // uniform: set by earlier kernels
  __shared__ int ok_sh;
  __shared__ double ecc_sh[NS][64];
  if (threadIdx.x == 0) ok_sh = 1;
  __syncthreads();
  const Hier& h = a.h;
  constexpr int CL = lanes_pow2<L>() * ROW_SLOTS;
  const long long stride = (long long)gridDim.x * blockDim.x;
  unsigned k = 0;
  bool ok = true;
  // forward sweep from zero: x0 = S_c^-1 r_c
  for (int colour = 0; colour < 8; ++colour) {
    const unsigned long long seen = l1_colour<L, NS>(a, colour, true);
    ok = l1_barrier(a, ++k, seen, &ok_sh);
  }
  // t = r_c - A_c x0
  {
    unsigned long long seen = 0;
    const long long total = (long long)h.ncells * CL * NS;
    for (long long base = (long long)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < total; base += stride) {
      const long long gtid = base + (threadIdx.x & 63);
      const int lane = int(gtid % CL);
      const int side = NS == 1 ? 0 : int((gtid / CL) % NS);
      const int l = lane / ROW_SLOTS, q = lane % ROW_SLOTS;
      const long long cell = gtid / (CL * NS);
      const bool row = gtid < total && l < L;
      const double* x = a.x[side];
      int cx = 0, cy = 0, cz = 0;
      if (row) {
        cx = int(cell % h.ncx);
        cy = int((cell / h.ncx) % h.ncy);
        cz = int(cell / ((long long)h.ncx * h.ncy));
      }
      const long long cs = row ? cell : 0;
      bool okk[SLOT_BLOCKS];
      long long ncs[SLOT_BLOCKS];
#pragma unroll
      for (int kk = 0; kk < SLOT_BLOCKS; ++kk) {
        const int bb = q + ROW_SLOTS * kk;
        bool okb = false;
        long long nc = 0;
        if (row && bb < 27) nc = nb_cell(h, cx, cy, cz, bb, okb);
        okk[kk] = okb;
        ncs[kk] = okb ? nc : cs;
      }
      double part = l1_block_products<L>(a.Ac + cs * 27 * L * L, x, row ? l : 0, q, okk, ncs);
#pragma unroll
      for (int off = 1; off < ROW_SLOTS; off <<= 1) part += __shfl_xor(part, off, 64);
      if (row && q == 0) seen |= coh_store(a.t[side] + cell * L + l, a.rc[side][cell * L + l] - part);
    }
    ok = l1_barrier(a, ++k, seen, &ok_sh);
  }
  // r_cc = R_cc t: one wave per entry (J, b) and side
  {
    unsigned long long seen = 0;
    const long long nw = (long long)h.ncc * h.Lcc * NS;
    const int lane = threadIdx.x & 63;
    for (long long w = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < nw; w += stride >> 6) {
      const int side = NS == 1 ? 0 : int(w % NS);
      const long long we = w / NS;
      const int J = int(we / h.Lcc), bidx = int(we % h.Lcc);
      const int d0 = a.cc_ptr[J], nd = a.cc_ptr[J + 1] - d0;
      const double* R = a.Rcc + (long long)h.Lcc * d0 + (long long)bidx * nd;
      const double* t = a.t[side];
      double sum = 0.0;
      // eight entries per lane at a time: the index loads, then the coherent
      // loads they address, then the products in the order d = lane, lane + 64, ...
      for (int db = lane; db < nd; db += 8 * 64) {
        int idx[8];
        double rv[8], tv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int d = db + 64 * u < nd ? db + 64 * u : 0;
          idx[u] = a.cc_dofs[d0 + d];
          rv[u] = R[d];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) tv[u] = coh_load(t + idx[u]);
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (db + 64 * u < nd) sum += rv[u] * tv[u];
      }
      sum = wave_sum(sum);
      if (lane == 0) seen |= coh_store(a.rcc[side] + we, sum);
    }
    ok = l1_barrier(a, ++k, seen, &ok_sh);
  }
  // per coarse-coarse cell J (one workgroup at a time): e_J = rows J of
  // A_cc^-1 r_cc (direct solve), then x1 = x0 + R_cc^T e_J on J's dofs
  {
    unsigned long long seen = 0;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
    for (int J = blockIdx.x; J < h.ncc; J += gridDim.x) {
      for (int b = wave; b < h.Lcc; b += nwaves) {
        const double* arow = a.AccInv + (long long)(J * h.Lcc + b) * a.n_cc;
        double sum[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) sum[q] = 0.0;
        // eight entries per lane at a time, summed in the order j = lane, lane + 64, ...
        for (int jb = lane; jb < a.n_cc; jb += 8 * 64) {
          double av[8], rv[NS][8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int j = jb + 64 * u < a.n_cc ? jb + 64 * u : 0;
            av[u] = arow[j];
#pragma unroll
            for (int q = 0; q < NS; ++q) rv[q][u] = coh_load(a.rcc[q] + j);
          }
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (jb + 64 * u < a.n_cc) {
#pragma unroll
              for (int q = 0; q < NS; ++q) sum[q] += av[u] * rv[q][u];
            }
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          sum[q] = wave_sum(sum[q]);
          if (lane == 0) ecc_sh[q][b] = sum[q];
        }
      }
      __syncthreads();
      const int d0 = a.cc_ptr[J], nd = a.cc_ptr[J + 1] - d0;
      const double* R = a.Rcc + (long long)h.Lcc * d0;
      for (int d = threadIdx.x; d < nd; d += blockDim.x) {
        const int gd = a.cc_dofs[d0 + d];
        double v[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) v[q] = coh_load(a.x[q] + gd);
        for (int b = 0; b < h.Lcc; ++b) {
          const double rv = R[(long long)b * nd + d];
#pragma unroll
          for (int q = 0; q < NS; ++q) v[q] += rv * ecc_sh[q][b];
        }
#pragma unroll
        for (int q = 0; q < NS; ++q) seen |= coh_store(a.x[q] + gd, v[q]);
      }
      __syncthreads();
    }
    ok = l1_barrier(a, ++k, seen, &ok_sh);
  }
  // backward sweep from x1 on r_c: x = x1 + S_c^-T (r_c - A_c x1) = e_c
  for (int colour = 7; colour >= 0; --colour) {
    const unsigned long long seen = l1_colour<L, NS>(a, colour, false);
    if (colour > 0) ok = l1_barrier(a, ++k, seen, &ok_sh);
    else asm volatile("" ::"v"(seen) : "memory");
  }
  // the last workgroup to leave resets the counters; a failed wait is reported
  __syncthreads();
  if (threadIdx.x == 0) {
    if (!ok) {
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        a.sc[q]->status = ST_SYNC_TIMEOUT;
        a.sc[q]->done = 1;
      }
    }
    const unsigned ticket = __hip_atomic_fetch_add(a.bar + L1B_EXIT, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ticket == gridDim.x - 1)
      for (int w = 0; w < L1B_WORDS; w += (w < L1B_EXIT ? L1B_LINE : 1))
        __hip_atomic_store(a.bar + w, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
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

int level1_barrier_words() { return L1B_WORDS; }

int level1_blocks() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) return 0;
  int per = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_level1<4, 2>), 512, 0) !=
          hipSuccess ||
      per < 1)
    return 0;
  return cus;  // one workgroup per compute unit (co-resident: per >= 1)
}

static Level1Args level1_args(const Ctx& c, unsigned* bar, unsigned spin_limit) {
  Level1Args a{};
  a.h = c.h;
  a.Ac = (const double*)c.cc.Ac;
  a.Dinv = (const double*)c.cc.AcDinv;
  a.Rcc = (const double*)c.cc.Rcc;
  a.cc_ptr = c.cc.cc_ptr;
  a.cc_dofs = c.cc.cc_dofs;
  a.AccInv = c.cc.AccInv;
  a.n_cc = c.cc.n_cc;
  a.bar = bar;
  a.spin_limit = spin_limit;
  return a;
}

hipError_t launch_level1(const Ctx& c, int blocks, const double* rc, double* x, double* t, double* rcc,
                         unsigned* bar, unsigned spin_limit, hipStream_t s) {
  if (c.cc.a_dt != DT_F64 || c.h.Lcc > 64 || blocks < 1) return hipErrorInvalidValue;
  Level1Args a = level1_args(c, bar, spin_limit);
  a.rc = one(rc);
  a.x = one(x);
  a.t = one(t);
  a.rcc = one(rcc);
  a.sc = one(c.sc);
  // An ordinary launch: `blocks` is at most the device's co-resident capacity
  // for this kernel (level1_blocks), and the kernels before it on the stream
  // finish without waiting for it, so every workgroup becomes resident; the
  // cooperative launch API gives the same guarantee but delays the start of
  // the kernel (about 20 us per launch measured at 256^3), and the bounded
  // waits turn any failure of the assumption into MSMG_ETIMEOUT instead of a
  // hang.
  COARSE_L_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_level1<LL, 1>), dim3(blocks), dim3(512), 0, s, a));
  return hipGetLastError();
}

hipError_t launch_level1_pair(const Ctx& c0, const Ctx& c1, int blocks, const double* rc0, const double* rc1,
                              double* x0, double* x1, double* t0, double* t1, double* rcc0, double* rcc1,
                              unsigned* bar, unsigned spin_limit, hipStream_t s) {
  if (c0.cc.a_dt != DT_F64 || c0.h.Lcc > 64 || blocks < 1) return hipErrorInvalidValue;
  Level1Args a = level1_args(c0, bar, spin_limit);
  a.rc = two(rc0, rc1);
  a.x = two(x0, x1);
  a.t = two(t0, t1);
  a.rcc = two(rcc0, rcc1);
  a.sc = two(c0.sc, c1.sc);
  COARSE_L_DISPATCH(c0.h.Lc, hipLaunchKernelGGL((k_level1<LL, 2>), dim3(blocks), dim3(512), 0, s, a));
  return hipGetLastError();
}

void launch_cc_prolong(const Ctx& c, const void* base, const double* ecc, void* out, hipStream_t s) {
  const long long n = c.cc.n_c;
  const dim3 gr((unsigned)((n + 255) / 256)), bl(256);
  hipLaunchKernelGGL((k_cc_prolong<double>), gr, bl, 0, s, c.h, c.cc.n_c, (const double*)c.cc.Rcc, c.cc.cc_ptr, c.cc.dof_cc, c.cc.dof_loc, (const double*)base, ecc, (double*)out, c.sc);
}

}  // namespace msmg
