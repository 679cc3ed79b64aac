// Shared device-side definitions for the MsMG HIP library (gfx950, wave64).
//
// Node layout: n = (k*(ny+1) + j)*(nx+1) + i, element layout e = (k*ny + j)*nx + i
// (x fastest).  Element-local node a = ax + 2*ay + 4*az.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MSMG_DEV __device__ __forceinline__
#define MSMG_HD __host__ __device__ __forceinline__

namespace msmg {

// ---------------------------------------------------------------------------
// bf16 storage: upper half of an IEEE binary32, round-to-nearest-even.
struct bf16 {
  uint16_t bits;
};

MSMG_HD float bf16_to_float(bf16 v) {
  union { uint32_t u; float f; } c;
  c.u = uint32_t(v.bits) << 16;
  return c.f;
}

MSMG_HD bf16 float_to_bf16(float f) {
  union { uint32_t u; float f; } c;
  c.f = f;
  uint32_t u = c.u;
  bf16 r;
  if ((u & 0x7f800000u) == 0x7f800000u) {  // inf / nan: truncate, keep nan quiet
    r.bits = uint16_t((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    return r;
  }
  u += 0x7fffu + ((u >> 16) & 1u);
  r.bits = uint16_t(u >> 16);
  return r;
}

template <typename T> MSMG_HD double to_f64(T v);
template <> MSMG_HD double to_f64<double>(double v) { return v; }
template <> MSMG_HD double to_f64<float>(float v) { return double(v); }
template <> MSMG_HD double to_f64<bf16>(bf16 v) { return double(bf16_to_float(v)); }

template <typename T> MSMG_HD float to_f32(T v);
template <> MSMG_HD float to_f32<double>(double v) { return float(v); }
template <> MSMG_HD float to_f32<float>(float v) { return v; }
template <> MSMG_HD float to_f32<bf16>(bf16 v) { return bf16_to_float(v); }

// load a stored value into the working type W
template <typename W, typename T> MSMG_HD W ld(const T* p, long long i);
template <> MSMG_HD double ld<double, double>(const double* p, long long i) { return p[i]; }
template <> MSMG_HD double ld<double, float>(const float* p, long long i) { return double(p[i]); }
template <> MSMG_HD double ld<double, bf16>(const bf16* p, long long i) { return double(bf16_to_float(p[i])); }
template <> MSMG_HD float ld<float, double>(const double* p, long long i) { return float(p[i]); }
template <> MSMG_HD float ld<float, float>(const float* p, long long i) { return p[i]; }
template <> MSMG_HD float ld<float, bf16>(const bf16* p, long long i) { return bf16_to_float(p[i]); }

// convert a raw stored value to the working type W
template <typename W, typename T> MSMG_HD W cvt(T v);
template <> MSMG_HD double cvt<double, double>(double v) { return v; }
template <> MSMG_HD double cvt<double, float>(float v) { return double(v); }
template <> MSMG_HD double cvt<double, bf16>(bf16 v) { return double(bf16_to_float(v)); }
template <> MSMG_HD float cvt<float, double>(double v) { return float(v); }
template <> MSMG_HD float cvt<float, float>(float v) { return v; }
template <> MSMG_HD float cvt<float, bf16>(bf16 v) { return bf16_to_float(v); }

template <typename T> MSMG_HD T from_f64(double v);
template <> MSMG_HD double from_f64<double>(double v) { return v; }
template <> MSMG_HD float from_f64<float>(double v) { return float(v); }
// One rounding from binary64 to bf16 (round to nearest even): the value is first
// rounded to binary32 *to odd* (truncate, then set the last bit when anything
// was cut off), which keeps the information the second rounding needs; binary32
// carries 16 more significand bits than bf16, so the second, nearest-even,
// rounding then equals a direct one.
template <> MSMG_HD bf16 from_f64<bf16>(double v) {
  union { uint32_t u; float f; } c;
  c.f = float(v);
  const double back = double(c.f);
  if (back != v && v == v) {
    if ((back < 0.0 ? -back : back) > (v < 0.0 ? -v : v)) c.u -= 1u;  // toward zero
    c.u |= 1u;
  }
  return float_to_bf16(c.f);
}

// ---------------------------------------------------------------------------
// Mesh geometry and the unit-conductivity Q1 stencil coefficients.
struct Geo {
  int nx, ny, nz;     // elements per axis
  int nnx, nny, nnz;  // nodes per axis
  long long nn;       // nodes
  long long ne;       // elements
  double hx, hy, hz, vol;
};

// Entries of the unit-k element matrix K0[a][b] grouped by which coordinates of
// a and b differ: self (none), ax[d] (only axis d), fd[d] (the two axes other
// than d), bd (all three).
struct Stencil {
  double self, ax[3], fd[3], bd;
  int cubic;  // 1 when every ax[d] is exactly zero (cube elements)
};

// Material law k = kmin + rho^p (kmax - kmin)  (paper eq. material).
struct Material {
  double kmin, kmax;
  int p;
};

template <typename W>
MSMG_DEV W conductivity(W rho, W kmin, W dk, int p) {
  W rp = rho;
  for (int t = 1; t < p; ++t) rp *= rho;
  return kmin + rp * dk;
}

// Coarse hierarchy geometry.
struct Hier {
  int H;                 // nodes per coarse cell per axis (last cell keeps the remainder)
  int ncx, ncy, ncz;     // coarse cells per axis
  int ncells;
  int Lc;                // basis vectors per coarse cell (padded)
  int sd;                // coarse cells per cc cell per axis (last keeps remainder)
  int nccx, nccy, nccz;  // cc cells per axis
  int ncc;
  int Lcc;
  int max_cc_cells;      // max coarse cells in one cc cell
};

MSMG_HD int owner_axis(int i, int H, int nc) {
  int c = i / H;
  return c < nc ? c : nc - 1;
}
MSMG_HD int cell_begin(int c, int H) { return c * H; }
MSMG_HD int cell_end(int c, int H, int nc, int nnodes_axis) {
  return (c == nc - 1) ? nnodes_axis : (c + 1) * H;
}
MSMG_HD int group_axis(int c, int sd, int ng) {
  int g = c / sd;
  return g < ng ? g : ng - 1;
}
MSMG_HD int group_begin(int g, int sd) { return g * sd; }
MSMG_HD int group_end(int g, int sd, int ng, int nc) { return (g == ng - 1) ? nc : (g + 1) * sd; }

MSMG_HD long long node_id(const Geo& g, int i, int j, int k) {
  return ((long long)k * g.nny + j) * g.nnx + i;
}
MSMG_HD long long elem_id(const Geo& g, int i, int j, int k) {
  return ((long long)k * g.ny + j) * g.nx + i;
}

MSMG_DEV bool mask_bit(const uint32_t* bits, long long n) {
  return (bits[n >> 5] >> (n & 31)) & 1u;
}

// ---------------------------------------------------------------------------
// Node-gather form of y = A x for one node (i, j, k), in difference form:
//   y = sum_{o != 0} pattern(o) * (sum of k_e over elements holding both n and
//       n+o) * (x(n+o) - x(n))
// which equals (A x)_n because every row of an element matrix sums to zero.
// The difference form keeps the rounding error proportional to the local
// variation of x instead of its magnitude (T reaches ~1/k_min on low
// conductivity islands, where the plain sum cancels terms ~1e9 times larger
// than the result).  kk[c], c = cx + 2 cy + 4 cz, is the conductivity of the
// element with lower corner (i-1+cx, j-1+cy, k-1+cz) (0 outside the mesh).
// The functor xv(i,j,k) returns the neighbour value; it is called only for
// nodes inside the mesh.
template <typename W, bool CUBIC, typename F>
MSMG_DEV W gather_apply(const Geo& g, const Stencil& st, const W kk[8], int i, int j, int k, F xv) {
  const W fx0 = kk[0] + kk[2] + kk[4] + kk[6], fx1 = kk[1] + kk[3] + kk[5] + kk[7];
  const W fy0 = kk[0] + kk[1] + kk[4] + kk[5], fy1 = kk[2] + kk[3] + kk[6] + kk[7];
  const W fz0 = kk[0] + kk[1] + kk[2] + kk[3], fz1 = kk[4] + kk[5] + kk[6] + kk[7];
  const bool xm = i > 0, xp = i < g.nnx - 1;
  const bool ym = j > 0, yp = j < g.nny - 1;
  const bool zm = k > 0, zp = k < g.nnz - 1;
  const W x0 = xv(i, j, k);
  W acc = W(0);
  if (!CUBIC) {
    const W ax = W(st.ax[0]), ay = W(st.ax[1]), az = W(st.ax[2]);
    if (xm) acc += ax * fx0 * (xv(i - 1, j, k) - x0);
    if (xp) acc += ax * fx1 * (xv(i + 1, j, k) - x0);
    if (ym) acc += ay * fy0 * (xv(i, j - 1, k) - x0);
    if (yp) acc += ay * fy1 * (xv(i, j + 1, k) - x0);
    if (zm) acc += az * fz0 * (xv(i, j, k - 1) - x0);
    if (zp) acc += az * fz1 * (xv(i, j, k + 1) - x0);
  }
  // face diagonals in the xy plane (z unchanged): 2 elements each, pattern fd[2]
  {
    const W p = W(st.fd[2]);
    if (xm && ym) acc += p * (kk[0] + kk[4]) * (xv(i - 1, j - 1, k) - x0);
    if (xp && ym) acc += p * (kk[1] + kk[5]) * (xv(i + 1, j - 1, k) - x0);
    if (xm && yp) acc += p * (kk[2] + kk[6]) * (xv(i - 1, j + 1, k) - x0);
    if (xp && yp) acc += p * (kk[3] + kk[7]) * (xv(i + 1, j + 1, k) - x0);
  }
  // xz plane (y unchanged): pattern fd[1]
  {
    const W p = W(st.fd[1]);
    if (xm && zm) acc += p * (kk[0] + kk[2]) * (xv(i - 1, j, k - 1) - x0);
    if (xp && zm) acc += p * (kk[1] + kk[3]) * (xv(i + 1, j, k - 1) - x0);
    if (xm && zp) acc += p * (kk[4] + kk[6]) * (xv(i - 1, j, k + 1) - x0);
    if (xp && zp) acc += p * (kk[5] + kk[7]) * (xv(i + 1, j, k + 1) - x0);
  }
  // yz plane (x unchanged): pattern fd[0]
  {
    const W p = W(st.fd[0]);
    if (ym && zm) acc += p * (kk[0] + kk[1]) * (xv(i, j - 1, k - 1) - x0);
    if (yp && zm) acc += p * (kk[2] + kk[3]) * (xv(i, j + 1, k - 1) - x0);
    if (ym && zp) acc += p * (kk[4] + kk[5]) * (xv(i, j - 1, k + 1) - x0);
    if (yp && zp) acc += p * (kk[6] + kk[7]) * (xv(i, j + 1, k + 1) - x0);
  }
  // body diagonals: one element each
  {
    const W p = W(st.bd);
    if (xm && ym && zm) acc += p * kk[0] * (xv(i - 1, j - 1, k - 1) - x0);
    if (xp && ym && zm) acc += p * kk[1] * (xv(i + 1, j - 1, k - 1) - x0);
    if (xm && yp && zm) acc += p * kk[2] * (xv(i - 1, j + 1, k - 1) - x0);
    if (xp && yp && zm) acc += p * kk[3] * (xv(i + 1, j + 1, k - 1) - x0);
    if (xm && ym && zp) acc += p * kk[4] * (xv(i - 1, j - 1, k + 1) - x0);
    if (xp && ym && zp) acc += p * kk[5] * (xv(i + 1, j - 1, k + 1) - x0);
    if (xm && yp && zp) acc += p * kk[6] * (xv(i - 1, j + 1, k + 1) - x0);
    if (xp && yp && zp) acc += p * kk[7] * (xv(i + 1, j + 1, k + 1) - x0);
  }
  return acc;
}

// Conductivities of the 8 elements around node (i, j, k), 0 outside the mesh.
template <typename W, typename RT>
MSMG_DEV void load_k8(const Geo& g, const RT* rho, W kmin, W dk, int p, int i, int j, int k, W kk[8]) {
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int ei = i - 1 + (c & 1), ej = j - 1 + ((c >> 1) & 1), ek = k - 1 + ((c >> 2) & 1);
    const bool in = ei >= 0 && ei < g.nx && ej >= 0 && ej < g.ny && ek >= 0 && ek < g.nz;
    kk[c] = in ? conductivity<W>(ld<W, RT>(rho, elem_id(g, ei, ej, ek)), kmin, dk, p) : W(0);
  }
}

// ---------------------------------------------------------------------------
// Cell-aligned tiles: a tile covers CX coarse cells along x, one along y and
// one along z.  Thread (lx, ly) of the (CX*H) x H block owns the node column
// x = cx*H + lx%H, y = cy*H + ly over the cell's z range; the last lane/row of
// the last cell also takes the remainder nodes, so each thread's nodes lie in
// one coarse cell.
struct Tile {
  int cx, cy, cz;        // coarse cell of this thread (cx may be >= ncx: idle)
  int xs, xe, ys, ye, zs, ze;
  bool active;
};

MSMG_DEV Tile tile_of_thread(const Geo& g, const Hier& h, int CX, long long tile) {
  const int ntx = (h.ncx + CX - 1) / CX;
  const int tx = int(tile % ntx);
  const int ty = int((tile / ntx) % h.ncy);
  const int tz = int(tile / ((long long)ntx * h.ncy));
  Tile t;
  const int lx = threadIdx.x, ly = threadIdx.y;
  t.cx = tx * CX + lx / h.H;
  t.cy = ty;
  t.cz = tz;
  t.active = (t.cx < h.ncx) && (lx < CX * h.H) && (tz < h.ncz);
  const int ox = lx % h.H;
  t.xs = t.cx * h.H + ox;
  t.xe = (ox == h.H - 1 && t.cx == h.ncx - 1) ? g.nnx : t.xs + 1;
  t.ys = t.cy * h.H + ly;
  t.ye = (ly == h.H - 1 && t.cy == h.ncy - 1) ? g.nny : t.ys + 1;
  t.zs = t.cz * h.H;
  t.ze = (t.cz == h.ncz - 1) ? g.nnz : t.zs + h.H;
  return t;
}

// ---------------------------------------------------------------------------
// Launches over one or two right-hand sides (the batched state/adjoint pair):
// kernels that read the operator's coefficients take each per-side pointer as
// a Two<T> and run NS workgroups per tile.  The two sides' workgroups of a tile
// are 8 apart, so the hardware deals them to the same XCD and the second
// side's coefficient reads hit that XCD's L2.
template <typename T>
struct Two {
  T v[2];
  MSMG_HD T operator[](int i) const { return v[i]; }
};
template <typename T>
MSMG_HD Two<T> two(T a, T b) {
  Two<T> t;
  t.v[0] = a;
  t.v[1] = b;
  return t;
}
template <typename T>
MSMG_HD Two<T> one(T a) {
  return two(a, a);
}

struct SideBlock {
  int side;
  long long blk, nblk;  // the workgroup's index and count within its side
};
// NS = 2 needs a grid of a multiple of 16 workgroups.
template <int NS>
MSMG_DEV SideBlock side_block() {
  SideBlock r;
  if (NS == 1) {
    r.side = 0;
    r.blk = blockIdx.x;
    r.nblk = gridDim.x;
  } else {
    const long long b = blockIdx.x;
    r.side = int((b >> 3) & 1);
    r.blk = (b & 7) | ((b >> 4) << 3);
    r.nblk = gridDim.x / 2;
  }
  return r;
}

// XCD-aware remap: workgroups are dealt round-robin to the 8 XCDs; give each
// XCD a contiguous run of tiles so neighbouring tiles share one L2.  nblocks
// must be a multiple of 8 (then the map is a bijection of [0, nblocks)).
MSMG_DEV long long xcd_tile(long long bid, long long nblocks) {
  const long long per = (nblocks + 7) / 8;
  return (bid & 7) * per + (bid >> 3);
}

// ---------------------------------------------------------------------------
// Reductions (fixed order, so results are bitwise reproducible).
template <typename T>
MSMG_DEV T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum of NV values per thread; result valid in thread 0.  `red` must hold
// NV * (blockDim/64) entries.
template <int NV>
MSMG_DEV void block_sum(double (&v)[NV], double* red) {
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthreads = blockDim.x * blockDim.y * blockDim.z;
  const int lane = tid & 63, wid = tid >> 6, nw = (nthreads + 63) >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) red[q * nw + wid] = v[q];
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += red[q * nw + w];
      v[q] = s;
    }
  }
  __syncthreads();
}

// Device-resident PCG scalars.
struct Scalars {
  double rz;       // r^T z of the current iterate
  double pq;       // p^T A p
  double alpha, beta;
  double rr;       // ||r||^2 (recursive)
  double bb;       // ||b||^2
  double tol2;     // (rtol ||b||)^2
  double zr, zq;   // partial products of the last V-cycle
  double true_rr;  // ||b - A x||^2
  int done;        // 1: stop issuing work (converged / failed)
  int xpend;       // 1: x still lacks alpha p of the current step (the next direction update adds it)
  int status;      // see SolveStatus
  int iters;
  int maxit;
};

enum SolveStatus {
  ST_RUNNING = 0,
  ST_CONV_RECURSIVE = 1,
  ST_MAXIT = 2,
  ST_BREAKDOWN = 3,
  ST_NONFINITE = 4,
  ST_SYNC_TIMEOUT = 5  // a bounded device-side wait gave up (grid-synchronised coarse-level kernel)
};

// Cross-block deterministic reduction: each block publishes its partials, the
// last block to finish sums all partials in block order and runs `fin`.
//
// No memory fence is used: on a multi-XCD device a fence at agent scope writes
// back and invalidates the whole L2 of the XCD, which costs far more than the
// reduction when every block issues one.  Instead the partials are published
// with agent-scope atomic exchanges; the block waits for their results before
// taking a ticket from the counter, so every partial is in place at the
// coherence point before the last ticket is handed out, and the last block
// reads them back with agent-scope atomic loads.
template <int NV, typename Fin>
MSMG_DEV void grid_reduce(double (&v)[NV], double* red, double* partials, unsigned* counter,
                          int nblocks, int bid, Fin fin) {
  block_sum<NV>(v, red);
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  unsigned long long* P = reinterpret_cast<unsigned long long*>(partials);
  __shared__ int is_last;
  if (tid == 0) {
    unsigned long long seen = 0;
#pragma unroll
    for (int q = 0; q < NV; ++q)
      seen |= __hip_atomic_exchange(&P[(long long)q * nblocks + bid], (unsigned long long)__double_as_longlong(v[q]),
                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    asm volatile("" ::"v"(seen) : "memory");  // the exchanges have completed
    const unsigned ticket = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (ticket == unsigned(nblocks - 1));
  }
  __syncthreads();
  if (!is_last) return;
  const int nthreads = blockDim.x * blockDim.y * blockDim.z;
  // Each thread sums the partials b = tid, tid + nthreads, ... in that order;
  // they are fetched RB at a time so that RB loads are in flight (one at a time,
  // each waited for before the next, left the rest of the device idle for
  // tens of microseconds behind the last block).
  constexpr int RB = 16;
  double s[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    s[q] = 0.0;
    const unsigned long long* Pq = P + (long long)q * nblocks;
    for (int b0 = tid; b0 < nblocks; b0 += RB * nthreads) {
      double t[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int b = b0 + u * nthreads;
        t[u] = b < nblocks ? __longlong_as_double((long long)__hip_atomic_load(&Pq[b], __ATOMIC_RELAXED,
                                                                               __HIP_MEMORY_SCOPE_AGENT))
                           : 0.0;
      }
#pragma unroll
      for (int u = 0; u < RB; ++u)
        if (b0 + u * nthreads < nblocks) s[q] += t[u];
    }
  }
  block_sum<NV>(s, red);
  if (tid == 0) {
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    fin(s);
  }
}

}  // namespace msmg
