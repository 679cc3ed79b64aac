// 2.5D plane march for the fine-level stencil kernels.
//
// A workgroup of MX x MY threads (64 x 4) owns an MX x MY column of nodes and
// marches over a chunk of z planes.  Each step stages one node plane (with a
// 1-node halo, (MX+2) x (MY+2) values) and one element layer ((MX+1) x (MY+1)
// conductivities) in LDS through coalesced loads.  The operator is split
// by element layer: the layer between planes z and z+1 contributes to the
// nodes of both planes, so a thread keeps only the 3 x 3 neighbourhood of its
// node in plane z and one carried partial sum; a step costs 9 + 4 LDS reads
// per node.  Two LDS buffers per plane type let one barrier per step suffice.
//
// Global loads are issued DEPTH steps ahead of their use into a register queue
// holding the raw stored values (the conversion to the working type happens
// when a slot is written to LDS), so no step waits on a load issued in the same
// step.  Per-node data the output needs (diagonal, right-hand side, mask word)
// is prefetched the same way.
#pragma once

#include <type_traits>
#include <utility>

#include "common.h"

#ifndef MSMG_MARCH_DEPTH8
#define MSMG_MARCH_DEPTH8 1
#endif
#ifndef MSMG_MARCH_DEPTH4
#define MSMG_MARCH_DEPTH4 2
#endif

namespace msmg {

#ifndef MSMG_MARCH_MX
#define MSMG_MARCH_MX 64
#endif
#ifndef MSMG_MARCH_MY
#define MSMG_MARCH_MY 4
#endif
#ifndef MSMG_MARCH_WAVES
#define MSMG_MARCH_WAVES 1
#endif

constexpr int MX = MSMG_MARCH_MX, MY = MSMG_MARCH_MY;  // node tile (a wave covers 64 / MX rows)
constexpr int PW = MX + 2, PH = MY + 2;                // node plane with halo
constexpr int EW = MX + 1, EH = MY + 1;                // element layer
constexpr int MARCH_THREADS = MX * MY;

// Kernel attributes of the marching kernels: the register budget is capped so
// that MSMG_MARCH_WAVES waves share each SIMD (several workgroups per CU at
// different phases of their march hide each other's memory waits).
#define MSMG_MARCH_KERNEL \
  __global__ __launch_bounds__(MARCH_THREADS) __attribute__((amdgpu_waves_per_eu(MSMG_MARCH_WAVES)))

struct March {
  int ntx, nty, nzc, zc;  // tiles along x, y; z chunks and their length
  long long blocks;       // ntx * nty * nzc rounded up to a multiple of 8
};

// Split the z range into chunks: every (x, y) tile column is cut into nzc
// chunks of zc planes.  `resident` is the number of marching workgroups the
// device runs at once; the chunk count minimises (rounds of resident
// workgroups) x (planes a workgroup stages, zc + 2 with the prologue).
inline March make_march(const Geo& g, long long resident = 2048, int min_chunk = 8, int mx = MX, int my = MY) {
  March m;
  m.ntx = (g.nnx + mx - 1) / mx;
  m.nty = (g.nny + my - 1) / my;
  const long long txy = (long long)m.ntx * m.nty;
  if (resident < 1) resident = 1;
  long long best_cost = -1;
  int best = 1;
  const int max_nzc = (g.nnz + min_chunk - 1) / min_chunk;
  for (int nzc = 1; nzc <= max_nzc; ++nzc) {
    const int zc = (g.nnz + nzc - 1) / nzc;
    const int used = (g.nnz + zc - 1) / zc;
    const long long rounds = (txy * used + resident - 1) / resident;
    const long long cost = rounds * (zc + 2);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = nzc;
    }
  }
  m.zc = (g.nnz + best - 1) / best;
  m.nzc = (g.nnz + m.zc - 1) / m.zc;
  m.blocks = ((txy * m.nzc + 7) / 8) * 8;
  return m;
}

// Contribution of one element layer to (A x)_n in difference form.  kq[c],
// c = cx + 2 cy, is the conductivity of the layer's element with lower corner
// (i-1+cx, j-1+cy) (0 outside the mesh); s is the 3 x 3 neighbourhood of the
// node in its own plane (s[4] = x_n, s[dy*3+dx] at offset (dx-1, dy-1)) and o
// the same neighbourhood in the layer's other plane.  Values outside the mesh
// are staged as 0 and meet a zero conductivity.
template <typename W, bool CUBIC>
MSMG_DEV W layer_apply(const Stencil& st, const W kq[4], const W s[9], const W o[9]) {
  const W x0 = s[4];
  W acc = W(st.fd[2]) * (kq[0] * (s[0] - x0) + kq[1] * (s[2] - x0) + kq[2] * (s[6] - x0) + kq[3] * (s[8] - x0));
  acc += W(st.fd[1]) * ((kq[0] + kq[2]) * (o[3] - x0) + (kq[1] + kq[3]) * (o[5] - x0));
  acc += W(st.fd[0]) * ((kq[0] + kq[1]) * (o[1] - x0) + (kq[2] + kq[3]) * (o[7] - x0));
  acc += W(st.bd) * (kq[0] * (o[0] - x0) + kq[1] * (o[2] - x0) + kq[2] * (o[6] - x0) + kq[3] * (o[8] - x0));
  if (!CUBIC) {
    acc += W(st.ax[0]) * ((kq[0] + kq[2]) * (s[3] - x0) + (kq[1] + kq[3]) * (s[5] - x0));
    acc += W(st.ax[1]) * ((kq[0] + kq[1]) * (s[1] - x0) + (kq[2] + kq[3]) * (s[7] - x0));
    acc += W(st.ax[2]) * ((kq[0] + kq[1] + kq[2] + kq[3]) * (o[4] - x0));
  }
  return acc;
}

// The same contribution as a plain sum sum_j a_nj x_j - (sum_j a_nj) x_n: the
// coefficient sum of a layer is (sum of its pattern weights) x (sum of kq), so
// about half the FP64 operations of the difference form.  Exact for the same
// linear operator; it differs from the difference form only by rounding (no
// cancellation of x_n inside each term), which the cycle, a preconditioner,
// does not need.
template <typename W, bool CUBIC>
MSMG_DEV W layer_apply_sum(const Stencil& st, const W kq[4], const W s[9], const W o[9]) {
  const W k02 = kq[0] + kq[2], k13 = kq[1] + kq[3], k01 = kq[0] + kq[1], k23 = kq[2] + kq[3];
  const W ksum = k01 + k23;
  W wsum = W(st.fd[2]) + W(st.fd[1]) + W(st.fd[0]) + W(st.bd);
  W acc = W(st.fd[2]) * (kq[0] * s[0] + kq[1] * s[2] + kq[2] * s[6] + kq[3] * s[8]);
  acc += W(st.fd[1]) * (k02 * o[3] + k13 * o[5]);
  acc += W(st.fd[0]) * (k01 * o[1] + k23 * o[7]);
  acc += W(st.bd) * (kq[0] * o[0] + kq[1] * o[2] + kq[2] * o[6] + kq[3] * o[8]);
  if (!CUBIC) {
    acc += W(st.ax[0]) * (k02 * s[3] + k13 * s[5]);
    acc += W(st.ax[1]) * (k01 * s[1] + k23 * s[7]);
    acc += W(st.ax[2]) * (ksum * o[4]);
    wsum += W(st.ax[0]) + W(st.ax[1]) + W(st.ax[2]);
  }
  return acc - (wsum * ksum) * s[4];
}

// The layer product of the cycle's marching kernels: the plain sum in FP64
// (MSMG_CYCLE_DIFFERENCE_FORM selects the difference form instead), the
// difference form for narrower types, whose rounding the cancellation would
// otherwise expose.
#ifndef MSMG_CYCLE_DIFFERENCE_FORM
#define MSMG_CYCLE_DIFFERENCE_FORM 0
#endif
template <typename W, bool CUBIC>
MSMG_DEV W cycle_layer(const Stencil& st, const W kq[4], const W s[9], const W o[9]) {
  if constexpr (MSMG_CYCLE_DIFFERENCE_FORM || sizeof(W) < 8) return layer_apply<W, CUBIC>(st, kq, s, o);
  else return layer_apply_sum<W, CUBIC>(st, kq, s, o);
}

// Element base + ofs of an array, with the plane base kept apart from the
// 32-bit in-plane offset.
template <typename T>
MSMG_DEV T plane_ld(const T* __restrict__ p, long long base, unsigned ofs) {
  return p[base + ofs];
}
template <typename T>
MSMG_DEV void plane_st(T* __restrict__ p, long long base, unsigned ofs, T v) {
  p[base + ofs] = v;
}

template <typename W>
constexpr int march_depth() {
  return sizeof(W) >= 8 ? MSMG_MARCH_DEPTH8 : MSMG_MARCH_DEPTH4;
}

// Nodes and elements are addressed as (plane base index, offset in the plane):
// loadn(b, o) -> raw stored value(s) of node b + o, convn(raw) -> staged value;
// loadk(b, o) -> raw value(s) of element b + o, convk(raw) -> conductivity;
// loadc(b, o) -> per-node data for the output of node b + o (prefetched);
// emit(b, o, Ax, xc, c) is called for every node of the tile inside the mesh
// with Ax = (A x)_n in difference form, xc the staged value at n and c the data
// loadc returned for n.
//
// Every load is issued unconditionally at a clamped in-mesh address (slots
// outside the mesh stage 0 when written to LDS) and the step loop has a fixed
// shape, so the compiler can count the loads in flight exactly and waits only
// for the queue slot a step consumes.
//
// after(z, za, zb) runs at the end of every step, in every thread of the
// workgroup (also for the padding steps past zb), after the step's emits: the
// place for work that needs the whole workgroup, such as a block reduction.
// The z chunk of workgroup tz is [tz * zc, tz * zc + zc), the last one up to
// the last plane (it may be longer than zc).
//
// loadn may also take (b, o, s, zz): the thread's staging slot s (node
// (x, y) = march_slot_xy(tile, s), clamped into the mesh) and the plane zz
// (clamped), for node data that depends on where the node lies; convn may
// take (raw, s).  Slot s of plane zz is converted before slot s of the next
// plane is loaded when the queue is one step deep.
template <int S>
MSMG_DEV void march_slot_xy(const Geo& g, const March& mg, long long tile, int& gx, int& gy) {
  const int tx = int(tile % mg.ntx), ty = int((tile / mg.ntx) % mg.nty);
  const int tid = threadIdx.x + MX * threadIdx.y;
  const int q = tid + S * MARCH_THREADS;
  gx = min(max(tx * MX - 1 + q % PW, 0), g.nnx - 1);
  gy = min(max(ty * MY - 1 + q / PW, 0), g.nny - 1);
}
constexpr int MARCH_NODE_SLOTS = (PW * PH + MARCH_THREADS - 1) / MARCH_THREADS;

template <typename LoadN>
MSMG_DEV auto march_loadn(LoadN& loadn, long long base, unsigned ofs, int s, int zz) {
  if constexpr (std::is_invocable_v<LoadN&, long long, unsigned, int, int>) return loadn(base, ofs, s, zz);
  else return loadn(base, ofs);
}
// convn may likewise take (raw, s)
template <typename ConvN, typename RN>
MSMG_DEV auto march_convn(ConvN& convn, const RN& raw, int s) {
  if constexpr (std::is_invocable_v<ConvN&, const RN&, int>) return convn(raw, s);
  else return convn(raw);
}

template <typename W, bool CUBIC, typename LoadN, typename ConvN, typename LoadK, typename ConvK, typename LoadC,
          typename Emit, typename After>
MSMG_DEV void march_ex(const Geo& g, const Stencil& st, const March& mg, long long tile, W* sx, W* sk, LoadN loadn,
                       ConvN convn, LoadK loadk, ConvK convk, LoadC loadc, Emit emit, After after) {
  using RN = decltype(march_loadn(loadn, 0LL, 0u, 0, 0));
  using RK = decltype(loadk(0LL, 0u));
  using CD = decltype(loadc(0LL, 0u));
  constexpr int DEPTH = march_depth<W>();
  const int tx = int(tile % mg.ntx), ty = int((tile / mg.ntx) % mg.nty), tz = int(tile / ((long long)mg.ntx * mg.nty));
  const int za = tz * mg.zc;
  if (tz >= mg.nzc || za >= g.nnz) return;  // uniform over the block
  const int zb = (tz == mg.nzc - 1) ? g.nnz : min(za + mg.zc, g.nnz);
  const int xa = tx * MX, ya = ty * MY;
  const int lx = threadIdx.x, ly = threadIdx.y, tid = lx + MX * ly;
  const int x = xa + lx, y = ya + ly;
  const bool inside = x < g.nnx && y < g.nny;

  // this thread's staging slots (fixed in x-y, the z offset changes per plane)
  constexpr int NS = (PW * PH + MARCH_THREADS - 1) / MARCH_THREADS;  // node slots per thread
  constexpr int ES = (EW * EH + MARCH_THREADS - 1) / MARCH_THREADS;  // element slots per thread
  const long long nplane = (long long)g.nnx * g.nny, eplane = (long long)g.nx * g.ny;
  unsigned nofs[NS], eofs[ES];
  unsigned nvalid = 0, evalid = 0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int q = tid + s * MARCH_THREADS;
    const int gx = xa - 1 + q % PW, gy = ya - 1 + q / PW;
    if (q < PW * PH && gx >= 0 && gx < g.nnx && gy >= 0 && gy < g.nny) nvalid |= 1u << s;
    nofs[s] = unsigned(min(max(gy, 0), g.nny - 1) * g.nnx + min(max(gx, 0), g.nnx - 1));
  }
#pragma unroll
  for (int s = 0; s < ES; ++s) {
    const int q = tid + s * MARCH_THREADS;
    const int ex = xa - 1 + q % EW, ey = ya - 1 + q / EW;
    if (q < EW * EH && ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny) evalid |= 1u << s;
    eofs[s] = unsigned(min(max(ey, 0), g.ny - 1) * g.nx + min(max(ex, 0), g.nx - 1));
  }
  const unsigned cxy = unsigned(min(y, g.nny - 1) * g.nnx + min(x, g.nnx - 1));

  RN pn[DEPTH][NS];
  RK pk[DEPTH][ES];
  CD pc[DEPTH];
  auto load_nodes = [&](int d, int zz) {
    const int zc = min(max(zz, 0), g.nnz - 1);
    const long long base = (long long)zc * nplane;
#pragma unroll
    for (int s = 0; s < NS; ++s) pn[d][s] = march_loadn(loadn, base, nofs[s], s, zc);
  };
  auto load_elems = [&](int d, int ez) {
    const long long base = (long long)min(max(ez, 0), g.nz - 1) * eplane;
#pragma unroll
    for (int s = 0; s < ES; ++s) pk[d][s] = loadk(base, eofs[s]);
  };
  auto load_centre = [&](int d, int zz) { pc[d] = loadc((long long)min(zz, g.nnz - 1) * nplane, cxy); };
  auto store_nodes = [&](int d, int buf, int zz) {
    const bool zin = zz >= 0 && zz < g.nnz;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int q = tid + s * MARCH_THREADS;
      const W v = march_convn(convn, pn[d][s], s);
      if (q < PW * PH) sx[buf * PW * PH + q] = (zin && ((nvalid >> s) & 1u)) ? v : W(0);
    }
  };
  auto store_elems = [&](int d, int buf, int ez) {
    const bool zin = ez >= 0 && ez < g.nz;
#pragma unroll
    for (int s = 0; s < ES; ++s) {
      const int q = tid + s * MARCH_THREADS;
      const W v = convk(pk[d][s]);
      if (q < EW * EH) sk[buf * EW * EH + q] = (zin && ((evalid >> s) & 1u)) ? v : W(0);
    }
  };
  auto read_plane = [&](int buf, W* dst) {
    const W* src = sx + buf * PW * PH;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) dst[dy * 3 + dx] = src[(ly + dy) * PW + (lx + dx)];
  };
  auto read_k = [&](int buf, W* kq) {
    const W* src = sk + buf * EW * EH;
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) kq[cy * 2 + cx] = src[(ly + cy) * EW + (lx + cx)];
  };

  // prologue: planes za-1 and za, element layer za-1 -> the partial sum of
  // node za from the layer below
  W A[9], carry;
  {
    load_nodes(0, za - 1);
    store_nodes(0, 0, za - 1);
    load_nodes(0, za);
    store_nodes(0, 1, za);
    load_elems(0, za - 1);
    store_elems(0, 0, za - 1);
    __syncthreads();
    W P[9], kq[4];
    read_plane(0, P);
    read_plane(1, A);
    read_k(0, kq);
    carry = cycle_layer<W, CUBIC>(st, kq, A, P);
    __syncthreads();
  }
#pragma unroll
  for (int d = 0; d < DEPTH; ++d) {
    load_nodes(d, za + 1 + d);
    load_elems(d, za + d);
    load_centre(d, za + d);
  }
  // whole rounds of DEPTH steps; steps past zb stage clamped planes and emit nothing
  const int zend = za + (zb - za + DEPTH - 1) / DEPTH * DEPTH;
  for (int z0 = za; z0 < zend; z0 += DEPTH) {
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
      const int z = z0 + d;
      const int buf = (z - za) & 1;
      store_nodes(d, buf, z + 1);
      store_elems(d, buf, z);
      const CD cur = pc[d];
      __syncthreads();
      // refill this queue slot; the other slots' loads are still in flight
      load_nodes(d, z + 1 + DEPTH);
      load_elems(d, z + DEPTH);
      load_centre(d, z + DEPTH);
      W B[9], kq[4];
      read_plane(buf, B);
      read_k(buf, kq);
      const W ax = carry + cycle_layer<W, CUBIC>(st, kq, A, B);
      if (inside && z < zb) emit((long long)z * nplane, cxy, ax, A[4], cur);
      carry = cycle_layer<W, CUBIC>(st, kq, B, A);
#pragma unroll
      for (int q = 0; q < 9; ++q) A[q] = B[q];
      after(z, za, zb);
    }
  }
}

template <typename W, bool CUBIC, typename LoadN, typename ConvN, typename LoadK, typename ConvK, typename LoadC,
          typename Emit>
MSMG_DEV void march(const Geo& g, const Stencil& st, const March& mg, long long tile, W* sx, W* sk, LoadN loadn,
                    ConvN convn, LoadK loadk, ConvK convk, LoadC loadc, Emit emit) {
  march_ex<W, CUBIC>(g, st, mg, tile, sx, sk, loadn, convn, loadk, convk, loadc, emit, [](int, int, int) {});
}


// ---------------------------------------------------------------------------
// Plane march with its prefetch queue in LDS (FP64 node and element arrays).
//
// gfx950's global-to-LDS loads (global_load_lds_dword) write the 64 dwords of a
// wave straight into LDS, so LDS_DEPTH bundles (node plane z+1 with halo,
// element layer z) are in flight per workgroup without holding registers.
// Bundles rotate through LDS_NB = LDS_DEPTH + 1 buffers, each its own LDS
// array so that the compiler can tell a read of one buffer from the loads
// still landing in the others.  A step waits until at most the loads issued
// for the LDS_DEPTH - 1 younger bundles are outstanding (vector-memory loads
// complete in issue order), one barrier then publishes the bundle to all
// waves, and the buffer read in the previous step is refilled.  Every load
// instruction runs with all lanes active (spare lanes fetch a valid address
// into padding), so the count of memory instructions per step is fixed.
// Slots outside the mesh fetch clamped, finite values; their element
// conductivities are zeroed when read, which removes their terms.
// three bundles in flight measured fastest (four and five were slower: the
// march at three waves per SIMD is then bound by its FP64 arithmetic)
constexpr int LDS_DEPTH = 3, LDS_NB = LDS_DEPTH + 1;
// its own tile shape (a wave is any 64 consecutive threads of the tile)
#ifndef MSMG_LDS_MX
#define MSMG_LDS_MX 32
#endif
constexpr int LMX = MSMG_LDS_MX, LMY = MARCH_THREADS / LMX;
constexpr int LPW = LMX + 2, LPH = LMY + 2, LEW = LMX + 1, LEH = LMY + 1;
static_assert(LMX * LMY == MARCH_THREADS && MARCH_THREADS % 64 == 0, "whole waves");

// LDS buffer of one bundle for element type KT.  A load instruction moves one
// 4-byte slot per lane (a 2-byte load lands zero-extended in the low half of
// its lane's slot): FP64 values take two lanes, FP32 and BF16 one.
template <typename KT>
struct LdsLayout {
  static constexpr int KB = sizeof(KT) >= 4 ? 4 : int(sizeof(KT));  // bytes one lane loads
  static constexpr int KL = int(sizeof(KT)) / KB;                     // lanes per element
  static constexpr int NI = (2 * LPW * LPH + MARCH_THREADS - 1) / MARCH_THREADS;  // node-plane loads
  static constexpr int EI = (KL * LEW * LEH + MARCH_THREADS - 1) / MARCH_THREADS;  // element-layer loads
  static constexpr int INSTR = NI + EI;
  static constexpr int ELEM0 = NI * MARCH_THREADS * 4;               // byte offset of the elements
  static constexpr int BUF_D = (ELEM0 + EI * MARCH_THREADS * 4) / 8;  // doubles per buffer
  // loads of the LDS_DEPTH - 1 younger bundles (the per-step centre loads
  // are not counted, so the wait holds however many a step issues)
  static constexpr int WAIT = (LDS_DEPTH - 1) * INSTR;
  static_assert(WAIT < 64, "vmcnt holds 6 bits");
};

typedef __attribute__((address_space(3))) void* lds_void_ptr;
typedef __attribute__((address_space(1))) void* glb_void_ptr;
typedef const __attribute__((address_space(1))) char* glb_char_ptr;

template <int N>
MSMG_DEV void wait_vm(void) {
  // s_waitcnt with vmcnt = N, expcnt and lgkmcnt left open
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}
MSMG_DEV void wait_vm0(void) { __builtin_amdgcn_s_waitcnt(0 | (0x7 << 4) | (0xF << 8)); }
// barrier without a memory fence (the fence would drain every LDS load in
// flight); the empty asm keeps the compiler from moving memory operations
// across it
MSMG_DEV void lds_barrier(void) {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int J>
struct StepIdx {
  static constexpr int value = J;
};

// f(StepIdx<J>) for J = 0, 1, ... in order (the buffer index of a step is a
// compile-time constant)
template <typename F, int... J>
MSMG_DEV void for_each_step(F&& f, std::integer_sequence<int, J...>) {
  (f(StepIdx<J>{}), ...);
}

// Staged nodes are FP64 (x), elements KT (an element array, turned into the
// FP64 conductivity by convk when read: a stored conductivity or the density
// through the material law).  loadc(b, o) -> per-node data of node b + o
// (register queue, LDS_NB slots); emit as in march().  bufs: the LDS_NB
// buffers of LdsLayout<KT>::BUF_D doubles, each a separate LDS array.
template <bool CUBIC, typename KT, typename ConvK, typename LoadC, typename Emit>
MSMG_DEV void march_lds(const Geo& g, const Stencil& st, const March& mg, long long tile, double* const* bufs,
                        const double* __restrict__ x, const KT* __restrict__ kc, ConvK convk, LoadC loadc,
                        Emit emit) {
  using LY = LdsLayout<KT>;
  constexpr int NI = LY::NI, INSTR = LY::INSTR, KL = LY::KL, KB = LY::KB, ELEM0 = LY::ELEM0;
  using CD = decltype(loadc(0LL, 0u));
  const int tx = int(tile % mg.ntx), ty = int((tile / mg.ntx) % mg.nty), tz = int(tile / ((long long)mg.ntx * mg.nty));
  const int za = tz * mg.zc;
  if (tz >= mg.nzc || za >= g.nnz) return;  // uniform over the block
  const int zb = (tz == mg.nzc - 1) ? g.nnz : min(za + mg.zc, g.nnz);
  const int xa = tx * LMX, ya = ty * LMY;
  const int lx = threadIdx.x, ly = threadIdx.y, tid = lx + LMX * ly;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int x0 = xa + lx, y0 = ya + ly;
  const bool inside = x0 < g.nnx && y0 < g.nny;
  const long long nplane = (long long)g.nnx * g.nny, eplane = (long long)g.nx * g.ny;
  const unsigned cxy = unsigned(min(y0, g.nny - 1) * g.nnx + min(x0, g.nnx - 1));

  // byte offset inside its plane of this lane's dword of each load
  // instruction (padding lanes re-read the plane's first dword)
  unsigned inpl[INSTR];
#pragma unroll
  for (int i = 0; i < INSTR; ++i) {
    const int dw = ((i < NI ? i : i - NI) * (MARCH_THREADS / 64) + wave) * 64 + lane;
    unsigned off = 0;
    if (i < NI) {
      const int q = dw >> 1;
      if (q < LPW * LPH) {
        const int gx = min(max(xa - 1 + q % LPW, 0), g.nnx - 1), gy = min(max(ya - 1 + q / LPW, 0), g.nny - 1);
        off = unsigned(gy * g.nnx + gx) * 8u + unsigned(dw & 1) * 4u;
      }
    } else {
      const int q = dw / KL;
      if (q < LEW * LEH) {
        const int ex = min(max(xa - 1 + q % LEW, 0), g.nx - 1), ey = min(max(ya - 1 + q / LEW, 0), g.ny - 1);
        off = unsigned(ey * g.nx + ex) * unsigned(sizeof(KT)) + unsigned(dw % KL) * unsigned(KB);
      }
    }
    inpl[i] = off;
  }
  // in-plane validity of the four elements around this thread's node
  bool ev[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int ex = x0 - 1 + (c & 1), ey = y0 - 1 + (c >> 1);
    ev[c] = ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny;
  }

  // uniform plane base + 32-bit lane offset: the loads take the scalar-base form
  const glb_char_ptr xg = (glb_char_ptr)x, kg = (glb_char_ptr)kc;
  auto issue = [&](double* buf, int z) {
    const glb_char_ptr nb = xg + (long long)min(max(z + 1, 0), g.nnz - 1) * nplane * 8;
    const glb_char_ptr eb = kg + (long long)min(max(z, 0), g.nz - 1) * eplane * (long long)sizeof(KT);
    char* dst = reinterpret_cast<char*>(buf) + wave * 256;
#pragma unroll
    for (int i = 0; i < INSTR; ++i) {
      if (i < NI)
        __builtin_amdgcn_global_load_lds((glb_void_ptr)(nb + inpl[i]), (lds_void_ptr)(dst + i * MARCH_THREADS * 4), 4,
                                         0, 0);
      else
        __builtin_amdgcn_global_load_lds((glb_void_ptr)(eb + inpl[i]), (lds_void_ptr)(dst + i * MARCH_THREADS * 4), LdsLayout<KT>::KB,
                                         0, 0);
    }
  };
  // conductivity of element slot e of a buffer's element region
  auto kval = [&](const double* buf, int e) -> double {
    const char* p = reinterpret_cast<const char*>(buf) + ELEM0;
    if constexpr (sizeof(KT) == 8) {
      return convk(*reinterpret_cast<const KT*>(p + 8 * e));
    } else if constexpr (sizeof(KT) == 4) {
      return convk(*reinterpret_cast<const KT*>(p + 4 * e));
    } else {
      KT v;
      __builtin_memcpy(&v, p + 4 * e, sizeof(KT));
      return convk(v);
    }
  };
  auto read_plane = [&](const double* src, double* dst) {
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) dst[dy * 3 + dx] = src[(ly + dy) * LPW + (lx + dx)];
  };
  auto read_k = [&](const double* buf, bool zin, double* kq) {
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) {
        const double v = kval(buf, (ly + cy) * LEW + (lx + cx));
        kq[cy * 2 + cx] = (zin && ev[cy * 2 + cx]) ? v : 0.0;
      }
  };
  CD pc[LDS_NB];
#pragma unroll
  for (int d = 0; d < LDS_DEPTH; ++d) {
    issue(bufs[d], za + d);
    pc[d] = loadc((long long)min(za + d, g.nnz - 1) * nplane, cxy);
  }

  // prologue in the buffer the first bundles leave free: planes za-1 and za,
  // element layer za-1 -> the partial sum of node za from the layer below
  double A[9], carry;
  {
    double* pb = bufs[LDS_NB - 1];
    auto stage_nodes = [&](int zz) {
      const bool zin = zz >= 0 && zz < g.nnz;
      const long long base = (long long)min(max(zz, 0), g.nnz - 1) * nplane;
      for (int q = tid; q < LPW * LPH; q += MARCH_THREADS) {
        const int gx = xa - 1 + q % LPW, gy = ya - 1 + q / LPW;
        const bool ok = zin && gx >= 0 && gx < g.nnx && gy >= 0 && gy < g.nny;
        pb[q] = ok ? x[base + (long long)gy * g.nnx + gx] : 0.0;
      }
    };
    stage_nodes(za - 1);
    {
      const int ez = za - 1;
      const bool zin = ez >= 0 && ez < g.nz;
      const long long base = (long long)min(max(ez, 0), g.nz - 1) * eplane;
      char* pe = reinterpret_cast<char*>(pb) + ELEM0;
      for (int q = tid; q < LEW * LEH; q += MARCH_THREADS) {
        const int ex = xa - 1 + q % LEW, ey = ya - 1 + q / LEW;
        const bool ok = zin && ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny;
        KT v;
        __builtin_memset(&v, 0, sizeof(KT));
        if (ok) v = kc[base + (long long)ey * g.nx + ex];
        __builtin_memcpy(pe + (sizeof(KT) == 8 ? 8 : 4) * q, &v, sizeof(KT));
      }
    }
    __syncthreads();
    double P[9], kq[4];
    read_plane(pb, P);
    read_k(pb, za - 1 >= 0, kq);  // the layer below the mesh has no elements
    __syncthreads();
    stage_nodes(za);
    __syncthreads();
    read_plane(pb, A);
    carry = layer_apply<double, CUBIC>(st, kq, A, P);
  }

  auto step = [&](auto jc, int z) {
    constexpr int j = decltype(jc)::value;
    constexpr int jn = (j + LDS_DEPTH) % LDS_NB;
    wait_vm<LY::WAIT>();
    lds_barrier();
    // refill the buffer read in the previous step
    issue(bufs[jn], z + LDS_DEPTH);
    pc[jn] = loadc((long long)min(z + LDS_DEPTH, g.nnz - 1) * nplane, cxy);
    const double* buf = bufs[j];
    double B[9], kq[4];
    read_plane(buf, B);
    read_k(buf, z < g.nz, kq);
    const double ax = carry + layer_apply<double, CUBIC>(st, kq, A, B);
    if (inside && z < zb) emit((long long)z * nplane, cxy, ax, A[4], pc[j]);
    carry = layer_apply<double, CUBIC>(st, kq, B, A);
#pragma unroll
    for (int q = 0; q < 9; ++q) A[q] = B[q];
  };
  const int zend = za + (zb - za + LDS_NB - 1) / LDS_NB * LDS_NB;
  for (int z0 = za; z0 < zend; z0 += LDS_NB)
    for_each_step([&](auto jc) { step(jc, z0 + decltype(jc)::value); }, std::make_integer_sequence<int, LDS_NB>{});
  // no load may still be writing this workgroup's LDS when it ends
  wait_vm0();
}

}  // namespace msmg
