// 2.5D plane march for the fine-level stencil kernels.
//
// A workgroup of 64 x 8 threads owns a 64 x 8 column of nodes and marches over
// a chunk of z planes.  Each step stages one node plane (with a 1-node halo,
// 66 x 10 values) and one element plane (65 x 9 conductivities, computed from
// rho once per element) in LDS through coalesced loads; every thread keeps the
// 3 x 3 x 3 window of its node and the 8 surrounding conductivities in
// registers, so a step costs 9 + 4 LDS reads per node.  Two LDS buffers per
// plane type let one barrier per step suffice.
#pragma once

#include "common.h"

namespace msmg {

constexpr int MX = 64, MY = 8;                  // node tile
constexpr int PW = MX + 2, PH = MY + 2;         // node plane with halo
constexpr int EW = MX + 1, EH = MY + 1;         // element plane
constexpr int MARCH_THREADS = MX * MY;

struct March {
  int ntx, nty, nzc, zc;  // tiles along x, y; z chunks and their length
  long long blocks;       // ntx * nty * nzc rounded up to a multiple of 8
};

inline March make_march(const Geo& g, int target_blocks = 2048, int min_chunk = 16) {
  March m;
  m.ntx = (g.nnx + MX - 1) / MX;
  m.nty = (g.nny + MY - 1) / MY;
  const long long txy = (long long)m.ntx * m.nty;
  long long nzc = (target_blocks + txy - 1) / txy;
  if (nzc < 1) nzc = 1;
  int zc = int((g.nnz + nzc - 1) / nzc);
  if (zc < min_chunk) zc = min_chunk;
  if (zc > g.nnz) zc = g.nnz;
  m.zc = zc;
  m.nzc = (g.nnz + zc - 1) / zc;
  m.blocks = ((txy * m.nzc + 7) / 8) * 8;
  return m;
}

// LDS words (of type W) one marching workgroup needs
constexpr int march_lds_words() { return 2 * PW * PH + 2 * EW * EH; }

// loadn(n) -> value staged for node n; loadk(e) -> conductivity of element e;
// emit(i, j, k, n, Ax, xc) is called for every node of the tile inside the
// mesh with Ax = (A x)_n in difference form and xc the staged value at n.
template <typename W, bool CUBIC, typename LoadN, typename LoadK, typename Emit>
MSMG_DEV void march(const Geo& g, const Stencil& st, const March& mg, long long tile, W* sx, W* sk, LoadN loadn,
                    LoadK loadk, Emit emit) {
  const int tx = int(tile % mg.ntx), ty = int((tile / mg.ntx) % mg.nty), tz = int(tile / ((long long)mg.ntx * mg.nty));
  const int za = tz * mg.zc;
  if (tz >= mg.nzc || za >= g.nnz) return;  // uniform over the block
  const int zb = min(za + mg.zc, g.nnz);
  const int xa = tx * MX, ya = ty * MY;
  const int lx = threadIdx.x, ly = threadIdx.y, tid = lx + MX * ly;
  const int x = xa + lx, y = ya + ly;
  const bool inside = x < g.nnx && y < g.nny;

  // this thread's staging slots (fixed in x-y, the z offset changes per plane)
  constexpr int NS = (PW * PH + MARCH_THREADS - 1) / MARCH_THREADS;  // node slots per thread
  constexpr int ES = (EW * EH + MARCH_THREADS - 1) / MARCH_THREADS;  // element slots per thread
  const long long nplane = (long long)g.nnx * g.nny, eplane = (long long)g.nx * g.ny;
  long long nofs[NS], eofs[ES];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int q = tid + s * MARCH_THREADS;
    const int gx = xa - 1 + q % PW, gy = ya - 1 + q / PW;
    nofs[s] = (q < PW * PH && gx >= 0 && gx < g.nnx && gy >= 0 && gy < g.nny) ? (long long)gy * g.nnx + gx : -1;
  }
#pragma unroll
  for (int s = 0; s < ES; ++s) {
    const int q = tid + s * MARCH_THREADS;
    const int ex = xa - 1 + q % EW, ey = ya - 1 + q / EW;
    eofs[s] = (q < EW * EH && ex >= 0 && ex < g.nx && ey >= 0 && ey < g.ny) ? (long long)ey * g.nx + ex : -1;
  }
  // prefetch queue: DEPTH planes of loads stay in flight (each queue slot keeps
  // its registers, the step loop is unrolled by DEPTH)
  constexpr int DEPTH = sizeof(W) >= 8 ? 3 : 5;
  W pn[DEPTH][NS], pk[DEPTH][ES];
  auto load_nodes = [&](int d, int zz) {
    const bool zin = zz >= 0 && zz < g.nnz;
#pragma unroll
    for (int s = 0; s < NS; ++s) pn[d][s] = (zin && nofs[s] >= 0) ? loadn(nofs[s] + zz * nplane) : W(0);
  };
  auto load_elems = [&](int d, int ez) {
    const bool zin = ez >= 0 && ez < g.nz;
#pragma unroll
    for (int s = 0; s < ES; ++s) pk[d][s] = (zin && eofs[s] >= 0) ? loadk(eofs[s] + ez * eplane) : W(0);
  };
  auto store_nodes = [&](int d, int buf) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int q = tid + s * MARCH_THREADS;
      if (q < PW * PH) sx[buf * PW * PH + q] = pn[d][s];
    }
  };
  auto store_elems = [&](int d, int buf) {
#pragma unroll
    for (int s = 0; s < ES; ++s) {
      const int q = tid + s * MARCH_THREADS;
      if (q < EW * EH) sk[buf * EW * EH + q] = pk[d][s];
    }
  };
  W win[27];
  W kk[8];
  auto read_plane = [&](int buf, int p) {
    const W* src = sx + buf * PW * PH;
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) win[p * 9 + dy * 3 + dx] = src[(ly + dy) * PW + (lx + dx)];
  };
  auto read_k = [&](int buf, int layer) {
    const W* src = sk + buf * EW * EH;
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) kk[layer * 4 + cy * 2 + cx] = src[(ly + cy) * EW + (lx + cx)];
  };

  // prologue: planes za-1, za and element plane za-1
  load_nodes(0, za - 1);
  store_nodes(0, 0);
  load_nodes(0, za);
  store_nodes(0, 1);
  load_elems(0, za - 1);
  store_elems(0, 0);
  __syncthreads();
  read_plane(0, 0);
  read_plane(1, 1);
  read_k(0, 0);
  __syncthreads();
#pragma unroll
  for (int d = 0; d < DEPTH; ++d) {
    load_nodes(d, za + 1 + d);
    load_elems(d, za + d);
  }
  for (int z0 = za; z0 < zb; z0 += DEPTH) {
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
      const int z = z0 + d;
      if (z >= zb) break;  // uniform over the block
      const int buf = (z - za) & 1;
      store_nodes(d, buf);
      store_elems(d, buf);
      __syncthreads();
      // refill this queue slot; the other slots' loads are still in flight
      if (z + DEPTH < zb) {
        load_nodes(d, z + 1 + DEPTH);
        load_elems(d, z + DEPTH);
      }
      read_plane(buf, 2);
      read_k(buf, 1);
      if (inside) {
        const W ax = gather_apply<W, CUBIC>(g, st, kk, x, y, z, [&](int a, int b, int c) {
          return win[(c - z + 1) * 9 + (b - y + 1) * 3 + (a - x + 1)];
        });
        emit(x, y, z, node_id(g, x, y, z), ax, win[13]);
      }
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        win[q] = win[9 + q];
        win[9 + q] = win[18 + q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) kk[q] = kk[4 + q];
    }
  }
}

}  // namespace msmg
