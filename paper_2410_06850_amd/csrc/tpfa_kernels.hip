// Cell-centred two-point flux finite volumes (paper section 2.2): the operator
// of eq. (new linear system) with the harmonic face conductivities of eq.
// (flux), and the level-0 kernels of Algorithm 1 on cell unknowns.
//
// Unknown K = (z ny + y) nx + x, one per cell.  For the face between K and its
// neighbour L along axis d, T_F = w_d * 2 k_K k_L / (k_K + k_L) with
// w_d = |F| / h_d (the harmonic mean of eq. (flux) times the face's area over
// the centre distance).  A Dirichlet face of K (a boundary face flagged in the
// cell's byte: bit 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z) adds 2 w_d k_K to the
// diagonal (the half-cell distance) and that times T_D to the right-hand
// side.  Products with A are taken in difference form,
//   (A x)_K = sum_F T_F (x_K - x_L) + wd_K x_K,
// so that the rounding follows the local variation of x.
//
// The stencil kernels march a 64 x 4 column tile of threads through a z range
// of cells, each thread one (x, y) column; the x and k values of the cells
// below, at and above the current one stay in registers, the four in-plane
// neighbours come through the caches (staging the planes in LDS measured
// slower: the barrier per plane exposes the load latency).
#include "internal.h"
#include "setup.h"

namespace msmg {

namespace {

constexpr int TX = 64, TY = 4;
// workgroups of one stencil launch at most (the reducing launches publish one
// partial per workgroup; the handle keeps at least this many slots)
constexpr long long TILE_BUDGET = 8192;

struct TGeo {
  int nx, ny, nz;
  long long n;
  double w[3];   // |F| / h_d
  int ntx, nty, ntz, zc;
  long long tiles;
};

TGeo tgeo(const Ctx& c) {
  TGeo t;
  t.nx = c.g.nx;
  t.ny = c.g.ny;
  t.nz = c.g.nz;
  t.n = c.g.ne;
  t.w[0] = c.g.hy * c.g.hz / c.g.hx;
  t.w[1] = c.g.hx * c.g.hz / c.g.hy;
  t.w[2] = c.g.hx * c.g.hy / c.g.hz;
  t.ntx = (t.nx + TX - 1) / TX;
  t.nty = (t.ny + TY - 1) / TY;
  // z chunks of about 8 cells, as many as the workgroup budget allows
  // (grids are padded to multiples of 8 for the XCD remap)
  const long long cols = (long long)t.ntx * t.nty;
  const long long want = (t.nz + 7) / 8;
  long long nzt = std::max<long long>(1, std::min<long long>(want, (TILE_BUDGET - 8) / std::max<long long>(cols, 1)));
  t.zc = int((t.nz + nzt - 1) / nzt);
  t.ntz = (t.nz + t.zc - 1) / t.zc;
  t.tiles = cols * t.ntz;
  return t;
}

unsigned tgrid(const TGeo& t) { return unsigned(((t.tiles + 7) / 8) * 8); }

MSMG_DEV double face_T(double w, double a, double b) { return w * (2.0 * a * b / (a + b)); }

// Dirichlet diagonal of a cell: sum over its flagged faces of 2 w_d k_K
MSMG_DEV double dir_w(const TGeo& t, unsigned f, double kc) {
  double s = 0.0;
  if (f & 3u) s += double(((f >> 0) & 1u) + ((f >> 1) & 1u)) * (2.0 * t.w[0] * kc);
  if (f & 12u) s += double(((f >> 2) & 1u) + ((f >> 3) & 1u)) * (2.0 * t.w[1] * kc);
  if (f & 48u) s += double(((f >> 4) & 1u) + ((f >> 5) & 1u)) * (2.0 * t.w[2] * kc);
  return s;
}

struct ColumnTile {
  int i, j, z0, z1;
  bool active;  // the thread's column lies in the mesh (and the tile is real)
  bool tile;    // the workgroup's tile is real (not grid padding)
};

MSMG_DEV ColumnTile column_tile(const TGeo& t) {
  const long long tile = xcd_tile(blockIdx.x, gridDim.x);
  ColumnTile c;
  const int tx = int(tile % t.ntx), ty = int((tile / t.ntx) % t.nty);
  const long long tz = tile / ((long long)t.ntx * t.nty);
  c.i = tx * TX + int(threadIdx.x);
  c.j = ty * TY + int(threadIdx.y);
  c.z0 = int(tz) * t.zc;
  c.z1 = min(c.z0 + t.zc, t.nz);
  c.tile = tile < t.tiles;
  c.active = c.tile && c.i < t.nx && c.j < t.ny;
  return c;
}

// A double from the neighbouring lane of the wave: lane i receives lane i - 1's
// value (PREV) or lane i + 1's (!PREV), by two DPP whole-wave shifts of the
// 32-bit halves; the lane at the end of the shift receives 0.
template <bool PREV>
MSMG_DEV double wave_shift(double v) {
  constexpr int ctrl = PREV ? 0x138 : 0x130;  // wave_shr:1, wave_shl:1
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b), ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), ctrl, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Marches the thread's column and calls body(n, kc, vc, acc) with
// acc = (A v)_n, where v_m = V(m) is any per-cell value (a vector, or a
// product of vectors formed on the fly).  Absent neighbours take the cell's
// own k and value, so their terms vanish without a branch.  A wave is one
// 64-cell x-row of the tile: the x-neighbours' k and v are the adjacent
// lanes' centre values (wave shifts), and only the two end lanes load theirs
// (one load per quantity, the other lanes re-reading their own cell).  The
// loads of the next z step (the two y-neighbours, the x-row ends, its flags
// and the cell two planes up) are issued before the current step's
// arithmetic, so that two steps' loads are in flight per thread.
// ALL: every thread of a real tile marches (columns outside the mesh on the
// clamped last column or row) and body gets the column's `active` flag as a
// fifth argument, so that wave-wide steps inside body see every lane.
template <bool ALL = false, typename VF, typename Body>
MSMG_DEV void tpfa_march(const TGeo& t, const ColumnTile& c, const double* __restrict__ k,
                         const uint8_t* __restrict__ df, VF V, Body body) {
  static_assert(TX == 64, "a wave is one x-row of the tile");
  if (ALL ? !c.tile : !c.active) return;
  const long long sx = 1, sy = t.nx, sz = (long long)t.nx * t.ny;
  const int ci = min(c.i, t.nx - 1), cj = min(c.j, t.ny - 1);
  const int lane = int(threadIdx.x);
  const bool xp = ci + 1 < t.nx, ym = cj > 0, yp = cj + 1 < t.ny;
  const long long oxm = ci > 0 ? -sx : 0, oxp = xp ? sx : 0, oym = ym ? -sy : 0, oyp = yp ? sy : 0;
  // the end lanes' x-neighbour (the lane's own cell for the others)
  const long long oe = lane == 0 ? oxm : (lane == TX - 1 ? oxp : 0);
  struct Ring {
    double kym, kyp, vym, vyp, ke, ve;
    unsigned f;
  };
  auto ring = [&](long long m) {
    Ring r;
    r.kym = k[m + oym];
    r.kyp = k[m + oyp];
    r.vym = V(m + oym);
    r.vyp = V(m + oyp);
    r.ke = k[m + oe];
    r.ve = V(m + oe);
    r.f = df[m];
    return r;
  };
  long long n = (long long)cj * sy + ci + (long long)c.z0 * sz;
  double kc = k[n], vc = V(n);
  double km = kc, vm = vc, kp = kc, vp = vc;
  if (c.z0 > 0) {
    km = k[n - sz];
    vm = V(n - sz);
  }
  if (c.z0 + 1 < t.nz) {
    kp = k[n + sz];
    vp = V(n + sz);
  }
  Ring cur = ring(n);
  for (int z = c.z0; z < c.z1; ++z, n += sz) {
    Ring nxt = cur;
    double kpp = kp, vpp = vp;
    if (z + 1 < c.z1) {
      nxt = ring(n + sz);
      if (z + 2 < t.nz) {
        kpp = k[n + 2 * sz];
        vpp = V(n + 2 * sz);
      }
    }
    const double kls = wave_shift<true>(kc), vls = wave_shift<true>(vc);
    const double krs = wave_shift<false>(kc), vrs = wave_shift<false>(vc);
    const double kxm = lane == 0 ? cur.ke : kls, vxm = lane == 0 ? cur.ve : vls;
    const double kxp = lane == TX - 1 ? cur.ke : (xp ? krs : kc);
    const double vxp = lane == TX - 1 ? cur.ve : (xp ? vrs : vc);
    double acc = dir_w(t, cur.f, kc) * vc;
    acc += face_T(t.w[0], kc, kxm) * (vc - vxm);
    acc += face_T(t.w[0], kc, kxp) * (vc - vxp);
    acc += face_T(t.w[1], kc, cur.kym) * (vc - cur.vym);
    acc += face_T(t.w[1], kc, cur.kyp) * (vc - cur.vyp);
    acc += face_T(t.w[2], kc, km) * (vc - vm);
    acc += face_T(t.w[2], kc, kp) * (vc - vp);
    if constexpr (ALL) body(n, kc, vc, acc, c.active);
    else body(n, kc, vc, acc);
    km = kc;
    vm = vc;
    kc = kp;
    vc = vp;
    kp = kpp;
    vp = vpp;
    cur = nxt;
  }
}

// q = A p; MODE 1 also reduces p^T q and sets alpha = rz / p^T q (the PCG step)
template <int MODE>
__global__ __launch_bounds__(TX* TY) void k_tpfa_apply(TGeo t, const double* __restrict__ k,
                                                      const uint8_t* __restrict__ df, const double* __restrict__ x,
                                                      double* __restrict__ y, Scalars* sc, double* partials,
                                                      unsigned* counter) {
  if (MODE == 1 && sc->done) return;
  __shared__ double red[16];
  double s[1] = {0.0};
  const ColumnTile c = column_tile(t);
  tpfa_march(t, c, k, df, [&](long long m) { return x[m]; }, [&](long long n, double, double vc, double acc) {
    y[n] = acc;
    if (MODE == 1) s[0] += vc * acc;
  });
  if (MODE != 1) return;
  grid_reduce<1>(s, red, partials, counter, gridDim.x, blockIdx.x, [&](double* tt) {
    sc->pq = tt[0];
    sc->xpend = 0;
    if (!(tt[0] > 0.0) || !(sc->rz > 0.0)) {
      sc->status = (tt[0] == tt[0] && sc->rz == sc->rz) ? ST_BREAKDOWN : ST_NONFINITE;
      sc->done = 1;
    } else {
      sc->alpha = sc->rz / tt[0];
    }
  });
}

// y = b - A (x + xlo) with the differences of both parts taken separately;
// ||y||^2 -> true_rr when sc is given
__global__ __launch_bounds__(TX* TY) void k_tpfa_residual(TGeo t, const double* __restrict__ k,
                                                         const uint8_t* __restrict__ df, const double* __restrict__ b,
                                                         const double* __restrict__ x, const float* __restrict__ xlo,
                                                         double* __restrict__ y, Scalars* sc, double* partials,
                                                         unsigned* counter) {
  __shared__ double red[16];
  double s[1] = {0.0};
  const ColumnTile c = column_tile(t);
  if (c.active) {
    const long long sy = t.nx, sz = (long long)t.nx * t.ny;
    for (int z = c.z0; z < c.z1; ++z) {
      const long long n = (long long)z * sz + (long long)c.j * sy + c.i;
      const double kc = k[n];
      long long nb[6];
      bool in[6];
      in[0] = c.i > 0; nb[0] = n - 1;
      in[1] = c.i + 1 < t.nx; nb[1] = n + 1;
      in[2] = c.j > 0; nb[2] = n - sy;
      in[3] = c.j + 1 < t.ny; nb[3] = n + sy;
      in[4] = z > 0; nb[4] = n - sz;
      in[5] = z + 1 < t.nz; nb[5] = n + sz;
      const double xc = x[n], lc = xlo ? double(xlo[n]) : 0.0;
      const double wd = dir_w(t, df[n], kc);
      double ahi = wd * xc, alo = wd * lc;
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        if (!in[f]) continue;
        const double T = face_T(t.w[f / 2], kc, k[nb[f]]);
        ahi += T * (xc - x[nb[f]]);
        if (xlo) alo += T * (lc - double(xlo[nb[f]]));
      }
      const double out = (b[n] - ahi) - alo;
      y[n] = out;
      s[0] += out * out;
    }
  }
  if (!sc) return;
  grid_reduce<1>(s, red, partials, counter, gridDim.x, blockIdx.x, [&](double* tt) { sc->true_rr = tt[0]; });
}

// out = r - A x (the cycle's residuals)
__global__ __launch_bounds__(TX* TY) void k_tpfa_vresidual(TGeo t, const double* __restrict__ k,
                                                          const uint8_t* __restrict__ df, const double* __restrict__ r,
                                                          const double* __restrict__ x, double* __restrict__ out,
                                                          const Scalars* sc) {
  if (sc && sc->done) return;
  const ColumnTile c = column_tile(t);
  tpfa_march(t, c, k, df, [&](long long m) { return x[m]; },
             [&](long long n, double, double, double acc) { out[n] = r[n] - acc; });
}

// The cycle's first residual fused with the restriction: rc = R_c (r - A x)
// without storing the residual.  Needs H | nx, ny, nz, H dividing the 64-lane
// x-row of a wave, and z chunks of whole coarse cells (tgeo_restrict).  Each
// thread sums R_c(n) (r - A x)_n over its column within a coarse cell; at
// the cell's last plane the H lanes of each coarse x-cell add their sums
// (xor shuffles) and the first writes one partial per (coarse cell, row j):
// part[((cz ny + j) ncx + cx) L + l].  k_tpfa_restrict_finish adds the H rows.
template <int L, int HH>
__global__ __launch_bounds__(TX* TY) void k_tpfa_vresidual_restrict(TGeo t, Hier h, const double* __restrict__ k,
                                                                   const uint8_t* __restrict__ df,
                                                                   const double* __restrict__ r,
                                                                   const double* __restrict__ x,
                                                                   const double* __restrict__ R,
                                                                   double* __restrict__ part, const Scalars* sc) {
  static_assert(TX == 64 && 64 % HH == 0, "a wave's x-row holds whole coarse cells");
  if (sc && sc->done) return;
  const ColumnTile c = column_tile(t);
  const long long sz = (long long)t.nx * t.ny;
  double a[L];
#pragma unroll
  for (int l = 0; l < L; ++l) a[l] = 0.0;
  tpfa_march<true>(t, c, k, df, [&](long long m) { return x[m]; },
                   [&](long long n, double, double, double acc, bool act) {
                     const int z = int(n / sz);
                     if (act) {
                       const double v = r[n] - acc;
#pragma unroll
                       for (int l = 0; l < L; ++l) a[l] += R[n * L + l] * v;
                     }
                     if ((z + 1) % HH == 0 || z + 1 == c.z1) {
#pragma unroll
                       for (int l = 0; l < L; ++l) {
                         double sum = a[l];
#pragma unroll
                         for (int off = 1; off < HH; off <<= 1) sum += __shfl_xor(sum, off, 64);
                         a[l] = sum;
                       }
                       if (act && c.i % HH == 0) {
                         const long long o = (((long long)(z / HH) * t.ny + c.j) * h.ncx + c.i / HH) * L;
#pragma unroll
                         for (int l = 0; l < L; ++l) part[o + l] = a[l];
                       }
#pragma unroll
                       for (int l = 0; l < L; ++l) a[l] = 0.0;
                     }
                   });
}

template <int L>
__global__ void k_tpfa_restrict_finish(TGeo t, Hier h, const double* __restrict__ part, double* __restrict__ rc,
                                       const Scalars* sc) {
  if (sc && sc->done) return;
  const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (q >= (long long)h.ncells * L) return;
  const int cell = int(q / L), l = int(q % L);
  const int cx = cell % h.ncx, cy = (cell / h.ncx) % h.ncy, cz = cell / (h.ncx * h.ncy);
  double s = 0.0;
  for (int j = cy * h.H; j < (cy + 1) * h.H; ++j) s += part[(((long long)cz * t.ny + j) * h.ncx + cx) * L + l];
  rc[q] = s;
}

// Chebyshev-Jacobi smoother on D^-1 A from a zero guess (the three-term
// recurrence of the Q1 path): x1 = d1 = D^-1 r / theta, then
// d_{s+1} = a_s d_s + b_s D^-1 (r - A x_s), x_{s+1} = x_s + d_{s+1}.
__global__ void k_tpfa_cheb_first(const double* __restrict__ r, const double* __restrict__ dinv,
                                  double* __restrict__ x, double* __restrict__ d, long long n, double inv_theta,
                                  const Scalars* sc) {
  if (sc && sc->done) return;
  for (long long m = blockIdx.x * (long long)blockDim.x + threadIdx.x; m < n; m += (long long)gridDim.x * blockDim.x) {
    const double v = r[m] * dinv[m] * inv_theta;
    x[m] = v;
    if (d) d[m] = v;
  }
}

// the first two steps fused: x1 = D^-1 r / theta formed for the neighbours on
// the fly, out = c0 x1 + c1 D^-1 (r - A x1); dout = out - x1 when given
__global__ __launch_bounds__(TX* TY) void k_tpfa_cheb2(TGeo t, const double* __restrict__ k,
                                                      const uint8_t* __restrict__ df, const double* __restrict__ r,
                                                      const double* __restrict__ dinv, double* __restrict__ out,
                                                      double* __restrict__ dout, double inv_theta, double c0,
                                                      double c1, const Scalars* sc) {
  if (sc && sc->done) return;
  const ColumnTile c = column_tile(t);
  tpfa_march(t, c, k, df, [&](long long m) { return r[m] * dinv[m] * inv_theta; },
             [&](long long n, double, double x1, double acc) {
               const double v = c0 * x1 + c1 * (dinv[n] * (r[n] - acc));
               out[n] = v;
               if (dout) dout[n] = v - x1;
             });
}

__global__ __launch_bounds__(TX* TY) void k_tpfa_cheb_step(TGeo t, const double* __restrict__ k,
                                                          const uint8_t* __restrict__ df,
                                                          const double* __restrict__ r, const double* __restrict__ dinv,
                                                          const double* __restrict__ x, double* __restrict__ d,
                                                          double* __restrict__ xout, double a, double b,
                                                          const Scalars* sc) {
  if (sc && sc->done) return;
  const ColumnTile c = column_tile(t);
  tpfa_march(t, c, k, df, [&](long long m) { return x[m]; }, [&](long long n, double, double xc, double acc) {
    const double dn = a * d[n] + b * (dinv[n] * (r[n] - acc));
    d[n] = dn;
    xout[n] = xc + dn;
  });
}

// The post-smoother fused with the cycle's output: the two Chebyshev steps of
// k_tpfa_cheb2 applied to `res`, then z = base + s with the PCG products
// z^T r (MODE 0, 1) and z^T q (MODE 1) reduced as the separate output kernel
// does (MODE 2: none).  s stays in registers; z is the value the separate
// smoother and output kernels compute.
template <int MODE>
__global__ __launch_bounds__(TX* TY) void k_tpfa_cheb2_out(TGeo t, const double* __restrict__ k,
                                                          const uint8_t* __restrict__ df,
                                                          const double* __restrict__ res,
                                                          const double* __restrict__ dinv, double inv_theta,
                                                          double c0, double c1, const double* __restrict__ base,
                                                          double* __restrict__ z, const double* __restrict__ r,
                                                          const double* __restrict__ q, Scalars* sc, double* partials,
                                                          unsigned* counter) {
  if (sc->done) return;
  __shared__ double red[32];
  double s[2] = {0.0, 0.0};
  const ColumnTile c = column_tile(t);
  tpfa_march(t, c, k, df, [&](long long m) { return res[m] * dinv[m] * inv_theta; },
             [&](long long n, double, double x1, double acc) {
               const double v = c0 * x1 + c1 * (dinv[n] * (res[n] - acc));
               const double zn = base[n] + v;
               z[n] = zn;
               if (MODE != 2) s[0] += zn * r[n];
               if (MODE == 1) s[1] += zn * q[n];
             });
  if (MODE == 2) return;
  grid_reduce<2>(s, red, partials, counter, gridDim.x, blockIdx.x, [&](double* tt) { vc_finish(sc, tt, MODE); });
}

// Jacobi diagonal inverse: 1 / (sum of the face transmissibilities + the Dirichlet part)
__global__ __launch_bounds__(TX* TY) void k_tpfa_diag_inv(TGeo t, const double* __restrict__ k,
                                                         const uint8_t* __restrict__ df, double* __restrict__ dinv) {
  const ColumnTile c = column_tile(t);
  // A applied to the unit vector of the cell itself: the diagonal is the
  // cell's row with every neighbour value zero
  if (!c.active) return;
  const long long sy = t.nx, sz = (long long)t.nx * t.ny;
  for (int z = c.z0; z < c.z1; ++z) {
    const long long n = (long long)z * sz + (long long)c.j * sy + c.i;
    const double kc = k[n];
    double d = dir_w(t, df[n], kc);
    if (c.i > 0) d += face_T(t.w[0], kc, k[n - 1]);
    if (c.i + 1 < t.nx) d += face_T(t.w[0], kc, k[n + 1]);
    if (c.j > 0) d += face_T(t.w[1], kc, k[n - sy]);
    if (c.j + 1 < t.ny) d += face_T(t.w[1], kc, k[n + sy]);
    if (z > 0) d += face_T(t.w[2], kc, k[n - sz]);
    if (z + 1 < t.nz) d += face_T(t.w[2], kc, k[n + sz]);
    dinv[n] = 1.0 / d;
  }
}

// b = f + wd_K T_D(K) (td per cell; null: b = f)
__global__ void k_tpfa_lift(TGeo t, const double* __restrict__ k, const uint8_t* __restrict__ df,
                            const double* __restrict__ f, const double* __restrict__ td, double* __restrict__ b) {
  for (long long m = blockIdx.x * (long long)blockDim.x + threadIdx.x; m < t.n; m += (long long)gridDim.x * blockDim.x) {
    double v = f[m];
    if (td) {
      const unsigned fl = df[m];
      if (fl) v += dir_w(t, fl, k[m]) * td[m];
    }
    b[m] = v;
  }
}

// copy the caller's face flags; counts[0] = flagged faces, counts[1] = flags
// on faces that are not on the domain boundary (or outside bits 0..5)
__global__ void k_tpfa_flags(TGeo t, const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                             unsigned long long* counts) {
  unsigned long long good = 0, bad = 0;
  for (long long m = blockIdx.x * (long long)blockDim.x + threadIdx.x; m < t.n; m += (long long)gridDim.x * blockDim.x) {
    const unsigned f = in[m];
    out[m] = uint8_t(f);
    if (!f) continue;
    const int i = int(m % t.nx), j = int((m / t.nx) % t.ny), z = int(m / ((long long)t.nx * t.ny));
    unsigned allowed = 0;
    if (i == 0) allowed |= 1u;
    if (i == t.nx - 1) allowed |= 2u;
    if (j == 0) allowed |= 4u;
    if (j == t.ny - 1) allowed |= 8u;
    if (z == 0) allowed |= 16u;
    if (z == t.nz - 1) allowed |= 32u;
    good += __popc(f & allowed);
    bad += __popc(f & ~allowed);
  }
  good = wave_sum(good);
  bad = wave_sum(bad);
  if ((threadIdx.x & 63) == 0) {
    if (good) atomicAdd(counts, good);
    if (bad) atomicAdd(counts + 1, bad);
  }
}

// load of a cell-wise constant source: f_K = s_K |K|
__global__ void k_tpfa_cell_load(long long n, const double* __restrict__ src, double sconst, double vol,
                                 double* __restrict__ f) {
  for (long long m = blockIdx.x * (long long)blockDim.x + threadIdx.x; m < n; m += (long long)gridDim.x * blockDim.x)
    f[m] = (src ? src[m] : sconst) * vol;
}

// heat source of eq. (material) integrated over each cell: f0 (1 - rho^p) |K|
template <typename RT>
__global__ void k_tpfa_heat_source_load(long long n, const RT* __restrict__ rho, int p, double f0, double vol,
                                        double* __restrict__ f) {
  for (long long m = blockIdx.x * (long long)blockDim.x + threadIdx.x; m < n; m += (long long)gridDim.x * blockDim.x) {
    const double r = double(rho[m]);
    double rp = r;
    for (int q = 1; q < p; ++q) rp *= r;
    f[m] = f0 * (1.0 - rp) * vol;
  }
}

// Design sensitivities (section 2.3) on the TPFA operator:
//   dc/drho_K = lam^T (db/drho_K - dA/drho_K t)
// with, per internal face F = (K, L), dT_F/dk_K = w_d 2 k_L^2 / (k_K + k_L)^2
// times -(lam_K - lam_L)(t_K - t_L), per Dirichlet face 2 w_d lam_K (T_D - t_K),
// all times dk/drho = p rho^(p-1) (k_max - k_min); SOURCE adds the heat
// source's lam_K (-f0 p rho^(p-1)) |K|.  lam null: lam = t (the compliance
// with zero Dirichlet values); td null: T_D = 0.
template <typename RT, bool SOURCE>
__global__ void k_tpfa_sensitivity(TGeo t, const RT* __restrict__ rho, Material mat, const double* __restrict__ T,
                                   const double* __restrict__ lam, const uint8_t* __restrict__ df,
                                   const double* __restrict__ td, double f0, double vol, double* __restrict__ dc) {
  const double dk = mat.kmax - mat.kmin;
  const long long sy = t.nx, sz = (long long)t.nx * t.ny;
  for (long long m = blockIdx.x * (long long)blockDim.x + threadIdx.x; m < t.n; m += (long long)gridDim.x * blockDim.x) {
    const int i = int(m % t.nx), j = int((m / t.nx) % t.ny), z = int(m / sz);
    const double r = double(rho[m]);
    const double kc = conductivity<double>(r, mat.kmin, dk, mat.p);
    const double tc = T[m], lc = lam ? lam[m] : tc;
    const bool in[6] = {i > 0, i + 1 < t.nx, j > 0, j + 1 < t.ny, z > 0, z + 1 < t.nz};
    const long long st[6] = {-1, 1, -sy, sy, -sz, sz};
    double g = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      if (!in[f]) continue;
      const long long q = m + st[f];
      const double kn = conductivity<double>(double(rho[q]), mat.kmin, dk, mat.p);
      const double s = kc + kn;
      const double dT = t.w[f / 2] * (2.0 * kn * kn / (s * s));
      const double ln = lam ? lam[q] : T[q];
      g -= dT * ((lc - ln) * (tc - T[q]));
    }
    const unsigned fl = df[m];
    if (fl) {
      const double tdv = td ? td[m] : 0.0;
#pragma unroll
      for (int f = 0; f < 6; ++f)
        if ((fl >> f) & 1u) g += 2.0 * t.w[f / 2] * lc * (tdv - tc);
    }
    double rp1 = 1.0;
    for (int q = 1; q < mat.p; ++q) rp1 *= r;
    g *= double(mat.p) * rp1 * dk;
    if (SOURCE) g += lc * (-f0 * double(mat.p) * rp1) * vol;
    dc[m] = g;
  }
}

// rc = R_c v: one workgroup per coarse cell sums its cells in a fixed order
template <int L>
__global__ __launch_bounds__(256) void k_tpfa_restrict(TGeo t, Hier h, const double* __restrict__ v,
                                                      const double* __restrict__ R, double* __restrict__ rc,
                                                      const Scalars* sc) {
  if (sc && sc->done) return;
  __shared__ double red[L * 4];
  const int cell = blockIdx.x;
  const int cx = cell % h.ncx, cy = (cell / h.ncx) % h.ncy, cz = cell / (h.ncx * h.ncy);
  const int x0 = cell_begin(cx, h.H), x1 = cell_end(cx, h.H, h.ncx, t.nx);
  const int y0 = cell_begin(cy, h.H), y1 = cell_end(cy, h.H, h.ncy, t.ny);
  const int z0 = cell_begin(cz, h.H), z1 = cell_end(cz, h.H, h.ncz, t.nz);
  const int lx = x1 - x0, ly = y1 - y0, nl = lx * ly * (z1 - z0);
  double acc[L];
#pragma unroll
  for (int l = 0; l < L; ++l) acc[l] = 0.0;
  for (int q = threadIdx.x; q < nl; q += blockDim.x) {
    const int a = q % lx, b = (q / lx) % ly, cc = q / (lx * ly);
    const long long n = ((long long)(z0 + cc) * t.ny + (y0 + b)) * t.nx + (x0 + a);
    const double vn = v[n];
#pragma unroll
    for (int l = 0; l < L; ++l) acc[l] += R[n * L + l] * vn;
  }
  block_sum<L>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int l = 0; l < L; ++l) rc[(long long)cell * L + l] = acc[l];
  }
}

// out = base + R_c^T (e1 + e2) (e2 may be null)
template <int L>
__global__ void k_tpfa_prolong(TGeo t, Hier h, const double* __restrict__ base, const double* __restrict__ R,
                               const double* __restrict__ e1, const double* __restrict__ e2,
                               double* __restrict__ out, const Scalars* sc) {
  if (sc && sc->done) return;
  for (long long m = blockIdx.x * (long long)blockDim.x + threadIdx.x; m < t.n; m += (long long)gridDim.x * blockDim.x) {
    const int i = int(m % t.nx), j = int((m / t.nx) % t.ny), z = int(m / ((long long)t.nx * t.ny));
    const long long cell = ((long long)owner_axis(z, h.H, h.ncz) * h.ncy + owner_axis(j, h.H, h.ncy)) * h.ncx +
                           owner_axis(i, h.H, h.ncx);
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const double e = e1[cell * L + l] + (e2 ? e2[cell * L + l] : 0.0);
      s += R[m * L + l] * e;
    }
    out[m] = base[m] + s;
  }
}

// Galerkin blocks A_c = R_c A R_c^T (drop_cc = 0) or the coarse-coarse form
// R_c K^cc R_c^T (drop_cc = 1: only the faces whose two cells share a
// coarse-coarse cell, no Dirichlet part), in the 27-block layout of the
// coarse levels ([cell][27][L][L], block (oz+1) 9 + (oy+1) 3 + (ox+1)).  One
// wave per (cell, block): the self block and the six face blocks are summed
// over the cell's (boundary) cells in a fixed order, the other twenty are
// zero (TPFA couples face neighbours only).
template <typename BT, int L>
__global__ __launch_bounds__(256) void k_tpfa_galerkin(TGeo t, Hier h, const double* __restrict__ k,
                                                      const uint8_t* __restrict__ df, const BT* __restrict__ R,
                                                      int drop_cc, double* __restrict__ out) {
  const long long wave = (long long)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (wave >= (long long)h.ncells * 27) return;
  const int cell = int(wave / 27), blk = int(wave % 27);
  const int ox = blk % 3 - 1, oy = (blk / 3) % 3 - 1, oz = blk / 9 - 1;
  double* o = out + ((long long)cell * 27 + blk) * L * L;
  const int nd = (ox != 0) + (oy != 0) + (oz != 0);
  const int cx = cell % h.ncx, cy = (cell / h.ncx) % h.ncy, cz = cell / (h.ncx * h.ncy);
  const int jx = cx + ox, jy = cy + oy, jz = cz + oz;
  const bool exists = jx >= 0 && jx < h.ncx && jy >= 0 && jy < h.ncy && jz >= 0 && jz < h.ncz;
  if (nd > 1 || !exists) {
    for (int e = lane; e < L * L; e += 64) o[e] = 0.0;
    return;
  }
  const int x0 = cell_begin(cx, h.H), x1 = cell_end(cx, h.H, h.ncx, t.nx);
  const int y0 = cell_begin(cy, h.H), y1 = cell_end(cy, h.H, h.ncy, t.ny);
  const int z0 = cell_begin(cz, h.H), z1 = cell_end(cz, h.H, h.ncz, t.nz);
  const int ax = ox != 0 ? 0 : (oy != 0 ? 1 : 2);  // axis of a face block
  const int side = ox + oy + oz;                  // -1 / +1 (0 for the self block)
  // the cells of this coarse cell that take part: all of them for the self
  // block, the boundary layer towards the neighbour for a face block
  int bx0 = x0, bx1 = x1, by0 = y0, by1 = y1, bz0 = z0, bz1 = z1;
  if (nd == 1) {
    if (ax == 0) { if (side > 0) bx0 = x1 - 1; else bx1 = x0 + 1; }
    if (ax == 1) { if (side > 0) by0 = y1 - 1; else by1 = y0 + 1; }
    if (ax == 2) { if (side > 0) bz0 = z1 - 1; else bz1 = z0 + 1; }
  }
  const int lx = bx1 - bx0, ly = by1 - by0, nl = lx * ly * (bz1 - bz0);
  const long long st[3] = {1, t.nx, (long long)t.nx * t.ny};
  const int nax[3] = {t.nx, t.ny, t.nz};
  // is the face between fine cells at coordinates p and p+1 along axis a
  // inside one coarse-coarse cell?
  const int ncs[3] = {h.ncx, h.ncy, h.ncz}, ngs[3] = {h.nccx, h.nccy, h.nccz};
  auto same_cc = [&](int a, int p) {
    const int g0 = group_axis(owner_axis(p, h.H, ncs[a]), h.sd, ngs[a]);
    const int g1 = group_axis(owner_axis(p + 1, h.H, ncs[a]), h.sd, ngs[a]);
    return g0 == g1;
  };
  double acc[L][L];
#pragma unroll
  for (int a = 0; a < L; ++a)
#pragma unroll
    for (int b = 0; b < L; ++b) acc[a][b] = 0.0;
  for (int q = lane; q < nl; q += 64) {
    const int pc[3] = {bx0 + q % lx, by0 + (q / lx) % ly, bz0 + q / (lx * ly)};
    const long long n = (pc[2] * (long long)t.ny + pc[1]) * t.nx + pc[0];
    const double kc = k[n];
    double ra[L];
#pragma unroll
    for (int a = 0; a < L; ++a) ra[a] = ld<double, BT>(R, n * L + a);
    if (nd == 1) {
      // the face towards the neighbour coarse cell: -T_F R_I(n) R_J(m)^T
      const long long m = n + side * st[ax];
      const int plo = side > 0 ? pc[ax] : pc[ax] - 1;
      if (drop_cc && !same_cc(ax, plo)) continue;
      const double T = face_T(t.w[ax], kc, k[m]);
#pragma unroll
      for (int b = 0; b < L; ++b) {
        const double rb = ld<double, BT>(R, m * L + b);
#pragma unroll
        for (int a = 0; a < L; ++a) acc[a][b] -= T * ra[a] * rb;
      }
    } else {
      // (A phi_I^b)(n) over the faces of n: the diagonal part from every face
      // (a neighbour outside the coarse cell only adds to it), the coupling
      // part from neighbours inside the coarse cell
      double diag = drop_cc ? 0.0 : dir_w(t, df[n], kc);
      double Ab[L];
#pragma unroll
      for (int b = 0; b < L; ++b) Ab[b] = 0.0;
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const int a = f / 2, sd = (f & 1) ? 1 : -1;
        const int p = pc[a] + sd;
        if (p < 0 || p >= nax[a]) continue;
        if (drop_cc && !same_cc(a, sd > 0 ? pc[a] : p)) continue;
        const long long m = n + sd * st[a];
        const double T = face_T(t.w[a], kc, k[m]);
        diag += T;
        const int lo = a == 0 ? x0 : (a == 1 ? y0 : z0), hi = a == 0 ? x1 : (a == 1 ? y1 : z1);
        if (p >= lo && p < hi) {
#pragma unroll
          for (int b = 0; b < L; ++b) Ab[b] -= T * ld<double, BT>(R, m * L + b);
        }
      }
#pragma unroll
      for (int b = 0; b < L; ++b) Ab[b] += diag * ld<double, BT>(R, n * L + b);
#pragma unroll
      for (int a = 0; a < L; ++a)
#pragma unroll
        for (int b = 0; b < L; ++b) acc[a][b] += ra[a] * Ab[b];
    }
  }
#pragma unroll
  for (int a = 0; a < L; ++a)
#pragma unroll
    for (int b = 0; b < L; ++b) {
      const double v = wave_sum(acc[a][b]);
      if (lane == 0) o[a * L + b] = v;
    }
}

#define TL_DISPATCH(Lrt, ...)                                 \
  do {                                                        \
    switch (Lrt) {                                            \
      case 1: { constexpr int LL = 1; __VA_ARGS__; } break;   \
      case 2: { constexpr int LL = 2; __VA_ARGS__; } break;   \
      case 3: { constexpr int LL = 3; __VA_ARGS__; } break;   \
      case 4: { constexpr int LL = 4; __VA_ARGS__; } break;   \
      case 5: { constexpr int LL = 5; __VA_ARGS__; } break;   \
      case 6: { constexpr int LL = 6; __VA_ARGS__; } break;   \
      case 7: { constexpr int LL = 7; __VA_ARGS__; } break;   \
      default: { constexpr int LL = 8; __VA_ARGS__; } break;  \
    }                                                         \
  } while (0)
static_assert(LC_MAX == 8, "TL_DISPATCH covers 1 .. 8");

}  // namespace

// ---------------------------------------------------------------------------
// launchers

bool tpfa_grid_fits(const Ctx& c) {
  const TGeo t = tgeo(c);
  return (long long)tgrid(t) <= TILE_BUDGET;
}

void launch_tpfa_apply(const Ctx& c, const double* x, double* y, bool reduce, hipStream_t s) {
  const TGeo t = tgeo(c);
  if (reduce)
    hipLaunchKernelGGL((k_tpfa_apply<1>), dim3(tgrid(t)), dim3(TX, TY), 0, s, t, c.kc, c.dface, x, y, c.sc, c.partials,
                       c.counter);
  else
    hipLaunchKernelGGL((k_tpfa_apply<0>), dim3(tgrid(t)), dim3(TX, TY), 0, s, t, c.kc, c.dface, x, y, c.sc, c.partials,
                       c.counter);
}

void launch_tpfa_residual(const Ctx& c, const double* b, const double* x, const float* xlo, double* y, bool reduce,
                          hipStream_t s) {
  const TGeo t = tgeo(c);
  hipLaunchKernelGGL(k_tpfa_residual, dim3(tgrid(t)), dim3(TX, TY), 0, s, t, c.kc, c.dface, b, x, xlo, y,
                     reduce ? c.sc : nullptr, c.partials, c.counter);
}

void launch_tpfa_vresidual(const Ctx& c, const double* r, const double* x, double* out, hipStream_t s) {
  const TGeo t = tgeo(c);
  hipLaunchKernelGGL(k_tpfa_vresidual, dim3(tgrid(t)), dim3(TX, TY), 0, s, t, c.kc, c.dface, r, x, out,
                     (const Scalars*)c.sc);
}

bool tpfa_restrict_fusable(const Ctx& c) {
  const int H = c.h.H;
  return (H == 4 || H == 8 || H == 16) && c.g.nx % H == 0 && c.g.ny % H == 0 && c.g.nz % H == 0;
}

long long tpfa_restrict_slots(const Ctx& c) { return (long long)c.g.nz / c.h.H * c.g.ny * c.h.ncx; }

void launch_tpfa_vresidual_restrict(const Ctx& c, const double* r, const double* x, double* part, double* rc,
                                    hipStream_t s) {
  TGeo t = tgeo(c);
  // z chunks of whole coarse cells
  const int H = c.h.H;
  t.zc = ((t.zc + H - 1) / H) * H;
  t.ntz = (t.nz + t.zc - 1) / t.zc;
  t.tiles = (long long)t.ntx * t.nty * t.ntz;
  const long long n = (long long)c.h.ncells * c.h.Lc;
#define VRR(HH) TL_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_tpfa_vresidual_restrict<LL, HH>), dim3(tgrid(t)), dim3(TX, TY), 0, s, t, c.h, c.kc, c.dface, r, x, (const double*)c.Rc, part, (const Scalars*)c.sc))
  if (H == 4) VRR(4); else if (H == 8) VRR(8); else VRR(16);
#undef VRR
  TL_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_tpfa_restrict_finish<LL>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                                         s, t, c.h, (const double*)part, rc, (const Scalars*)c.sc));
}

void launch_tpfa_smooth(const Ctx& c, const double* in, double* out, hipStream_t s) {
  const TGeo t = tgeo(c);
  const int deg = c.cheb.degree;
  const double* dinv = (const double*)c.dinv;
  const Scalars* sc = c.sc;
  if (deg == 1) {
    hipLaunchKernelGGL(k_tpfa_cheb_first, dim3(grid1d(t.n, 256, 8192)), dim3(256), 0, s, in, dinv, out,
                       (double*)nullptr, t.n, c.cheb.inv_theta, sc);
    return;
  }
  // first two steps fused; further steps ping-pong between out and t1 so that
  // the last one lands in out
  double* d = deg > 2 ? (double*)c.vc_t0 : nullptr;
  double* xa = (deg % 2 == 0) ? out : (double*)c.vc_t1;
  double* xb = (xa == out) ? (double*)c.vc_t1 : out;
  hipLaunchKernelGGL(k_tpfa_cheb2, dim3(tgrid(t)), dim3(TX, TY), 0, s, t, c.kc, c.dface, in, dinv, xa, d,
                     c.cheb.inv_theta, c.cheb.c0, c.cheb.c1, sc);
  for (int step = 2; step < deg; ++step) {
    hipLaunchKernelGGL(k_tpfa_cheb_step, dim3(tgrid(t)), dim3(TX, TY), 0, s, t, c.kc, c.dface, in, dinv, xa, d, xb,
                       c.cheb.step_a[step], c.cheb.step_b[step], sc);
    double* tmp = xa;
    xa = xb;
    xb = tmp;
  }
}

void launch_tpfa_smooth_output(const Ctx& c, const double* res, const double* base, double* z, const double* r,
                               const double* q, int mode, hipStream_t s) {
  const TGeo t = tgeo(c);
#define SO(MD) hipLaunchKernelGGL((k_tpfa_cheb2_out<MD>), dim3(tgrid(t)), dim3(TX, TY), 0, s, t, c.kc, c.dface, res, (const double*)c.dinv, c.cheb.inv_theta, c.cheb.c0, c.cheb.c1, base, z, r, q, c.sc, c.partials, c.counter)
  if (mode == 0) SO(0); else if (mode == 1) SO(1); else SO(2);
#undef SO
}

void launch_tpfa_restrict(const Ctx& c, const double* v, double* rc, hipStream_t s) {
  const TGeo t = tgeo(c);
  TL_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_tpfa_restrict<LL>), dim3((unsigned)c.h.ncells), dim3(256), 0, s, t, c.h, v,
                                         (const double*)c.Rc, rc, (const Scalars*)c.sc));
}

void launch_tpfa_prolong(const Ctx& c, const double* base, const double* e1, const double* e2, double* out,
                         hipStream_t s) {
  const TGeo t = tgeo(c);
  TL_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_tpfa_prolong<LL>), dim3(grid1d(t.n, 256, 8192)), dim3(256), 0, s, t, c.h,
                                         base, (const double*)c.Rc, e1, e2, out, (const Scalars*)c.sc));
}

void launch_tpfa_diag_inv(const Ctx& c, double* dinv, hipStream_t s) {
  const TGeo t = tgeo(c);
  hipLaunchKernelGGL(k_tpfa_diag_inv, dim3(tgrid(t)), dim3(TX, TY), 0, s, t, c.kc, c.dface, dinv);
}

void launch_tpfa_lift(const Ctx& c, const double* f, const double* td, double* b, hipStream_t s) {
  const TGeo t = tgeo(c);
  hipLaunchKernelGGL(k_tpfa_lift, dim3(grid1d(t.n, 256, 8192)), dim3(256), 0, s, t, c.kc, c.dface, f, td, b);
}

void launch_tpfa_flags(const Ctx& c, const uint8_t* in, uint8_t* out, unsigned long long* counts, hipStream_t s) {
  const TGeo t = tgeo(c);
  hipLaunchKernelGGL(k_tpfa_flags, dim3(grid1d(t.n, 256, 8192)), dim3(256), 0, s, t, in, out, counts);
}

void launch_tpfa_cell_load(const Ctx& c, const double* src, double sconst, double* f, hipStream_t s) {
  hipLaunchKernelGGL(k_tpfa_cell_load, dim3(grid1d(c.g.ne, 256, 8192)), dim3(256), 0, s, c.g.ne, src, sconst, c.g.vol,
                     f);
}

void launch_tpfa_heat_source_load(const Ctx& c, double f0, double* f, hipStream_t s) {
  const dim3 gr(grid1d(c.g.ne, 256, 8192)), bl(256);
  if (c.rho_dt == DT_F64)
    hipLaunchKernelGGL((k_tpfa_heat_source_load<double>), gr, bl, 0, s, c.g.ne, (const double*)c.rho, c.mat.p, f0,
                       c.g.vol, f);
  else
    hipLaunchKernelGGL((k_tpfa_heat_source_load<float>), gr, bl, 0, s, c.g.ne, (const float*)c.rho, c.mat.p, f0,
                       c.g.vol, f);
}

void launch_tpfa_sensitivity(const Ctx& c, const double* T, const double* lam, const double* td, double f0,
                             bool source, double* dc, hipStream_t s) {
  const TGeo t = tgeo(c);
  const dim3 gr(grid1d(t.n, 256, 8192)), bl(256);
#define TS(RT, SRC) hipLaunchKernelGGL((k_tpfa_sensitivity<RT, SRC>), gr, bl, 0, s, t, (const RT*)c.rho, c.mat, T, lam, c.dface, td, f0, c.g.vol, dc)
  if (c.rho_dt == DT_F64) { if (source) TS(double, true); else TS(double, false); }
  else { if (source) TS(float, true); else TS(float, false); }
#undef TS
}

int launch_tpfa_galerkin(const Ctx& c, const void* R, int b_dt, int drop_cc, double* out, hipStream_t s) {
  const TGeo t = tgeo(c);
  const long long waves = (long long)c.h.ncells * 27;
  const dim3 gr((unsigned)((waves + 3) / 4)), bl(256);
  if (b_dt == DT_F64)
    TL_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_tpfa_galerkin<double, LL>), gr, bl, 0, s, t, c.h, c.kc, c.dface,
                                           (const double*)R, drop_cc, out));
  else if (b_dt == DT_F32)
    TL_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_tpfa_galerkin<float, LL>), gr, bl, 0, s, t, c.h, c.kc, c.dface,
                                           (const float*)R, drop_cc, out));
  else
    return MSMG_EINVAL;
  return hipGetLastError() == hipSuccess ? MSMG_OK : MSMG_EHIP;
}

}  // namespace msmg
