// Fine-level kernels: matrix-free Q1 apply with the SIMP material law fused in,
// PCG vector updates with deterministic reductions, the level-0 Chebyshev-Jacobi
// smoother, restriction / prolongation with the local spectral basis R_c,
// element sensitivities, consistent loads and grid-to-grid interpolation.
//
// Paper anchors: material law eq. (material); the system A t = f of section
// 2.2 (here with Q1 elements); Algorithm 1 (three-grid cycle) lines for the
// fine level; adjoint sensitivity of section 2.3.
#include <algorithm>

#include "internal.h"
#include "setup.h"

namespace msmg {

// ---------------------------------------------------------------------------
// small elementwise kernels

__global__ void k_pack_mask(const uint8_t* __restrict__ mask, uint32_t* __restrict__ bits, long long nn) {
  const long long w = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long nw = (nn + 31) >> 5;
  if (w >= nw) return;
  uint32_t v = 0;
  const long long base = w << 5;
  for (int b = 0; b < 32; ++b) {
    const long long n = base + b;
    if (n < nn && mask[n]) v |= (1u << b);
  }
  bits[w] = v;
}

template <typename Tin, typename Tout>
__global__ void k_convert(const Tin* __restrict__ in, Tout* __restrict__ out, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = from_f64<Tout>(to_f64<Tin>(in[i]));
}

// Element conductivities k_e = k_min + rho_e^p (k_max - k_min) in FP64 (the
// material law), computed once per density field for the cycle's kernels.
// OT: the stored type (FP64, or the cycle's copy rounded as k_convert rounds).
template <typename RT, typename OT>
__global__ void k_conductivity(const RT* __restrict__ rho, OT* __restrict__ kc, long long ne, Material m) {
  const double dk = m.kmax - m.kmin;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne; e += (long long)gridDim.x * blockDim.x)
    kc[e] = from_f64<OT>(conductivity<double>(to_f64<RT>(rho[e]), m.kmin, dk, m.p));
}

// Jacobi diagonal inverse: D_n = self * sum of the 8 k_e around n; 0 on fixed nodes.
template <typename RT, typename VT>
__global__ void k_diag_inv(Geo g, Stencil st, const RT* __restrict__ rho, Material m,
                           const uint32_t* __restrict__ bits, VT* __restrict__ dinv) {
  const long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (n >= g.nn) return;
  const int i = int(n % g.nnx), j = int((n / g.nnx) % g.nny), k = int(n / ((long long)g.nnx * g.nny));
  double kk[8];
  load_k8<double, RT>(g, rho, m.kmin, m.kmax - m.kmin, m.p, i, j, k, kk);
  double s = 0.0;
  for (int c = 0; c < 8; ++c) s += kk[c];
  const double d = st.self * s;
  dinv[n] = from_f64<VT>(mask_bit(bits, n) ? 0.0 : 1.0 / d);
}

__global__ void k_zero_fixed_copy(const double* __restrict__ in, double* __restrict__ out,
                                  const uint32_t* __restrict__ bits, long long nn) {
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < nn; n += (long long)gridDim.x * blockDim.x)
    out[n] = mask_bit(bits, n) ? 0.0 : in[n];
}

// T = x on free nodes, fixed values (or 0) on fixed nodes.
__global__ void k_finish_solution(double* __restrict__ T, const double* __restrict__ tfix,
                                  const uint32_t* __restrict__ bits, long long nn) {
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < nn; n += (long long)gridDim.x * blockDim.x)
    if (mask_bit(bits, n)) T[n] = tfix ? tfix[n] : 0.0;
}

// ||v||^2 over all nodes (v is zero on fixed nodes); fin sets bb / tol2 or rr.
__global__ void k_norm2(const double* __restrict__ v, long long nn, int what, double rtol2, Scalars* sc,
                        double* partials, unsigned* counter) {
  __shared__ double red[16];
  double s[1] = {0.0};
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < nn; n += (long long)gridDim.x * blockDim.x)
    s[0] += v[n] * v[n];
  grid_reduce<1>(s, red, partials, counter, gridDim.x, blockIdx.x, [&](double* t) {
    if (what == 0) {
      sc->bb = t[0];
      sc->tol2 = rtol2 * t[0];
    } else if (what == 1) {
      sc->rr = t[0];
    } else {
      sc->true_rr = t[0];
    }
  });
}

// x += alpha p in double-double (x = xhi + xlo, the product's rounding error is
// kept with an FMA), r -= alpha q ; rr = ||r||^2, convergence flags.  The
// iterate needs the extra precision at high contrast: T reaches ~1/k_min on
// low-conductivity islands and a binary64 T cannot resolve the flux inside
// high-conductivity regions to a relative residual of 1e-8.
MSMG_DEV void dd_add(double& hi, double& lo, double a, double ae) {
  // (hi, lo) += (a, ae)
  const double s = hi + a;
  const double bb = s - hi;
  const double err = (hi - (s - bb)) + (a - bb);
  const double t = lo + ae + err;
  hi = s + t;
  lo = t - (hi - s);
}

// r -= alpha q and ||r||^2 with the stop tests.  The iterate is not touched
// here: its update x += alpha p is deferred to the direction update, which
// reads p anyway (xpend marks it outstanding).
__global__ void k_update_r(double* __restrict__ r, const double* __restrict__ q, long long nn, Scalars* sc,
                           double* partials, unsigned* counter) {
  if (sc->done) return;
  __shared__ double red[16];
  const double a = sc->alpha;
  double s[1] = {0.0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  // four elements per pass with every load issued before the first store (the
  // compiler cannot move a load of r[n + stride] above the store to r[n] on
  // its own); the sum runs over n, n + stride, ... as in the plain loop
  for (; n + 3 * stride < nn; n += 4 * stride) {
    double rv[4], qv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      rv[u] = r[n + u * stride];
      qv[u] = __builtin_nontemporal_load(q + n + u * stride);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double rn = rv[u] - a * qv[u];
      r[n + u * stride] = rn;
      s[0] += rn * rn;
    }
  }
  for (; n < nn; n += stride) {
    const double rn = r[n] - a * __builtin_nontemporal_load(q + n);
    r[n] = rn;
    s[0] += rn * rn;
  }
  grid_reduce<1>(s, red, partials, counter, gridDim.x, blockIdx.x, [&](double* t) {
    sc->rr = t[0];
    sc->iters += 1;
    sc->xpend = 1;
    if (!(t[0] == t[0]) || t[0] > 1.7e308) {
      sc->status = ST_NONFINITE;
      sc->done = 1;
    } else if (t[0] <= sc->tol2) {
      sc->status = ST_CONV_RECURSIVE;
      sc->done = 1;
    } else if (sc->iters >= sc->maxit) {
      sc->status = ST_MAXIT;
      sc->done = 1;
    }
  });
}

// x += alpha p in double-double: (x, xlo) + the exact product a p as a pair.
// The iterate is streamed with non-temporal accesses: it is not read again
// until the next step, and caching it would evict the direction p that the
// operator apply reads next.
MSMG_DEV void dd_axpy(double* __restrict__ x, float* __restrict__ xlo, long long n, double a, double pn) {
  const double prod = a * pn;
  const double perr = fma(a, pn, -prod);
  double hi = __builtin_nontemporal_load(x + n), lo = double(__builtin_nontemporal_load(xlo + n));
  dd_add(hi, lo, prod, perr);
  __builtin_nontemporal_store(hi, x + n);
  __builtin_nontemporal_store(float(lo), xlo + n);  // |lo| <= ulp(hi) / 2: FP32 keeps about 77 bits of the sum
}

// The outstanding x += alpha p once the iteration has stopped (ignores `done`).
__global__ void k_update_x_pending(double* __restrict__ x, float* __restrict__ xlo, const double* __restrict__ p,
                                   long long nn, const Scalars* sc) {
  if (!sc->xpend) return;
  const double a = sc->alpha;
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < nn; n += (long long)gridDim.x * blockDim.x)
    dd_axpy(x, xlo, n, a, p[n]);
}

// T = xhi + xlo rounded (or xlo copied out when tlo is given) on free nodes;
// fixed values (or 0) on fixed nodes.
__global__ void k_finish_solution_dd(double* __restrict__ T, const float* __restrict__ xlo, double* __restrict__ tlo,
                                     const double* __restrict__ tfix, const uint32_t* __restrict__ bits, long long nn) {
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < nn; n += (long long)gridDim.x * blockDim.x) {
    if (mask_bit(bits, n)) {
      T[n] = tfix ? tfix[n] : 0.0;
      if (tlo) tlo[n] = 0.0;
    } else if (tlo) {
      tlo[n] = double(xlo[n]);
    } else {
      T[n] = T[n] + double(xlo[n]);
    }
  }
}

// x += alpha p (when outstanding), then p = z + beta p: one read of the old p.
__global__ void k_update_px(double* __restrict__ x, float* __restrict__ xlo, double* __restrict__ p,
                            const double* __restrict__ z, long long nn, const Scalars* sc) {
  if (sc->done) return;
  const double a = sc->alpha, b = sc->beta;
  if (sc->xpend) {
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < nn; n += (long long)gridDim.x * blockDim.x) {
      const double pn = p[n];
      dd_axpy(x, xlo, n, a, pn);
      p[n] = __builtin_nontemporal_load(z + n) + b * pn;
    }
  } else {
    for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < nn; n += (long long)gridDim.x * blockDim.x)
      p[n] = z[n] + b * p[n];
  }
}

// ---------------------------------------------------------------------------
// Stencil kernels on cell-aligned tiles.

#define TILE_PROLOGUE                                                     \
  const long long tile = xcd_tile(blockIdx.x, gridDim.x);                 \
  const Tile t = tile_of_thread(g, h, CX, tile);

// The LDS-queue march's buffers: one LDS array each, so that the compiler can
// tell a read of one from the loads still landing in the others.
#define MSMG_LDS_BUFFERS(KT)                                                                        \
  __shared__ double lb0[LdsLayout<KT>::BUF_D], lb1[LdsLayout<KT>::BUF_D], lb2[LdsLayout<KT>::BUF_D], \
      lb3[LdsLayout<KT>::BUF_D];                                                                    \
  static_assert(LDS_NB == 4, "four LDS buffers");                                                   \
  double* const bufs[4] = {lb0, lb1, lb2, lb3};

// per-node data of the apply's output
struct ApplyCentre {
  uint32_t w;  // mask word of the node
  double x;    // x_n (MODE 2 only)
};

// y = A x on free rows (MODE 0: 0 on fixed rows; MODE 1: also p^T (A p) ->
// alpha; MODE 2: xr, the caller's raw input, on fixed rows), on the march
// whose prefetch queue sits in LDS.  The staged input x is zero on fixed nodes.
// KT double: the stored FP64 conductivities; KT float: the FP32 canonical
// density, taken through the material law as the element layers are read (the
// value k_conductivity stores), so the apply streams 4 B per element.
template <bool CUBIC, int MODE, int NS, typename KT>
MSMG_MARCH_KERNEL void k_apply(
    Geo g, Stencil st, March mg, const KT* __restrict__ kin, Material mat, const uint32_t* __restrict__ bits,
    Two<const double*> xs, Two<const double*> xrs, Two<double*> ys, Two<Scalars*> scs, Two<double*> partials,
    Two<unsigned*> counters) {
  const SideBlock sb = side_block<NS>();
  Scalars* sc = scs[sb.side];
  if (MODE == 1 && sc->done) return;
  const double* __restrict__ x = xs[sb.side];
  const double* __restrict__ xr = xrs[sb.side];
  double* __restrict__ y = ys[sb.side];
  MSMG_LDS_BUFFERS(KT)
  __shared__ double red[16];
  const long long tile = xcd_tile(sb.blk, sb.nblk);
  double s[1] = {0.0};
  const double dk = mat.kmax - mat.kmin;
  march_lds<CUBIC>(
      g, st, mg, tile, bufs, x, kin,
      [&](KT v) {
        if constexpr (sizeof(KT) == 8) return double(v);
        else return conductivity<double>(to_f64<KT>(v), mat.kmin, dk, mat.p);
      },
      [&](long long b, unsigned o) {
        ApplyCentre c;
        c.w = bits[(b + o) >> 5];
        c.x = MODE == 2 ? plane_ld(xr, b, o) : 0.0;
        return c;
      },
      [&](long long b, unsigned o, double ax, double xc, const ApplyCentre& c) {
        double out = ax;
        if ((c.w >> ((b + o) & 31)) & 1u) out = (MODE == 2) ? c.x : 0.0;
        plane_st(y, b, o, out);
        if (MODE == 1) s[0] += xc * out;
      });
  if (MODE != 1) return;
  grid_reduce<1>(s, red, partials[sb.side], counters[sb.side], int(sb.nblk), int(sb.blk), [&](double* tt) {
    sc->pq = tt[0];
    sc->xpend = 0;  // every block of the preceding direction update has read it
    if (!(tt[0] > 0.0) || !(sc->rz > 0.0)) {
      sc->status = (tt[0] == tt[0] && sc->rz == sc->rz) ? ST_BREAKDOWN : ST_NONFINITE;
      sc->done = 1;
    } else {
      sc->alpha = sc->rz / tt[0];
    }
  });
}

// y = b - A x on free rows (0 on fixed rows); ||y||^2 -> true_rr (if sc).  With
// xlo the iterate is x + xlo and neighbour differences are taken on both parts.
template <typename RT, bool CUBIC>
__global__ void k_residual(Geo g, Stencil st, Hier h, int CX, const RT* __restrict__ rho, Material m,
                           const uint32_t* __restrict__ bits, const double* __restrict__ b,
                           const double* __restrict__ x, const float* __restrict__ xlo, double* __restrict__ y,
                           Scalars* sc, double* partials, unsigned* counter) {
  __shared__ double red[16];
  TILE_PROLOGUE
  const double dk = m.kmax - m.kmin;
  double s[1] = {0.0};
  if (t.active) {
    for (int k = t.zs; k < t.ze; ++k)
      for (int j = t.ys; j < t.ye; ++j)
        for (int i = t.xs; i < t.xe; ++i) {
          const long long n = node_id(g, i, j, k);
          double out = 0.0;
          if (!mask_bit(bits, n)) {
            double kk[8];
            load_k8<double, RT>(g, rho, m.kmin, dk, m.p, i, j, k, kk);
            out = b[n] - gather_apply<double, CUBIC>(g, st, kk, i, j, k,
                                                     [&](int a, int bb, int c) { return x[node_id(g, a, bb, c)]; });
            if (xlo)
              out -= gather_apply<double, CUBIC>(g, st, kk, i, j, k,
                                                 [&](int a, int bb, int c) { return double(xlo[node_id(g, a, bb, c)]); });
          }
          y[n] = out;
          s[0] += out * out;
        }
  }
  if (!sc) return;
  grid_reduce<1>(s, red, partials, counter, gridDim.x, blockIdx.x, [&](double* tt) { sc->true_rr = tt[0]; });
}

// ---------------------------------------------------------------------------
// Level-0 of Algorithm 1.  Chebyshev coefficients for the interval [lo, hi] of
// D^-1 A: theta = (hi+lo)/2, delta = (hi-lo)/2, sigma = theta/delta.

// Step 1 of the smoother (degree 1, or the start of higher degrees): x1 = D^-1 r / theta.
template <typename VT, typename IT, typename DT>
__global__ void k_cheb_first(const IT* __restrict__ r, const DT* __restrict__ dinv, VT* __restrict__ x,
                             VT* __restrict__ d, long long nn, double inv_theta, const Scalars* sc) {
  if (sc && sc->done) return;
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < nn; n += (long long)gridDim.x * blockDim.x) {
    const VT v = VT(ld<VT, IT>(r, n) * VT(dinv[n]) * VT(inv_theta));
    x[n] = v;
    if (d) d[n] = v;
  }
}

// Fused first two Chebyshev steps, started from a zero guess:
//   z1 = D^-1 r / theta,  out = (1 + rho1 rho0) z1 + (2 rho1 / delta) D^-1 (r - A z1)
// with z1 staged for the neighbours straight from r and D^-1.  When `dout` is
// given the second direction d1 = out - z1 is stored for further steps.
template <typename DT, typename IT>
struct RD {
  IT r;
  DT di;
};

template <typename VT, typename KT, typename IT, typename DT, bool CUBIC, int NS>
MSMG_MARCH_KERNEL void k_cheb2(Geo g, Stencil st, March mg, const KT* __restrict__ kv, Two<const IT*> rs,
                               const DT* __restrict__ dinv, Two<VT*> outs, VT* __restrict__ dout, ChebCoef cc,
                               Two<const Scalars*> scs) {
  const SideBlock sb = side_block<NS>();
  const Scalars* sc = scs[sb.side];
  if (sc && sc->done) return;
  const IT* __restrict__ r = rs[sb.side];
  VT* __restrict__ out = outs[sb.side];
  __shared__ VT sx[2 * PW * PH];
  __shared__ VT sk[2 * EW * EH];
  const long long tile = xcd_tile(sb.blk, sb.nblk);
  const VT it = VT(cc.inv_theta), c0 = VT(cc.c0), c1 = VT(cc.c1);
  auto loadrd = [&](long long b, unsigned o) {
    RD<DT, IT> v;
    v.r = plane_ld(r, b, o);
    v.di = plane_ld(dinv, b, o);
    return v;
  };
  march<VT, CUBIC>(
      g, st, mg, tile, sx, sk, loadrd, [&](const RD<DT, IT>& v) { return cvt<VT, IT>(v.r) * VT(v.di) * it; },
      [&](long long b, unsigned o) { return plane_ld(kv, b, o); }, [&](KT v) { return cvt<VT, KT>(v); }, loadrd,
      [&](long long b, unsigned o, VT az, VT z1, const RD<DT, IT>& c) {
        VT v = VT(0);
        if (c.di != DT(0)) v = c0 * z1 + c1 * VT(c.di) * (cvt<VT, IT>(c.r) - az);
        plane_st(out, b, o, v);
        if (dout) plane_st(dout, b, o, VT(v - z1));
      });
}

// Generic Chebyshev step k >= 3:  res = r - A x;  d = a d + b D^-1 res;  xout = x + d.
template <typename VT, typename IT, typename DT>
struct RDD {
  IT r;
  DT di;
  VT d;
};

template <typename VT, typename KT, typename IT, typename DT, bool CUBIC>
MSMG_MARCH_KERNEL void k_cheb_step(Geo g, Stencil st, March mg, const KT* __restrict__ kv,
                                                             const IT* __restrict__ r,
                                                             const DT* __restrict__ dinv, const VT* __restrict__ x,
                                                             VT* __restrict__ d, VT* __restrict__ xout, double ca,
                                                             double cb, const Scalars* sc) {
  if (sc && sc->done) return;
  __shared__ VT sx[2 * PW * PH];
  __shared__ VT sk[2 * EW * EH];
  const long long tile = xcd_tile(blockIdx.x, gridDim.x);
  march<VT, CUBIC>(
      g, st, mg, tile, sx, sk, [&](long long b, unsigned o) { return plane_ld(x, b, o); }, [&](VT v) { return v; },
      [&](long long b, unsigned o) { return plane_ld(kv, b, o); }, [&](KT v) { return cvt<VT, KT>(v); },
      [&](long long b, unsigned o) {
        RDD<VT, IT, DT> c;
        c.r = plane_ld(r, b, o);
        c.di = plane_ld(dinv, b, o);
        c.d = plane_ld(d, b, o);
        return c;
      },
      [&](long long b, unsigned o, VT ax, VT xc, const RDD<VT, IT, DT>& c) {
        if (c.di == DT(0)) {
          plane_st(d, b, o, VT(0));
          plane_st(xout, b, o, VT(0));
          return;
        }
        const VT dn = VT(ca) * c.d + VT(cb) * VT(c.di) * (cvt<VT, IT>(c.r) - ax);
        plane_st(d, b, o, dn);
        plane_st(xout, b, o, VT(xc + dn));
      });
}

// One row of R_c (L basis values of node n) widened to FP64, with one vector
// load when the row is 4, 8, 16 or 32 bytes (rows start at multiples of the
// row size, so these loads are aligned).
template <typename BT, int L>
MSMG_DEV void load_row(const BT* __restrict__ Rc, long long n, double out[L]) {
  constexpr int B = L * int(sizeof(BT));
  BT v[L];
  if constexpr (B == 32) {
    const uint4* p = reinterpret_cast<const uint4*>(Rc + n * L);
    const uint4 w0 = p[0], w1 = p[1];
    __builtin_memcpy(v, &w0, 16);
    __builtin_memcpy(reinterpret_cast<char*>(v) + 16, &w1, 16);
  } else if constexpr (B == 16) {
    const uint4 w = *reinterpret_cast<const uint4*>(Rc + n * L);
    __builtin_memcpy(v, &w, 16);
  } else if constexpr (B == 8) {
    const uint2 w = *reinterpret_cast<const uint2*>(Rc + n * L);
    __builtin_memcpy(v, &w, 8);
  } else if constexpr (B == 4) {
    const uint32_t w = *reinterpret_cast<const uint32_t*>(Rc + n * L);
    __builtin_memcpy(v, &w, 4);
  } else {
#pragma unroll
    for (int l = 0; l < L; ++l) v[l] = Rc[n * L + l];
  }
#pragma unroll
  for (int l = 0; l < L; ++l) out[l] = to_f64(v[l]);
}

// Restriction of Algorithm 1:  rc[cell][l] = sum_{n in cell} R_c[n][l] r_n over
// the nodes a cell owns (r and R_c vanish on fixed nodes).  One block holds
// whole coarse cells, so the per-cell sums finish in the block (fixed order).
template <typename VT, typename BT, int L>
__global__ void k_restrict(Geo g, Hier h, int CX, const VT* __restrict__ r, const BT* __restrict__ Rc,
                           double* __restrict__ rc, const Scalars* sc) {
  if (sc && sc->done) return;
  extern __shared__ double smem[];
  TILE_PROLOGUE
  double acc[L];
#pragma unroll
  for (int l = 0; l < L; ++l) acc[l] = 0.0;
  if (t.active) {
    for (int j = t.ys; j < t.ye; ++j)
      for (int i = t.xs; i < t.xe; ++i) {
        const long long n0 = node_id(g, i, j, t.zs), pl = (long long)g.nnx * g.nny;
#pragma unroll 4
        for (int k = 0; k < t.ze - t.zs; ++k) {
          const long long n = n0 + k * pl;
          double row[L];
          load_row<BT, L>(Rc, n, row);
          const double res = double(r[n]);
#pragma unroll
          for (int l = 0; l < L; ++l) acc[l] += row[l] * res;
        }
      }
  }
  // per-cell reduction in fixed order.  Each wave is one node row of the tile
  // (blockDim.x = CX*H = 64 when H divides 64): groups of H lanes belong to one
  // cell, so a segmented xor-shuffle sums the row, then the H rows are summed.
  const int nthr = blockDim.x * blockDim.y;
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;
  const int ntx = (h.ncx + CX - 1) / CX;
  const int tx = int(tile % ntx), ty = int((tile / ntx) % h.ncy), tz = int(tile / ((long long)ntx * h.ncy));
  double* red = smem;
  const bool pow2 = (h.H & (h.H - 1)) == 0 && blockDim.x == 64;
  if (pow2) {
#pragma unroll
    for (int l = 0; l < L; ++l) {
      double v = acc[l];
      for (int off = 1; off < h.H; off <<= 1) v += __shfl_xor(v, off, 64);
      acc[l] = v;
    }
    if ((threadIdx.x % h.H) == 0) {
      const int cl = threadIdx.x / h.H;
#pragma unroll
      for (int l = 0; l < L; ++l) red[(threadIdx.y * CX + cl) * L + l] = acc[l];
    }
    __syncthreads();
    for (int q = tid; q < CX * L; q += nthr) {
      const int cl = q / L, l = q % L;
      const int cx = tx * CX + cl;
      if (cx >= h.ncx || tz >= h.ncz) continue;
      double sum = 0.0;
      for (int ly = 0; ly < (int)blockDim.y; ++ly) sum += red[(ly * CX + cl) * L + l];
      const long long cell = ((long long)tz * h.ncy + ty) * h.ncx + cx;
      rc[cell * L + l] = sum;
    }
    return;
  }
#pragma unroll
  for (int l = 0; l < L; ++l) red[l * nthr + tid] = acc[l];
  __syncthreads();
  for (int q = tid; q < CX * L; q += nthr) {
    const int cl = q / L, l = q % L;
    const int cx = tx * CX + cl;
    if (cx >= h.ncx || tz >= h.ncz) continue;
    double sum = 0.0;
    for (int ly = 0; ly < (int)blockDim.y; ++ly)
      for (int lx = cl * h.H; lx < (cl + 1) * h.H; ++lx) sum += red[l * nthr + ly * blockDim.x + lx];
    const long long cell = ((long long)tz * h.ncy + ty) * h.ncx + cx;
    rc[cell * L + l] = sum;
  }
}

// Prolongation of Algorithm 1: out = base + sum_l R_c[n][l] (e1 + e2)[owner(n)][l]
// (e2 optional).  Fixed nodes stay 0 (R_c vanishes there).
// With NS = 2 each thread prolongs both sides' corrections with one read of
// the basis row (a side whose solve has stopped is skipped).
template <typename VT, typename BT, int L, int NS>
__global__ void k_prolong(Geo g, Hier h, int CX, Two<const VT*> bases, const BT* __restrict__ Rc,
                          Two<const double*> e1s, Two<const double*> e2s, Two<double*> outs,
                          Two<const Scalars*> scs) {
  bool live[NS];
  bool any = false;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    live[q] = !(scs[q] && scs[q]->done);
    any = any || live[q];
  }
  if (!any) return;
  TILE_PROLOGUE
  if (!t.active) return;
  const long long cell = ((long long)t.cz * h.ncy + t.cy) * h.ncx + t.cx;
  double e[NS][L];
#pragma unroll
  for (int q = 0; q < NS; ++q)
#pragma unroll
    for (int l = 0; l < L; ++l) e[q][l] = live[q] ? e1s[q][cell * L + l] + (e2s[q] ? e2s[q][cell * L + l] : 0.0) : 0.0;
  for (int j = t.ys; j < t.ye; ++j)
    for (int i = t.xs; i < t.xe; ++i) {
      const long long n0 = node_id(g, i, j, t.zs), pl = (long long)g.nnx * g.nny;
#pragma unroll 4
      for (int k = 0; k < t.ze - t.zs; ++k) {
        const long long n = n0 + k * pl;
        double row[L];
        load_row<BT, L>(Rc, n, row);
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          if (!live[q]) continue;
          double v = bases[q] ? double(bases[q][n]) : 0.0;
#pragma unroll
          for (int l = 0; l < L; ++l) v += row[l] * e[q][l];
          outs[q][n] = v;
        }
      }
    }
}

// V-cycle residual on level 0:  out = r - A x (free rows).  The stencil runs in
// the type of x: after the coarse correction x carries the large, nearly flat
// values of the low-energy modes and is kept in FP64.
template <typename IT>
struct RW {
  IT r;
  uint32_t w;
};

template <typename VT, typename KT, typename IT, typename XT, bool CUBIC, int NS>
MSMG_MARCH_KERNEL void k_vresidual(Geo g, Stencil st, March mg, const KT* __restrict__ kv,
                                   const uint32_t* __restrict__ bits, Two<const IT*> rs, Two<const XT*> xs,
                                   Two<VT*> outs, Two<const Scalars*> scs) {
  const SideBlock sb = side_block<NS>();
  const Scalars* sc = scs[sb.side];
  if (sc && sc->done) return;
  const IT* __restrict__ r = rs[sb.side];
  const XT* __restrict__ x = xs[sb.side];
  VT* __restrict__ out = outs[sb.side];
  __shared__ XT sx[2 * PW * PH];
  __shared__ XT sk[2 * EW * EH];
  const long long tile = xcd_tile(sb.blk, sb.nblk);
  march<XT, CUBIC>(
      g, st, mg, tile, sx, sk, [&](long long b, unsigned o) { return plane_ld(x, b, o); }, [&](XT v) { return v; },
      [&](long long b, unsigned o) { return plane_ld(kv, b, o); }, [&](KT v) { return cvt<XT, KT>(v); },
      [&](long long b, unsigned o) {
        RW<IT> c;
        c.r = plane_ld(r, b, o);
        c.w = bits[(b + o) >> 5];
        return c;
      },
      [&](long long b, unsigned o, XT ax, XT, const RW<IT>& c) {
        plane_st(out, b, o, ((c.w >> ((b + o) & 31)) & 1u) ? VT(0) : VT(cvt<XT, IT>(c.r) - ax));
      });
}

// ---------------------------------------------------------------------------
// Residual fused with the restriction of Algorithm 1: rc = R_c (r - A x).  The
// march computes the residual of each node (rounded to the cycle's vector type
// VT, as the stored residual would be) and accumulates R_c[n][l] times it for
// the node's coarse cell; the residual itself is never stored.  At the end of
// every coarse z-cell of its chunk a workgroup reduces the sums per coarse
// cell it meets (lanes of one cell row by shuffles, then rows) and writes them
// to its own slots of rpart; k_restrict_finish adds the slots of each cell in
// a fixed order, so the result is bitwise reproducible.
template <typename IT, typename BT, int L>
struct RWB {
  IT r;
  uint32_t w;
  BT row[L];
};

template <typename BT, int L>
MSMG_DEV void load_row_raw(const BT* __restrict__ Rc, long long n, BT out[L]) {
  constexpr int B = L * int(sizeof(BT));
  if constexpr (B == 32) {
    const uint4* p = reinterpret_cast<const uint4*>(Rc + n * L);
    const uint4 w0 = p[0], w1 = p[1];
    __builtin_memcpy(out, &w0, 16);
    __builtin_memcpy(reinterpret_cast<char*>(out) + 16, &w1, 16);
  } else if constexpr (B == 16) {
    const uint4 w = *reinterpret_cast<const uint4*>(Rc + n * L);
    __builtin_memcpy(out, &w, 16);
  } else if constexpr (B == 8) {
    const uint2 w = *reinterpret_cast<const uint2*>(Rc + n * L);
    __builtin_memcpy(out, &w, 8);
  } else if constexpr (B == 4) {
    const uint32_t w = *reinterpret_cast<const uint32_t*>(Rc + n * L);
    __builtin_memcpy(out, &w, 4);
  } else {
#pragma unroll
    for (int l = 0; l < L; ++l) out[l] = Rc[n * L + l];
  }
}

// The residual after the coarse correction with the prolongation fused in:
// x = base + R_c^T e (e = e1 + e2 per coarse cell) is formed for every node
// the march stages, halo included, in the order k_prolong uses, so that
// out = r - A x and the prolonged vector x2 (written for the owned nodes) are
// those of the two separate kernels to the bit.  Each staging slot keeps the
// e of its current coarse cell in registers and reloads it when the march
// enters the next coarse z-cell.
template <typename VT, typename BT, int L>
struct PRN {
  VT base;
  BT row[L];
};

template <typename VT, typename KT, typename BT, int L, bool CUBIC>
MSMG_MARCH_KERNEL void k_vresidual_prolong(Geo g, Stencil st, March mg, Hier h, const KT* __restrict__ kv,
                                           const uint32_t* __restrict__ bits, const double* __restrict__ r,
                                           const VT* __restrict__ base, const BT* __restrict__ Rc,
                                           const double* __restrict__ e1, const double* __restrict__ e2,
                                           VT* __restrict__ out, double* __restrict__ x2, const Scalars* sc) {
  if (sc && sc->done) return;
  static_assert(march_depth<double>() == 1, "the e registers assume a one-step queue");
  static_assert(MARCH_NODE_SLOTS == 2, "two node slots per thread");
  __shared__ double sx[2 * PW * PH];
  __shared__ double sk[2 * EW * EH];
  const long long tile = xcd_tile(blockIdx.x, gridDim.x);
  // coarse cell column (x, y) of each staging slot, and its current e
  int ccx[2], ccy[2], ecz[2] = {-1, -1};
  double ev[2][L];
  {
    int gx, gy;
    march_slot_xy<0>(g, mg, tile, gx, gy);
    ccx[0] = owner_axis(gx, h.H, h.ncx);
    ccy[0] = owner_axis(gy, h.H, h.ncy);
    march_slot_xy<1>(g, mg, tile, gx, gy);
    ccx[1] = owner_axis(gx, h.H, h.ncx);
    ccy[1] = owner_axis(gy, h.H, h.ncy);
  }
  march<double, CUBIC>(
      g, st, mg, tile, sx, sk,
      [&](long long b, unsigned o, int slot, int zz) {
        const int cz = owner_axis(zz, h.H, h.ncz);
        if (cz != ecz[slot]) {
          const long long cell = ((long long)cz * h.ncy + ccy[slot]) * h.ncx + ccx[slot];
#pragma unroll
          for (int l = 0; l < L; ++l) ev[slot][l] = e1[cell * L + l] + (e2 ? e2[cell * L + l] : 0.0);
          ecz[slot] = cz;
        }
        PRN<VT, BT, L> v;
        v.base = plane_ld(base, b, o);
        load_row_raw<BT, L>(Rc, b + o, v.row);
        return v;
      },
      [&](const PRN<VT, BT, L>& v, int slot) {
        double x = double(v.base);
#pragma unroll
        for (int l = 0; l < L; ++l) x += to_f64(v.row[l]) * ev[slot][l];
        return x;
      },
      [&](long long b, unsigned o) { return plane_ld(kv, b, o); }, [&](KT v) { return cvt<double, KT>(v); },
      [&](long long b, unsigned o) {
        RW<double> c;
        c.r = plane_ld(r, b, o);
        c.w = bits[(b + o) >> 5];
        return c;
      },
      [&](long long b, unsigned o, double ax, double xc, const RW<double>& c) {
        plane_st(out, b, o, ((c.w >> ((b + o) & 31)) & 1u) ? VT(0) : VT(c.r - ax));
        plane_st(x2, b, o, xc);
      });
}

template <typename VT, typename KT, typename XT, typename BT, int L, bool CUBIC, int NS>
MSMG_MARCH_KERNEL void k_vresidual_restrict(Geo g, Stencil st, Hier h, RestrictGeo rg, const KT* __restrict__ kv,
                                            const uint32_t* __restrict__ bits, Two<const double*> rs,
                                            Two<const XT*> xs, const BT* __restrict__ Rc, Two<double*> rparts,
                                            Two<const Scalars*> scs) {
  const SideBlock sb = side_block<NS>();
  const Scalars* sc = scs[sb.side];
  if (sc && sc->done) return;
  const double* __restrict__ r = rs[sb.side];
  const XT* __restrict__ x = xs[sb.side];
  double* __restrict__ rpart = rparts[sb.side];
  __shared__ XT sx[2 * PW * PH];
  __shared__ XT sk[2 * EW * EH];
  __shared__ double red[MY * (MX / 2) * L];  // [row][cell of the row][l], at most MX / 2 cells per row
  const long long tile = xcd_tile(sb.blk, sb.nblk);
  const March& mg = rg.m;
  const int tx = int(tile % mg.ntx), ty = int((tile / mg.ntx) % mg.nty);
  const int xa = tx * MX, ya = ty * MY;
  const int lx = threadIdx.x, ly = threadIdx.y, tid = lx + MX * ly;
  const int H = h.H;
  const int cx0 = owner_axis(xa, H, h.ncx), cy0 = owner_axis(ya, H, h.ncy);
  double acc[L];
#pragma unroll
  for (int l = 0; l < L; ++l) acc[l] = 0.0;
  march_ex<XT, CUBIC>(
      g, st, mg, tile, sx, sk, [&](long long b, unsigned o) { return plane_ld(x, b, o); }, [&](XT v) { return v; },
      [&](long long b, unsigned o) { return plane_ld(kv, b, o); }, [&](KT v) { return cvt<XT, KT>(v); },
      [&](long long b, unsigned o) {
        RWB<double, BT, L> c;
        c.r = plane_ld(r, b, o);
        c.w = bits[(b + o) >> 5];
        load_row_raw<BT, L>(Rc, b + o, c.row);
        return c;
      },
      [&](long long b, unsigned o, XT ax, XT, const RWB<double, BT, L>& c) {
        if ((c.w >> ((b + o) & 31)) & 1u) return;  // fixed node: residual and basis vanish
        const double res = double(VT(cvt<XT, double>(c.r) - ax));
#pragma unroll
        for (int l = 0; l < L; ++l) acc[l] += to_f64(c.row[l]) * res;
      },
      [&](int z, int za, int zb) {
        if (z >= zb) return;
        const int czl = owner_axis(z, H, h.ncz);
        if (z + 1 < zb && owner_axis(z + 1, H, h.ncz) == czl) return;  // uniform over the workgroup
        // cell sums of this row: groups of H lanes (a row is one wave, MX = 64)
#pragma unroll
        for (int l = 0; l < L; ++l) {
          double v = acc[l];
          for (int off = 1; off < H; off <<= 1) v += __shfl_xor(v, off, 64);
          if (lx % H == 0) red[(ly * (MX / 2) + lx / H) * L + l] = v;
          acc[l] = 0.0;
        }
        __syncthreads();
        // the last cell of an axis keeps the remainder nodes, so it may hold
        // several lane groups (and rows): add the groups by owner cell
        const int lcz = czl - owner_axis(za, H, h.ncz);
        const int ngrp = MX / H;
        for (int q = tid; q < rg.nlx * rg.nly * L; q += MARCH_THREADS) {
          const int l = q % L, lc = q / L, lcx = lc % rg.nlx, lcy = lc / rg.nlx;
          double sum = 0.0;
          for (int row = 0; row < MY; ++row) {
            if (owner_axis(ya + row, H, h.ncy) - cy0 != lcy) continue;
            for (int grp = 0; grp < ngrp; ++grp)
              if (owner_axis(xa + grp * H, H, h.ncx) - cx0 == lcx) sum += red[(row * (MX / 2) + grp) * L + l];
          }
          rpart[(((tile * rg.nlz + lcz) * rg.nly + lcy) * rg.nlx + lcx) * L + l] = sum;
        }
        __syncthreads();
      });
}

// rc[cell][l] = sum of the cell's slots, over the workgroups whose column
// blocks meet the cell (y, then x), in its one z chunk.
template <int L>
__global__ void k_restrict_finish(Geo g, Hier h, RestrictGeo rg, const double* __restrict__ rpart,
                                  double* __restrict__ rc, const Scalars* sc) {
  if (sc && sc->done) return;
  const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (q >= (long long)h.ncells * L) return;
  const int l = int(q % L);
  const long long cell = q / L;
  const int cx = int(cell % h.ncx), cy = int((cell / h.ncx) % h.ncy), cz = int(cell / ((long long)h.ncx * h.ncy));
  const int H = h.H;
  const int tx0 = (cx * H) / MX, tx1 = (cell_end(cx, H, h.ncx, g.nnx) - 1) / MX;
  const int ty0 = (cy * H) / MY, ty1 = (cell_end(cy, H, h.ncy, g.nny) - 1) / MY;
  const int tz = cz / rg.czc, lcz = cz - tz * rg.czc;
  double sum = 0.0;
  for (int ty = ty0; ty <= ty1; ++ty) {
    const int lcy = cy - owner_axis(ty * MY, H, h.ncy);
    for (int tx = tx0; tx <= tx1; ++tx) {
      const int lcx = cx - owner_axis(tx * MX, H, h.ncx);
      const long long tile = tx + (long long)rg.m.ntx * (ty + (long long)rg.m.nty * tz);
      sum += rpart[(((tile * rg.nlz + lcz) * rg.nly + lcy) * rg.nlx + lcx) * L + l];
    }
  }
  rc[cell * L + l] = sum;
}

// z = a + b (V-cycle type) written as FP64, with the PCG products z^T r and
// z^T q; fin computes beta (Polak-Ribiere) and the new r^T z.
//   mode 0: initial (beta = 0); mode 1: iteration; mode 2: no reduction.
template <typename AT_, typename VT>
__global__ void k_vc_output(const AT_* __restrict__ a, const VT* __restrict__ b, double* __restrict__ z,
                            const double* __restrict__ r, const double* __restrict__ q, long long nn, int mode,
                            Scalars* sc, double* partials, unsigned* counter) {
  if (sc && sc->done) return;
  __shared__ double red[32];
  double s[2] = {0.0, 0.0};
#pragma unroll 4
  for (long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x; n < nn; n += (long long)gridDim.x * blockDim.x) {
    const double v = double(a[n]) + (b ? double(b[n]) : 0.0);
    z[n] = v;
    if (mode != 2) {
      s[0] += v * r[n];
      if (mode == 1) s[1] += v * q[n];
    }
  }
  if (mode == 2) return;
  grid_reduce<2>(s, red, partials, counter, gridDim.x, blockIdx.x, [&](double* tt) { vc_finish(sc, tt, mode); });
}

// Post-smoother fused with the V-cycle output (degree-2 Chebyshev): the two
// Chebyshev steps of k_cheb2 applied to `res`, then z = base + v written as
// FP64 with the PCG products z^T r (MODE 0, 1) and z^T q (MODE 1) reduced as
// in k_vc_output.  `base` (the prolonged correction) may be null.  v is
// rounded to VT before the sum, so z is the value the unfused pair computes.
template <typename DT, typename IT>
struct RDZ {
  IT r;
  DT di;
  double b, rr, q;
};

template <typename VT, typename KT, typename IT, typename DT, bool CUBIC, int MODE, int NS>
MSMG_MARCH_KERNEL void k_cheb2_out(Geo g, Stencil st, March mg, const KT* __restrict__ kv, Two<const IT*> ress,
                                   const DT* __restrict__ dinv, ChebCoef cc, Two<const double*> bases,
                                   Two<double*> zs, Two<const double*> rs, Two<const double*> qs, Two<Scalars*> scs,
                                   Two<double*> partials, Two<unsigned*> counters) {
  const SideBlock sb = side_block<NS>();
  Scalars* sc = scs[sb.side];
  if (sc->done) return;
  const IT* __restrict__ res = ress[sb.side];
  const double* __restrict__ base = bases[sb.side];
  double* __restrict__ z = zs[sb.side];
  const double* __restrict__ r = rs[sb.side];
  const double* __restrict__ q = qs[sb.side];
  __shared__ VT sx[2 * PW * PH];
  __shared__ VT sk[2 * EW * EH];
  __shared__ double red[32];
  const long long tile = xcd_tile(sb.blk, sb.nblk);
  const VT it = VT(cc.inv_theta), c0 = VT(cc.c0), c1 = VT(cc.c1);
  double s[2] = {0.0, 0.0};
  march<VT, CUBIC>(
      g, st, mg, tile, sx, sk,
      [&](long long b, unsigned o) {
        RD<DT, IT> v;
        v.r = plane_ld(res, b, o);
        v.di = plane_ld(dinv, b, o);
        return v;
      },
      [&](const RD<DT, IT>& v) { return cvt<VT, IT>(v.r) * VT(v.di) * it; },
      [&](long long b, unsigned o) { return plane_ld(kv, b, o); }, [&](KT v) { return cvt<VT, KT>(v); },
      [&](long long b, unsigned o) {
        // the output's operands ride in the prefetch queue with the planes
        // (one wave per SIMD fewer than k_cheb2, still faster than loading
        // them at the output)
        RDZ<DT, IT> c;
        c.r = plane_ld(res, b, o);
        c.di = plane_ld(dinv, b, o);
        c.b = base ? plane_ld(base, b, o) : 0.0;
        c.rr = MODE != 2 ? plane_ld(r, b, o) : 0.0;
        c.q = MODE == 1 ? plane_ld(q, b, o) : 0.0;
        return c;
      },
      [&](long long b, unsigned o, VT az, VT z1, const RDZ<DT, IT>& c) {
        VT v = VT(0);
        if (c.di != DT(0)) v = c0 * z1 + c1 * VT(c.di) * (cvt<VT, IT>(c.r) - az);
        const double zz = c.b + double(v);
        plane_st(z, b, o, zz);
        if (MODE != 2) s[0] += zz * c.rr;
        if (MODE == 1) s[1] += zz * c.q;
      });
  if (MODE == 2) return;
  grid_reduce<2>(s, red, partials[sb.side], counters[sb.side], int(sb.nblk), int(sb.blk),
                 [&](double* tt) { vc_finish(sc, tt, MODE); });
}

// ---------------------------------------------------------------------------
// Sensitivity (section 2.3): dc/drho_e = lam^T (df/drho_e - dA/drho_e T)
//   = -p rho^(p-1) [ (kmax - kmin) lam_e^T K0 T_e + f0 (V/8) sum_a lam_a ],
// the second term only for the design-dependent source f0 (1 - rho^p) of
// eq. (material) (SRC = true).
template <typename RT, bool SRC>
__global__ void k_sensitivity(Geo g, Stencil st, const RT* __restrict__ rho, Material m,
                              const double* __restrict__ T, const double* __restrict__ lam,
                              const uint32_t* __restrict__ bits, double f0, double* __restrict__ dc) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= g.ne) return;
  const int i = int(e % g.nx), j = int((e / g.nx) % g.ny), k = int(e / ((long long)g.nx * g.ny));
  double tv[8], lv[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const long long n = node_id(g, i + (a & 1), j + ((a >> 1) & 1), k + ((a >> 2) & 1));
    tv[a] = T[n];
    lv[a] = lam ? lam[n] : (mask_bit(bits, n) ? 0.0 : T[n]);
  }
  // pattern of K0[a][b] by the axes where a and b differ
  double pat[8];
  pat[0] = st.self;
  pat[1] = st.ax[0];
  pat[2] = st.ax[1];
  pat[4] = st.ax[2];
  pat[3] = st.fd[2];
  pat[5] = st.fd[1];
  pat[6] = st.fd[0];
  pat[7] = st.bd;
  // lam^T K0 T = -sum_{a<b} K0[a][b] (lam_a - lam_b)(T_a - T_b)  (zero row sums):
  // differences keep the product accurate where T is large and nearly flat
  double q = 0.0;
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = a + 1; b < 8; ++b) q -= pat[a ^ b] * (lv[a] - lv[b]) * (tv[a] - tv[b]);
  const double r = to_f64<RT>(rho[e]);
  double rp = 1.0;
  for (int t = 1; t < m.p; ++t) rp *= r;
  if (SRC) {
    double ls = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) ls += lv[a];
    // the stiffness term rounds exactly as in the source-free case, so f0 = 0 gives its value
    dc[e] = -double(m.p) * rp * (m.kmax - m.kmin) * q - double(m.p) * rp * (f0 * (g.vol / 8.0) * ls);
  } else {
    dc[e] = -double(m.p) * rp * (m.kmax - m.kmin) * q;
  }
}

// Nodal load of the design-dependent heat source of eq. (material):
// f_n = sum_{e ni n} f0 (1 - rho_e^p) V / 8.
template <typename RT>
__global__ void k_heat_source_load(Geo g, const RT* __restrict__ rho, int p, double f0, double* __restrict__ f) {
  const long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (n >= g.nn) return;
  const int i = int(n % g.nnx), j = int((n / g.nnx) % g.nny), k = int(n / ((long long)g.nnx * g.nny));
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int ei = i - 1 + (c & 1), ej = j - 1 + ((c >> 1) & 1), ek = k - 1 + ((c >> 2) & 1);
    if (ei >= 0 && ei < g.nx && ej >= 0 && ej < g.ny && ek >= 0 && ek < g.nz) {
      const double r = to_f64<RT>(rho[elem_id(g, ei, ej, ek)]);
      double rp = r;
      for (int t = 1; t < p; ++t) rp *= r;
      s += f0 * (1.0 - rp);
    }
  }
  f[n] = s * (g.vol / 8.0);
}

// Consistent load of an element-wise constant source: f_n = sum_{e ni n} s_e V / 8.
__global__ void k_element_load(Geo g, const double* __restrict__ src, double sconst, double* __restrict__ f) {
  const long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (n >= g.nn) return;
  const int i = int(n % g.nnx), j = int((n / g.nnx) % g.nny), k = int(n / ((long long)g.nnx * g.nny));
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int ei = i - 1 + (c & 1), ej = j - 1 + ((c >> 1) & 1), ek = k - 1 + ((c >> 2) & 1);
    if (ei >= 0 && ei < g.nx && ej >= 0 && ej < g.ny && ek >= 0 && ek < g.nz)
      s += src ? src[elem_id(g, ei, ej, ek)] : sconst;
  }
  f[n] = s * (g.vol / 8.0);
}

// Nodal trilinear prolongation (nx,ny,nz) -> (2nx,2ny,2nz): the coarse Q1
// function evaluated at the fine nodes (averages of 1, 2, 4 or 8 coarse nodes).
__global__ void k_prolong_nodal(int nx, int ny, int nz, const double* __restrict__ tc, double* __restrict__ tf) {
  const long long fnx = 2LL * nx + 1, fny = 2LL * ny + 1, fnz = 2LL * nz + 1;
  const long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (n >= fnx * fny * fnz) return;
  const int i = int(n % fnx), j = int((n / fnx) % fny), k = int(n / (fnx * fny));
  const int i0 = i >> 1, j0 = j >> 1, k0 = k >> 1;
  const int i1 = i0 + (i & 1), j1 = j0 + (j & 1), k1 = k0 + (k & 1);
  const long long cnx = nx + 1, cny = ny + 1;
  auto at = [&](int a, int b, int c) { return tc[((long long)c * cny + b) * cnx + a]; };
  const double v = at(i0, j0, k0) + at(i1, j0, k0) + at(i0, j1, k0) + at(i1, j1, k0) + at(i0, j0, k1) +
                   at(i1, j0, k1) + at(i0, j1, k1) + at(i1, j1, k1);
  tf[n] = 0.125 * v;
}

// Element injection (nx,ny,nz) -> (2nx,2ny,2nz): each child takes its parent's value.
// Streaming reference of the operator apply's memory traffic: y = x + k over
// the first ne entries, y = x beyond, i.e. exactly one read of every x and k
// value and one write of every y value (8 B per node twice, 8 B per element),
// coalesced, with no stencil and no halo.  Its rate is the bandwidth this
// access mix reaches on the device, the practical ceiling of k_apply.
typedef double dvec2 __attribute__((ext_vector_type(2)));
__global__ void k_stream_ceiling(const dvec2* __restrict__ x, const dvec2* __restrict__ k, dvec2* __restrict__ y,
                                 long long nn2, long long ne2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn2; i += (long long)gridDim.x * blockDim.x) {
    dvec2 v = __builtin_nontemporal_load(x + i);
    if (i < ne2) v += __builtin_nontemporal_load(k + i);
    __builtin_nontemporal_store(v, y + i);
  }
}

template <typename T>
__global__ void k_prolong_element(int nx, int ny, int nz, const T* __restrict__ rc, T* __restrict__ rf) {
  const long long fnx = 2LL * nx, fny = 2LL * ny, fnz = 2LL * nz;
  const long long n = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (n >= fnx * fny * fnz) return;
  const int i = int(n % fnx), j = int((n / fnx) % fny), k = int(n / (fnx * fny));
  rf[n] = rc[((long long)(k >> 1) * ny + (j >> 1)) * nx + (i >> 1)];
}


// ---------------------------------------------------------------------------
// utilities

__global__ void k_fill(double* __restrict__ x, double v, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] = v;
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ void k_zero_free(double* __restrict__ x, const uint32_t* __restrict__ bits, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    if (!mask_bit(bits, i)) x[i] = 0.0;
}

// full = 1: fresh solve (iteration count, maxit, status); 0: clear done/status only.
__global__ void k_sc_reset(Scalars* sc, int full, int maxit) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  sc->done = 0;
  sc->status = ST_RUNNING;
  sc->xpend = 0;
  if (full) {
    sc->iters = 0;
    sc->maxit = maxit;
    sc->alpha = sc->beta = 0.0;
  }
}

__global__ void k_count_bits(const uint32_t* __restrict__ bits, long long nw, unsigned* out) {
  unsigned c = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nw; i += (long long)gridDim.x * blockDim.x)
    c += __popc(bits[i]);
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

void launch_fill(const Ctx& c, double* x, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(2048), dim3(256), 0, s, x, v, c.g.nn);
}
void launch_copy(const Ctx& c, const double* a, double* b, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(2048), dim3(256), 0, s, a, b, c.g.nn);
}
void launch_zero_free(const Ctx& c, double* x, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_free, dim3(2048), dim3(256), 0, s, x, c.bits, c.g.nn);
}
void launch_sc_reset(const Ctx& c, int full, int maxit, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_reset, dim3(1), dim3(64), 0, s, c.sc, full, maxit);
}
int count_fixed(const Ctx& c, int* nfixed, hipStream_t s) {
  unsigned* d = c.counter + CTR_FIXED;
  if (hipMemsetAsync(d, 0, 4, s) != hipSuccess) return MSMG_EHIP;
  const long long nw = (c.g.nn + 31) >> 5;
  hipLaunchKernelGGL(k_count_bits, dim3(512), dim3(256), 0, s, c.bits, nw, d);
  unsigned hv = 0;
  if (hipMemcpyAsync(&hv, d, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return MSMG_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return MSMG_EHIP;
  *nfixed = int(hv);
  return MSMG_OK;
}

// ===========================================================================
// Launchers
// ===========================================================================


void launch_pack_mask(const uint8_t* mask, uint32_t* bits, long long nn, hipStream_t s) {
  const long long nw = (nn + 31) >> 5;
  hipLaunchKernelGGL(k_pack_mask, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, mask, bits, nn);
}

void launch_convert(const void* in, int din, void* out, int dout, long long n, hipStream_t s) {
  const dim3 gr(grid1d(n, 256, 8192)), bl(256);
#define CONV(TI, TO) hipLaunchKernelGGL((k_convert<TI, TO>), gr, bl, 0, s, (const TI*)in, (TO*)out, n)
  if (din == DT_F64 && dout == DT_F64) CONV(double, double);
  else if (din == DT_F64 && dout == DT_F32) CONV(double, float);
  else if (din == DT_F64 && dout == DT_BF16) CONV(double, bf16);
  else if (din == DT_F32 && dout == DT_F64) CONV(float, double);
  else if (din == DT_F32 && dout == DT_F32) CONV(float, float);
  else if (din == DT_F32 && dout == DT_BF16) CONV(float, bf16);
  else if (din == DT_BF16 && dout == DT_F64) CONV(bf16, double);
  else if (din == DT_BF16 && dout == DT_F32) CONV(bf16, float);
  else CONV(bf16, bf16);
#undef CONV
}

void launch_conductivity(const Ctx& c, const void* rho, int rdt, void* kc, int kdt, hipStream_t s) {
  const dim3 gr(grid1d(c.g.ne, 256, 8192)), bl(256);
#define KCD(RT, OT) hipLaunchKernelGGL((k_conductivity<RT, OT>), gr, bl, 0, s, (const RT*)rho, (OT*)kc, c.g.ne, c.mat)
  if (rdt == DT_F64) {
    if (kdt == DT_F64) KCD(double, double); else if (kdt == DT_F32) KCD(double, float); else KCD(double, bf16);
  } else {
    if (kdt == DT_F64) KCD(float, double); else if (kdt == DT_F32) KCD(float, float); else KCD(float, bf16);
  }
#undef KCD
}

void launch_diag_inv(const Ctx& c, const void* rho, int rdt, void* dinv, int vdt, hipStream_t s) {
  const dim3 gr((unsigned)((c.g.nn + 255) / 256)), bl(256);
#define DI(RT, VT) hipLaunchKernelGGL((k_diag_inv<RT, VT>), gr, bl, 0, s, c.g, c.st, (const RT*)rho, c.mat, c.bits, (VT*)dinv)
  if (rdt == DT_F64 && vdt == DT_F64) DI(double, double);
  else if (rdt == DT_F64) DI(double, float);
  else if (rdt == DT_F32 && vdt == DT_F64) DI(float, double);
  else DI(float, float);
#undef DI
}

void launch_zero_fixed_copy(const Ctx& c, const double* in, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_fixed_copy, dim3(grid1d(c.g.nn, 256, 8192)), dim3(256), 0, s, in, out, c.bits, c.g.nn);
}

void launch_finish_solution(const Ctx& c, double* T, const double* tfix, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_solution, dim3(grid1d(c.g.nn, 256, 8192)), dim3(256), 0, s, T, tfix, c.bits, c.g.nn);
}

void launch_norm2(const Ctx& c, const double* v, int what, double rtol2, hipStream_t s) {
  const int nb = grid1d(c.g.nn, 256, c.red_blocks);
  hipLaunchKernelGGL(k_norm2, dim3(nb), dim3(256), 0, s, v, c.g.nn, what, rtol2, c.sc, c.partials, c.counter);
}

void launch_update_r(const Ctx& c, double* r, const double* q, hipStream_t s) {
  const int nb = grid1d(c.g.nn, 256, c.red_blocks);
  hipLaunchKernelGGL(k_update_r, dim3(nb), dim3(256), 0, s, r, q, c.g.nn, c.sc, c.partials, c.counter);
}

void launch_update_x_pending(const Ctx& c, double* x, float* xlo, const double* p, hipStream_t s) {
  hipLaunchKernelGGL(k_update_x_pending, dim3(grid1d(c.g.nn, 256, 8192)), dim3(256), 0, s, x, xlo, p, c.g.nn, c.sc);
}

void launch_finish_solution_dd(const Ctx& c, double* T, const float* xlo, double* tlo, const double* tfix, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_solution_dd, dim3(grid1d(c.g.nn, 256, 8192)), dim3(256), 0, s, T, xlo, tlo, tfix, c.bits, c.g.nn);
}

void launch_update_px(const Ctx& c, double* x, float* xlo, double* p, const double* z, hipStream_t s) {
  hipLaunchKernelGGL(k_update_px, dim3(grid1d(c.g.nn, 256, 8192)), dim3(256), 0, s, x, xlo, p, z, c.g.nn, c.sc);
}

static inline dim3 tile_block(const Ctx& c) { return dim3(c.CX * c.h.H, c.h.H); }
// tiles are remapped per XCD (xcd_tile), which needs a multiple of 8 workgroups
static inline dim3 tile_grid(const Ctx& c) { return dim3((unsigned)(((c.ntiles + 7) / 8) * 8)); }

static inline dim3 march_grid(const Ctx& c) { return dim3((unsigned)c.mg.blocks); }

long long march_resident_blocks() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 2048;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 2048;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_vresidual<double, bf16, double, double, true, 1>),
                                                   MARCH_THREADS, 0) != hipSuccess)
    return 2048;
  return (long long)(per > 0 ? per : 1) * (cus > 0 ? cus : 1);
}
static inline dim3 march_block() { return dim3(MX, MY); }

long long apply_resident_blocks() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 2048;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 2048;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_apply<true, 1, 1, double>),
                                                   MARCH_THREADS, 0) != hipSuccess)
    return 2048;
  return (long long)(per > 0 ? per : 1) * (cus > 0 ? cus : 1);
}

void launch_apply(const Ctx& c, const double* x, double* y, int mode, hipStream_t s, const double* xraw) {
  const dim3 gr((unsigned)c.mgl.blocks), bl(LMX, LMY);
#define APL(CU, MD, KT, P) hipLaunchKernelGGL((k_apply<CU, MD, 1, KT>), gr, bl, 0, s, c.g, c.st, c.mgl, (const KT*)(P), c.mat, c.bits, one(x), one(xraw), one(y), one(c.sc), one(c.partials), one(c.counter))
#define AP_M(CU, KT, P) do { if (mode == 0) APL(CU, 0, KT, P); else if (mode == 1) APL(CU, 1, KT, P); else APL(CU, 2, KT, P); } while (0)
  // FP64 density: the stored FP64 conductivities; FP32: the density itself
  if (c.kc) { if (c.st.cubic) AP_M(true, double, c.kc); else AP_M(false, double, c.kc); }
  else { if (c.st.cubic) AP_M(true, float, c.rho); else AP_M(false, float, c.rho); }
#undef AP_M
#undef APL
}

void launch_apply_pair(const Ctx& a, const Ctx& b, const double* xa, const double* xb, double* ya, double* yb,
                       hipStream_t s) {
  const dim3 gr((unsigned)(2 * a.mgl.blocks)), bl(LMX, LMY);
#define APL(CU, KT, P) hipLaunchKernelGGL((k_apply<CU, 1, 2, KT>), gr, bl, 0, s, a.g, a.st, a.mgl, (const KT*)(P), a.mat, a.bits, two(xa, xb), two((const double*)nullptr, (const double*)nullptr), two(ya, yb), two(a.sc, b.sc), two(a.partials, b.partials), two(a.counter, b.counter))
  if (a.kc) { if (a.st.cubic) APL(true, double, a.kc); else APL(false, double, a.kc); }
  else { if (a.st.cubic) APL(true, float, a.rho); else APL(false, float, a.rho); }
#undef APL
}

void launch_residual(const Ctx& c, const double* b, const double* x, const float* xlo, double* y, bool reduce,
                     hipStream_t s) {
  const dim3 gr = tile_grid(c), bl = tile_block(c);
  Scalars* sc = reduce ? c.sc : nullptr;
#define RS(RT, CU) hipLaunchKernelGGL((k_residual<RT, CU>), gr, bl, 0, s, c.g, c.st, c.h, c.CX, (const RT*)c.rho, c.mat, c.bits, b, x, xlo, y, sc, c.partials, c.counter)
  if (c.rho_dt == DT_F64) { if (c.st.cubic) RS(double, true); else RS(double, false); }
  else { if (c.st.cubic) RS(float, true); else RS(float, false); }
#undef RS
}

// --- V-cycle level 0 ---------------------------------------------------------

// dispatch over the cycle's types and CUBIC: VT vectors, KVT conductivity
// copy, BT basis R_c, DVT the Jacobi diagonal (FP64 only on the all-FP64 path)
#define VC_CASE(VT_, KVT_, BT_, DVT_, ...)                                 \
  {                                                                        \
    using VT = VT_;                                                        \
    using KVT = KVT_;                                                      \
    using BT = BT_;                                                        \
    using DVT = DVT_;                                                      \
    if (c.st.cubic) {                                                      \
      constexpr bool CU = true;                                            \
      __VA_ARGS__;                                                         \
    } else {                                                               \
      constexpr bool CU = false;                                           \
      __VA_ARGS__;                                                         \
    }                                                                      \
  }
#define VC_DISPATCH(...)                                                                       \
  do {                                                                                         \
    if (c.v_dt == DT_F64) {                                                                    \
      if (c.b_dt == DT_F64) VC_CASE(double, double, double, double, __VA_ARGS__)               \
      else if (c.b_dt == DT_BF16) VC_CASE(double, bf16, bf16, float, __VA_ARGS__)              \
      else if (c.kv_dt == DT_BF16) VC_CASE(double, bf16, float, float, __VA_ARGS__)            \
      else VC_CASE(double, float, float, float, __VA_ARGS__)                                   \
    } else {                                                                                   \
      if (c.kv_dt == DT_BF16 && c.b_dt == DT_BF16) VC_CASE(float, bf16, bf16, float, __VA_ARGS__) \
      else if (c.kv_dt == DT_BF16) VC_CASE(float, bf16, float, float, __VA_ARGS__)           \
      else if (c.b_dt == DT_BF16) VC_CASE(float, float, bf16, float, __VA_ARGS__)              \
      else VC_CASE(float, float, float, float, __VA_ARGS__)                                    \
    }                                                                                          \
  } while (0)

// Level-0 smoother S^-1 applied to `in` (FP64 PCG residual when in_is_f64, else
// a V-cycle vector): out = Chebyshev_d(in).  Uses vc.t0 / vc.t1 as scratch.
void launch_smooth(const Ctx& c, const void* in, bool in_is_f64, void* out, hipStream_t s) {
  const dim3 gr = march_grid(c), bl = march_block();
  const int deg = c.cheb.degree;
  VC_DISPATCH({
    (void)sizeof(BT);
    const DVT* dinv = (const DVT*)c.dinv;
    VT* o = (VT*)out;
    if (deg == 1) {
      if (in_is_f64)
        hipLaunchKernelGGL((k_cheb_first<VT, double, DVT>), dim3(grid1d(c.g.nn, 256, 8192)), dim3(256), 0, s, (const double*)in, dinv, o, (VT*)nullptr, c.g.nn, c.cheb.inv_theta, c.sc);
      else
        hipLaunchKernelGGL((k_cheb_first<VT, VT, DVT>), dim3(grid1d(c.g.nn, 256, 8192)), dim3(256), 0, s, (const VT*)in, dinv, o, (VT*)nullptr, c.g.nn, c.cheb.inv_theta, c.sc);
    } else {
      // first two steps fused; further steps ping-pong between out and t1
      VT* d = deg > 2 ? (VT*)c.vc_t0 : nullptr;
      VT* xa = (deg % 2 == 0) ? o : (VT*)c.vc_t1;  // so that the last step lands in `out`
      VT* xb = (xa == o) ? (VT*)c.vc_t1 : o;
      if (in_is_f64)
        hipLaunchKernelGGL((k_cheb2<VT, KVT, double, DVT, CU, 1>), gr, bl, 0, s, c.g, c.st, c.mg, (const KVT*)c.kv, one((const double*)in), dinv, one(xa), d, c.cheb, one((const Scalars*)c.sc));
      else
        hipLaunchKernelGGL((k_cheb2<VT, KVT, VT, DVT, CU, 1>), gr, bl, 0, s, c.g, c.st, c.mg, (const KVT*)c.kv, one((const VT*)in), dinv, one(xa), d, c.cheb, one((const Scalars*)c.sc));
      for (int step = 2; step < deg; ++step) {
        const double ca = c.cheb.step_a[step], cb = c.cheb.step_b[step];
        if (in_is_f64)
          hipLaunchKernelGGL((k_cheb_step<VT, KVT, double, DVT, CU>), gr, bl, 0, s, c.g, c.st, c.mg, (const KVT*)c.kv, (const double*)in, dinv, xa, d, xb, ca, cb, c.sc);
        else
          hipLaunchKernelGGL((k_cheb_step<VT, KVT, VT, DVT, CU>), gr, bl, 0, s, c.g, c.st, c.mg, (const KVT*)c.kv, (const VT*)in, dinv, xa, d, xb, ca, cb, c.sc);
        VT* tmp = xa; xa = xb; xb = tmp;
      }
    }
  });
}

// The degree-2 smoother S^-1 applied to two FP64 residuals at once.
void launch_smooth_pair(const Ctx& a, const Ctx& b, const double* ina, const double* inb, void* outa, void* outb,
                        hipStream_t s) {
  const Ctx& c = a;
  const dim3 gr((unsigned)(2 * c.mg.blocks)), bl = march_block();
  VC_DISPATCH({
    (void)sizeof(BT);
    hipLaunchKernelGGL((k_cheb2<VT, KVT, double, DVT, CU, 2>), gr, bl, 0, s, c.g, c.st, c.mg, (const KVT*)c.kv,
                       two(ina, inb), (const DVT*)c.dinv, two((VT*)outa, (VT*)outb), (VT*)nullptr, c.cheb,
                       two((const Scalars*)a.sc, (const Scalars*)b.sc));
  });
}

// dispatch over the number of basis vectors per cell (1 .. LC_MAX)
#define L_DISPATCH(Lrt, ...)                  \
  do {                                        \
    switch (Lrt) {                            \
      case 1: { constexpr int LL = 1; __VA_ARGS__; } break; \
      case 2: { constexpr int LL = 2; __VA_ARGS__; } break; \
      case 3: { constexpr int LL = 3; __VA_ARGS__; } break; \
      case 4: { constexpr int LL = 4; __VA_ARGS__; } break; \
      case 5: { constexpr int LL = 5; __VA_ARGS__; } break; \
      case 6: { constexpr int LL = 6; __VA_ARGS__; } break; \
      case 7: { constexpr int LL = 7; __VA_ARGS__; } break; \
      default: { constexpr int LL = 8; __VA_ARGS__; } break; \
    }                                         \
  } while (0)
static_assert(LC_MAX == 8, "L_DISPATCH covers 1 .. 8");

void launch_restrict(const Ctx& c, const void* r, void* rc, hipStream_t s) {
  const dim3 gr = tile_grid(c), bl = tile_block(c);
  const size_t nthr = size_t(bl.x) * bl.y;
  VC_DISPATCH({
    (void)sizeof(KVT);
    (void)sizeof(DVT);
    (void)CU;
    const size_t sh = nthr * c.h.Lc * sizeof(double);
    L_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_restrict<VT, BT, LL>), gr, bl, sh, s, c.g, c.h, c.CX, (const VT*)r, (const BT*)c.Rc, (double*)rc, c.sc));
  });
}

void launch_prolong(const Ctx& c, const void* base, const void* e1, const void* e2, void* out, hipStream_t s) {
  const dim3 gr = tile_grid(c), bl = tile_block(c);
  VC_DISPATCH({
    (void)sizeof(KVT);
    (void)sizeof(DVT);
    (void)CU;
    L_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_prolong<VT, BT, LL, 1>), gr, bl, 0, s, c.g, c.h, c.CX, one((const VT*)base), (const BT*)c.Rc, one((const double*)e1), one((const double*)e2), one((double*)out), one((const Scalars*)c.sc)));
  });
}

void launch_prolong_pair(const Ctx& a, const Ctx& b, const void* basea, const void* baseb, const void* ea,
                         const void* eb, void* outa, void* outb, hipStream_t s) {
  const Ctx& c = a;
  const dim3 gr = tile_grid(c), bl = tile_block(c);
  VC_DISPATCH({
    (void)sizeof(KVT);
    (void)sizeof(DVT);
    (void)CU;
    L_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_prolong<VT, BT, LL, 2>), gr, bl, 0, s, c.g, c.h, c.CX, two((const VT*)basea, (const VT*)baseb), (const BT*)c.Rc, two((const double*)ea, (const double*)eb), two((const double*)nullptr, (const double*)nullptr), two((double*)outa, (double*)outb), two((const Scalars*)a.sc, (const Scalars*)b.sc)));
  });
}

void launch_vresidual(const Ctx& c, const void* r, bool r_is_f64, const void* x, bool x_is_f64, void* out,
                      hipStream_t s) {
  const dim3 gr = march_grid(c), bl = march_block();
  VC_DISPATCH({
    (void)sizeof(BT);
    (void)sizeof(DVT);
    if (x_is_f64) {
      hipLaunchKernelGGL((k_vresidual<VT, KVT, double, double, CU, 1>), gr, bl, 0, s, c.g, c.st, c.mg, (const KVT*)c.kv, c.bits, one((const double*)r), one((const double*)x), one((VT*)out), one((const Scalars*)c.sc));
    } else {
      hipLaunchKernelGGL((k_vresidual<VT, KVT, double, VT, CU, 1>), gr, bl, 0, s, c.g, c.st, c.mg, (const KVT*)c.kv, c.bits, one((const double*)r), one((const VT*)x), one((VT*)out), one((const Scalars*)c.sc));
    }
    (void)r_is_f64;
  });
}

// out = r - A x for two sides at once (FP64 r and x, the prolonged iterates)
void launch_vresidual_pair(const Ctx& a, const Ctx& b, const double* ra, const double* rb, const double* xa,
                           const double* xb, void* outa, void* outb, hipStream_t s) {
  const Ctx& c = a;
  const dim3 gr((unsigned)(2 * c.mg.blocks)), bl = march_block();
  VC_DISPATCH({
    (void)sizeof(BT);
    (void)sizeof(DVT);
    hipLaunchKernelGGL((k_vresidual<VT, KVT, double, double, CU, 2>), gr, bl, 0, s, c.g, c.st, c.mg, (const KVT*)c.kv,
                       c.bits, two(ra, rb), two(xa, xb), two((VT*)outa, (VT*)outb),
                       two((const Scalars*)a.sc, (const Scalars*)b.sc));
  });
}

void launch_vresidual_prolong(const Ctx& c, const double* r, const void* base, const double* e1, const double* e2,
                              void* out, double* x2, hipStream_t s) {
  const dim3 gr = march_grid(c), bl = march_block();
  VC_DISPATCH({
    (void)sizeof(DVT);
    L_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_vresidual_prolong<VT, KVT, BT, LL, CU>), gr, bl, 0, s, c.g, c.st, c.mg,
                                          c.h, (const KVT*)c.kv, c.bits, r, (const VT*)base, (const BT*)c.Rc, e1, e2,
                                          (VT*)out, x2, (const Scalars*)c.sc));
  });
}

RestrictGeo make_restrict_geo(const Geo& g, const Hier& h, long long resident) {
  RestrictGeo rg{};
  rg.m.ntx = (g.nnx + MX - 1) / MX;
  rg.m.nty = (g.nny + MY - 1) / MY;
  const long long txy = (long long)rg.m.ntx * rg.m.nty;
  if (resident < 1) resident = 1;
  // coarse z-cells per chunk: the fewest rounds of resident workgroups times
  // planes staged per workgroup (as make_march)
  long long best_cost = -1;
  int best = 1;
  for (int czc = 1; czc <= h.ncz; ++czc) {
    const int nzc = (h.ncz + czc - 1) / czc;
    const long long rounds = (txy * nzc + resident - 1) / resident;
    const long long cost = rounds * (czc * h.H + 2);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = czc;
    }
  }
  rg.czc = best;
  rg.m.zc = best * h.H;
  rg.m.nzc = (h.ncz + best - 1) / best;
  rg.m.blocks = ((txy * rg.m.nzc + 7) / 8) * 8;
  rg.nlx = MX / h.H > 0 ? MX / h.H : 1;
  rg.nly = MY / h.H > 0 ? MY / h.H : 1;
  rg.nlz = best;
  rg.slots = txy * rg.m.nzc * rg.nlx * rg.nly * rg.nlz;
  return rg;
}

void launch_vresidual_restrict(const Ctx& c, const double* r, const void* x, double* rc, hipStream_t s) {
  const dim3 gr((unsigned)c.rg.m.blocks), bl = march_block();
  VC_DISPATCH({
    (void)sizeof(DVT);
    L_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_vresidual_restrict<VT, KVT, VT, BT, LL, CU, 1>), gr, bl, 0, s, c.g, c.st, c.h, c.rg, (const KVT*)c.kv, c.bits, one(r), one((const VT*)x), (const BT*)c.Rc, one(c.rpart), one((const Scalars*)c.sc)));
  });
  const long long n = (long long)c.h.ncells * c.h.Lc;
  L_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_restrict_finish<LL>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c.g, c.h, c.rg, (const double*)c.rpart, rc, c.sc));
}

void launch_vresidual_restrict_pair(const Ctx& a, const Ctx& b, const double* ra, const double* rb, const void* xa,
                                    const void* xb, double* rca, double* rcb, hipStream_t s) {
  const Ctx& c = a;
  const dim3 gr((unsigned)(2 * c.rg.m.blocks)), bl = march_block();
  VC_DISPATCH({
    (void)sizeof(DVT);
    L_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_vresidual_restrict<VT, KVT, VT, BT, LL, CU, 2>), gr, bl, 0, s, c.g, c.st, c.h, c.rg, (const KVT*)c.kv, c.bits, two(ra, rb), two((const VT*)xa, (const VT*)xb), (const BT*)c.Rc, two(a.rpart, b.rpart), two((const Scalars*)a.sc, (const Scalars*)b.sc)));
  });
  const long long n = (long long)c.h.ncells * c.h.Lc;
  L_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_restrict_finish<LL>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a.g, a.h, a.rg, (const double*)a.rpart, rca, a.sc));
  L_DISPATCH(c.h.Lc, hipLaunchKernelGGL((k_restrict_finish<LL>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b.g, b.h, b.rg, (const double*)b.rpart, rcb, b.sc));
}

void launch_vc_output(const Ctx& c, const void* a, bool a_is_f64, const void* b, double* z, const double* r,
                      const double* q, int mode, hipStream_t s) {
  const int nb = grid1d(c.g.nn, 256, c.red_blocks);
  Scalars* sc = mode == 2 ? nullptr : c.sc;
  if (c.v_dt == DT_F64)
    hipLaunchKernelGGL((k_vc_output<double, double>), dim3(nb), dim3(256), 0, s, (const double*)a, (const double*)b, z, r, q, c.g.nn, mode, sc, c.partials, c.counter);
  else if (a_is_f64)
    hipLaunchKernelGGL((k_vc_output<double, float>), dim3(nb), dim3(256), 0, s, (const double*)a, (const float*)b, z, r, q, c.g.nn, mode, sc, c.partials, c.counter);
  else
    hipLaunchKernelGGL((k_vc_output<float, float>), dim3(nb), dim3(256), 0, s, (const float*)a, (const float*)b, z, r, q, c.g.nn, mode, sc, c.partials, c.counter);
}

bool smooth_output_fused(const Ctx& c) { return c.cheb.degree == 2; }

void launch_smooth_output(const Ctx& c, const void* in, bool in_is_f64, const double* base, double* z,
                          const double* r, const double* q, int mode, hipStream_t s) {
  const dim3 gr = march_grid(c), bl = march_block();
#define SO(IT_, MD) hipLaunchKernelGGL((k_cheb2_out<VT, KVT, IT_, DVT, CU, MD, 1>), gr, bl, 0, s, c.g, c.st, c.mg, (const KVT*)c.kv, one((const IT_*)in), (const DVT*)c.dinv, c.cheb, one(base), one(z), one(r), one(q), one(c.sc), one(c.partials), one(c.counter))
#define SO_M(IT_) do { if (mode == 0) SO(IT_, 0); else if (mode == 1) SO(IT_, 1); else SO(IT_, 2); } while (0)
  VC_DISPATCH({
    (void)sizeof(BT);
    if (in_is_f64) SO_M(double); else SO_M(VT);
  });
#undef SO_M
#undef SO
}

// The fused post-smoother and output for two sides (V-cycle vectors in, PCG
// reductions of `mode` 0 or 1 per side).
void launch_smooth_output_pair(const Ctx& a, const Ctx& b, const void* ina, const void* inb, const double* basea,
                               const double* baseb, double* za, double* zb, const double* ra, const double* rb,
                               const double* qa, const double* qb, int mode, hipStream_t s) {
  const Ctx& c = a;
  const dim3 gr((unsigned)(2 * c.mg.blocks)), bl = march_block();
#define SOP(MD) hipLaunchKernelGGL((k_cheb2_out<VT, KVT, VT, DVT, CU, MD, 2>), gr, bl, 0, s, c.g, c.st, c.mg, (const KVT*)c.kv, two((const VT*)ina, (const VT*)inb), (const DVT*)c.dinv, c.cheb, two(basea, baseb), two(za, zb), two(ra, rb), two(qa, qb), two(a.sc, b.sc), two(a.partials, b.partials), two(a.counter, b.counter))
  VC_DISPATCH({
    (void)sizeof(BT);
    if (mode == 0) SOP(0); else SOP(1);
  });
#undef SOP
}

void launch_sensitivity(const Ctx& c, const double* T, const double* lam, double* dc, hipStream_t s) {
  const dim3 gr((unsigned)((c.g.ne + 255) / 256)), bl(256);
  if (c.rho_dt == DT_F64)
    hipLaunchKernelGGL((k_sensitivity<double, false>), gr, bl, 0, s, c.g, c.st, (const double*)c.rho, c.mat, T, lam,
                       c.bits, 0.0, dc);
  else
    hipLaunchKernelGGL((k_sensitivity<float, false>), gr, bl, 0, s, c.g, c.st, (const float*)c.rho, c.mat, T, lam,
                       c.bits, 0.0, dc);
}

void launch_sensitivity_heat_source(const Ctx& c, const double* T, const double* lam, double f0, double* dc,
                                    hipStream_t s) {
  const dim3 gr((unsigned)((c.g.ne + 255) / 256)), bl(256);
  if (c.rho_dt == DT_F64)
    hipLaunchKernelGGL((k_sensitivity<double, true>), gr, bl, 0, s, c.g, c.st, (const double*)c.rho, c.mat, T, lam,
                       c.bits, f0, dc);
  else
    hipLaunchKernelGGL((k_sensitivity<float, true>), gr, bl, 0, s, c.g, c.st, (const float*)c.rho, c.mat, T, lam,
                       c.bits, f0, dc);
}

void launch_heat_source_load(const Ctx& c, double f0, double* f, hipStream_t s) {
  const dim3 gr((unsigned)((c.g.nn + 255) / 256)), bl(256);
  if (c.rho_dt == DT_F64)
    hipLaunchKernelGGL((k_heat_source_load<double>), gr, bl, 0, s, c.g, (const double*)c.rho, c.mat.p, f0, f);
  else
    hipLaunchKernelGGL((k_heat_source_load<float>), gr, bl, 0, s, c.g, (const float*)c.rho, c.mat.p, f0, f);
}

void launch_element_load(const Geo& g, const double* src, double sconst, double* f, hipStream_t s) {
  hipLaunchKernelGGL(k_element_load, dim3((unsigned)((g.nn + 255) / 256)), dim3(256), 0, s, g, src, sconst, f);
}

void launch_prolong_nodal(int nx, int ny, int nz, const double* tc, double* tf, hipStream_t s) {
  const long long n = (2LL * nx + 1) * (2LL * ny + 1) * (2LL * nz + 1);
  hipLaunchKernelGGL(k_prolong_nodal, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, nx, ny, nz, tc, tf);
}

void launch_stream_ceiling(const double* x, const double* k, double* y, long long nn, long long ne, hipStream_t s) {
  const long long nn2 = nn / 2, ne2 = ne / 2;
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const dim3 gr((unsigned)std::max<long long>(1, std::min<long long>((nn2 + 255) / 256, 16LL * cus))), bl(256);
  hipLaunchKernelGGL(k_stream_ceiling, gr, bl, 0, s, (const dvec2*)x, (const dvec2*)k, (dvec2*)y, nn2, ne2);
}

void launch_prolong_element(int nx, int ny, int nz, const void* rc, void* rf, int dt, hipStream_t s) {
  const long long n = 8LL * nx * ny * nz;
  const dim3 gr((unsigned)((n + 255) / 256)), bl(256);
  if (dt == DT_F64) hipLaunchKernelGGL((k_prolong_element<double>), gr, bl, 0, s, nx, ny, nz, (const double*)rc, (double*)rf);
  else if (dt == DT_F32) hipLaunchKernelGGL((k_prolong_element<float>), gr, bl, 0, s, nx, ny, nz, (const float*)rc, (float*)rf);
  else hipLaunchKernelGGL((k_prolong_element<uint16_t>), gr, bl, 0, s, nx, ny, nz, (const uint16_t*)rc, (uint16_t*)rf);
}

}  // namespace msmg
