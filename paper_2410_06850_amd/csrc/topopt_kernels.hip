// Design-update kernels around the solve: the density filter and the
// optimality-criteria (OC) update used by the topology-optimisation loop.
#include <cmath>
#include <mutex>

#include "common.h"
#include "internal.h"

namespace msmg {

// ---------------------------------------------------------------------------
// Density filter with the linear hat weights w(e, f) = max(0, r - |c_e - c_f|)
// (distances between element centres, in elements).
//   forward:   out_e = sum_f w(e,f) in_f / W_e,  W_e = sum_f w(e,f)
//   transpose: out_f = sum_e w(e,f) in_e / W_e   (the chain rule of forward)
// Sums run over elements inside the mesh; R = the largest offset with w > 0.
MSMG_DEV double hat(double r, int dx, int dy, int dz) {
  const double d = sqrt(double(dx * dx + dy * dy + dz * dz));
  return d < r ? r - d : 0.0;
}

MSMG_DEV double filter_weight_sum(int nx, int ny, int nz, int R, double r, int i, int j, int k) {
  double W = 0.0;
  for (int dz = -R; dz <= R; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const int a = i + dx, b = j + dy, c = k + dz;
        if (a < 0 || a >= nx || b < 0 || b >= ny || c < 0 || c >= nz) continue;
        W += hat(r, dx, dy, dz);
      }
  return W;
}

template <bool TRANSPOSE>
__global__ void k_density_filter(int nx, int ny, int nz, int R, double r, const double* __restrict__ in,
                                 double* __restrict__ out) {
  const long long ne = (long long)nx * ny * nz;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne; e += (long long)gridDim.x * blockDim.x) {
    const int i = int(e % nx), j = int((e / nx) % ny), k = int(e / ((long long)nx * ny));
    double acc = 0.0, W = 0.0;
    for (int dz = -R; dz <= R; ++dz)
      for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
          const int a = i + dx, b = j + dy, c = k + dz;
          if (a < 0 || a >= nx || b < 0 || b >= ny || c < 0 || c >= nz) continue;
          const double w = hat(r, dx, dy, dz);
          if (w == 0.0) continue;
          const long long f = ((long long)c * ny + b) * nx + a;
          if (TRANSPOSE)
            acc += w * in[f] / filter_weight_sum(nx, ny, nz, R, r, a, b, c);
          else
            acc += w * in[f];
          W += w;
        }
    out[e] = TRANSPOSE ? acc : acc / W;
  }
}

void launch_density_filter(int nx, int ny, int nz, double r, const double* in, double* out, bool transpose,
                           hipStream_t s) {
  int R = int(r);
  if (double(R) >= r) R -= 1;  // offsets with |d| < r
  const long long ne = (long long)nx * ny * nz;
  const dim3 gr(grid1d(ne, 256, 65536)), bl(256);
  if (transpose)
    hipLaunchKernelGGL(k_density_filter<true>, gr, bl, 0, s, nx, ny, nz, R, r, in, out);
  else
    hipLaunchKernelGGL(k_density_filter<false>, gr, bl, 0, s, nx, ny, nz, R, r, in, out);
}

// ---------------------------------------------------------------------------
// OC update: x_new(lambda) = clamp(x (-dc / (lambda dv))^eta, max(x_min, x - m), min(1, x + m))
// with lambda chosen so that sum x_new = volume (the volume is decreasing in
// lambda).  The multiplier is bracketed on a log scale: every pass evaluates
// the volume at OC_NL points of the current bracket in one sweep over the
// design and keeps the sub-interval that holds the target.
constexpr int OC_NL = 32;
constexpr int OC_BLOCKS = 256;

struct OCState {
  double log_lo, log_hi;  // bracket of log(lambda)
};

MSMG_DEV double oc_new(double x, double dc, double dv, double lam, double move, double eta, double xmin) {
  const double lo = fmax(xmin, x - move), hi = fmin(1.0, x + move);
  const double B = fmax(0.0, -dc) / (lam * dv);
  double v = x * pow(B, eta);
  v = fmin(fmax(v, lo), hi);
  return v;
}

__global__ void k_oc_init(OCState* st, double log_lo, double log_hi, unsigned* counter) {
  st->log_lo = log_lo;
  st->log_hi = log_hi;
  if (counter) *counter = 0u;
}

__global__ void k_oc_volumes(long long ne, const double* __restrict__ x, const double* __restrict__ dc,
                             const double* __restrict__ dv, double move, double eta, double xmin, double target,
                             OCState* st, double* partials, unsigned* counter) {
  __shared__ double red[OC_NL * 16];
  const double llo = st->log_lo, lhi = st->log_hi;
  double lam[OC_NL];
#pragma unroll
  for (int q = 0; q < OC_NL; ++q) lam[q] = exp(llo + (lhi - llo) * q / double(OC_NL - 1));
  double v[OC_NL];
#pragma unroll
  for (int q = 0; q < OC_NL; ++q) v[q] = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne; e += (long long)gridDim.x * blockDim.x) {
    const double xe = x[e], de = dc[e], ve = dv[e];
#pragma unroll
    for (int q = 0; q < OC_NL; ++q) v[q] += oc_new(xe, de, ve, lam[q], move, eta, xmin);
  }
  grid_reduce<OC_NL>(v, red, partials, counter, gridDim.x, blockIdx.x, [&](double* vol) {
    // vol[q] is non-increasing in q; keep [lambda_q, lambda_{q+1}] with
    // vol[q] >= target >= vol[q+1] (the ends when the target is outside)
    int q = 0;
    while (q < OC_NL - 2 && vol[q + 1] >= target) ++q;
    const double step = (lhi - llo) / double(OC_NL - 1);
    st->log_lo = llo + step * q;
    st->log_hi = llo + step * (q + 1);
  });
}

__global__ void k_oc_apply(long long ne, const double* __restrict__ x, const double* __restrict__ dc,
                           const double* __restrict__ dv, double move, double eta, double xmin,
                           const OCState* st, double* __restrict__ xnew, double* lam_out) {
  const double lam = exp(0.5 * (st->log_lo + st->log_hi));
  if (lam_out && blockIdx.x == 0 && threadIdx.x == 0) *lam_out = lam;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne; e += (long long)gridDim.x * blockDim.x)
    xnew[e] = oc_new(x[e], dc[e], dv[e], lam, move, eta, xmin);
}

void launch_oc_update(long long ne, const double* x, const double* dc, const double* dv, double volume, double move,
                      double eta, double xmin, double* xnew, double* lam_out, void* state, double* partials,
                      unsigned* counter, int passes, hipStream_t s) {
  OCState* st = (OCState*)state;
  hipLaunchKernelGGL(k_oc_init, dim3(1), dim3(1), 0, s, st, std::log(1e-40), std::log(1e40), (unsigned*)nullptr);
  for (int it = 0; it < passes; ++it)
    hipLaunchKernelGGL(k_oc_volumes, dim3(OC_BLOCKS), dim3(256), 0, s, ne, x, dc, dv, move, eta, xmin, volume, st,
                       partials, counter);
  hipLaunchKernelGGL(k_oc_apply, dim3(grid1d(ne, 256, 65536)), dim3(256), 0, s, ne, x, dc, dv, move, eta, xmin, st,
                     xnew, lam_out);
}

// ---------------------------------------------------------------------------
// Objective values and chain-rule scalings of the optimisation loop: a^T b in
// a fixed order (the compliance f^T T, the mean temperature w^T T), and
// y = c s x with s a device scalar (an upstream gradient).

__global__ void k_dot(const double* __restrict__ a, const double* __restrict__ b, long long n, double* out,
                      double* partials, unsigned* counter) {
  __shared__ double red[16];
  double s[1] = {0.0};
  for (long long m = blockIdx.x * (long long)blockDim.x + threadIdx.x; m < n; m += (long long)gridDim.x * blockDim.x)
    s[0] += a[m] * b[m];
  grid_reduce<1>(s, red, partials, counter, gridDim.x, blockIdx.x, [&](double* t) { *out = t[0]; });
}

__global__ void k_scale(const double* __restrict__ x, long long n, double c, const double* __restrict__ sdev,
                        double* __restrict__ y) {
  const double f = sdev ? c * sdev[0] : c;
  for (long long m = blockIdx.x * (long long)blockDim.x + threadIdx.x; m < n; m += (long long)gridDim.x * blockDim.x)
    y[m] = f * x[m];
}

void launch_dot(const double* a, const double* b, long long n, double* out, double* partials, unsigned* counter,
                int max_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_dot, dim3(grid1d(n, 256, max_blocks)), dim3(256), 0, s, a, b, n, out, partials, counter);
}

void launch_scale(const double* x, long long n, double c, const double* sdev, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(grid1d(n, 256, 8192)), dim3(256), 0, s, x, n, c, sdev, y);
}

// ---------------------------------------------------------------------------
// Method of moving asymptotes (Svanberg 1987; the parameter conventions of his
// 2007 note on MMA and GCMMA), the optimiser of the paper's section 2.3, for the
// one linear volume constraint f1(x) = dv . x / N - vf <= 0 on
// x_min <= x <= x_max.  The separable convex approximation at x has
//   p = (U - x)^2 (1.001 g+ + 0.001 g- + raa0 / span),
//   q = (x - L)^2 (0.001 g+ + 1.001 g- + raa0 / span)
// per function (g+ / g- the positive / negative part of its derivative); the
// approximate problem (with the elastic variable y, weights c = 1000, d = 1) is
// solved through its dual: for a multiplier lam every x_e minimises
// (p0 + lam p1) / (U - x) + (q0 + lam q1) / (x - L) on [alpha, beta] in closed
// form, and the dual slope (approximate constraint minus y = max(0, lam - c))
// is non-increasing in lam.  lam = 0 when the slope at 0 is not positive;
// otherwise its root is bracketed on a log scale as in the OC update.
constexpr double MMA_ASYINIT = 0.5, MMA_ASYINCR = 1.2, MMA_ASYDECR = 0.7, MMA_ALBEFA = 0.1, MMA_RAA0 = 1e-5,
                 MMA_C = 1000.0;

struct MMAState {
  double log_lo, log_hi;  // bracket of log(lambda)
  int zero;               // 1: the constraint is inactive, lambda = 0
};
static_assert(sizeof(MMAState) <= 64, "fits the handle's 64-byte state slot");

// Asymptotes of update `it` (0-based) from the last two steps; in/out low, upp.
__global__ void k_mma_asymptotes(int it, long long ne, const double* __restrict__ x, const double* __restrict__ x1,
                                 const double* __restrict__ x2, double* __restrict__ low, double* __restrict__ upp,
                                 double span) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne; e += (long long)gridDim.x * blockDim.x) {
    const double xe = x[e];
    double lo, up;
    if (it < 2) {
      lo = xe - MMA_ASYINIT * span;
      up = xe + MMA_ASYINIT * span;
    } else {
      const double sg = (xe - x1[e]) * (x1[e] - x2[e]);
      const double gam = sg < 0.0 ? MMA_ASYDECR : (sg > 0.0 ? MMA_ASYINCR : 1.0);
      lo = xe - gam * (x1[e] - low[e]);
      up = xe + gam * (upp[e] - x1[e]);
      lo = fmin(fmax(lo, xe - 10.0 * span), xe - 0.01 * span);
      up = fmin(fmax(up, xe + 0.01 * span), xe + 10.0 * span);
    }
    low[e] = lo;
    upp[e] = up;
  }
}

// The element's share of the approximate problem at x with asymptotes lo, up.
struct MMAElem {
  double p0, q0, p1, q1, lo, up, alpha, beta, base;  // base: the x-independent part of its constraint term
};

MSMG_DEV MMAElem mma_elem(double x, double lo, double up, double df0, double g1, double move, double xmin,
                          double xmax) {
  MMAElem m;
  const double span = xmax - xmin, reg = MMA_RAA0 / span;
  const double gp0 = fmax(df0, 0.0), gm0 = fmax(-df0, 0.0), gp1 = fmax(g1, 0.0), gm1 = fmax(-g1, 0.0);
  const double du = up - x, dl = x - lo;
  m.p0 = du * du * (1.001 * gp0 + 0.001 * gm0 + reg);
  m.q0 = dl * dl * (0.001 * gp0 + 1.001 * gm0 + reg);
  m.p1 = du * du * (1.001 * gp1 + 0.001 * gm1 + reg);
  m.q1 = dl * dl * (0.001 * gp1 + 1.001 * gm1 + reg);
  m.lo = lo;
  m.up = up;
  m.alpha = fmax(fmax(xmin, lo + MMA_ALBEFA * dl), x - move * span);
  m.beta = fmin(fmin(xmax, up - MMA_ALBEFA * du), x + move * span);
  // constraint term at x_new minus its value at x plus the linear part g1 x
  m.base = g1 * x - (m.p1 / du + m.q1 / dl);
  return m;
}

MSMG_DEV double mma_x(const MMAElem& m, double lam) {
  const double P = sqrt(m.p0 + lam * m.p1), Q = sqrt(m.q0 + lam * m.q1);
  return fmin(fmax((P * m.lo + Q * m.up) / (P + Q), m.alpha), m.beta);
}

MSMG_DEV double mma_con(const MMAElem& m, double xn) { return m.p1 / (m.up - xn) + m.q1 / (xn - m.lo) + m.base; }

// Dual slope at lambda = 0: decides whether the constraint is active.
__global__ void k_mma_slope0(long long ne, const double* __restrict__ x, const double* __restrict__ low,
                             const double* __restrict__ upp, const double* __restrict__ df0,
                             const double* __restrict__ dv, double inv_n, double vf, double move, double xmin,
                             double xmax, MMAState* st, double* partials, unsigned* counter) {
  __shared__ double red[16];
  double v[1] = {0.0};
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne; e += (long long)gridDim.x * blockDim.x) {
    const MMAElem m = mma_elem(x[e], low[e], upp[e], df0[e], dv[e] * inv_n, move, xmin, xmax);
    v[0] += mma_con(m, mma_x(m, 0.0));
  }
  grid_reduce<1>(v, red, partials, counter, gridDim.x, blockIdx.x, [&](double* t) {
    st->zero = (t[0] - vf <= 0.0) ? 1 : 0;
    st->log_lo = log(1e-40);
    st->log_hi = log(1e40);
  });
}

// One bracketing pass: the dual slope at OC_NL points of the bracket; keeps the
// sub-interval where it changes sign (the ends when it does not).
__global__ void k_mma_slopes(long long ne, const double* __restrict__ x, const double* __restrict__ low,
                             const double* __restrict__ upp, const double* __restrict__ df0,
                             const double* __restrict__ dv, double inv_n, double vf, double move, double xmin,
                             double xmax, MMAState* st, double* partials, unsigned* counter) {
  __shared__ double red[OC_NL * 16];
  if (st->zero) return;  // uniform
  const double llo = st->log_lo, lhi = st->log_hi;
  double lam[OC_NL], v[OC_NL];
#pragma unroll
  for (int q = 0; q < OC_NL; ++q) {
    lam[q] = exp(llo + (lhi - llo) * q / double(OC_NL - 1));
    v[q] = 0.0;
  }
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne; e += (long long)gridDim.x * blockDim.x) {
    const MMAElem m = mma_elem(x[e], low[e], upp[e], df0[e], dv[e] * inv_n, move, xmin, xmax);
#pragma unroll
    for (int q = 0; q < OC_NL; ++q) v[q] += mma_con(m, mma_x(m, lam[q]));
  }
  grid_reduce<OC_NL>(v, red, partials, counter, gridDim.x, blockIdx.x, [&](double* sum) {
    // slope[q] = sum[q] - vf - max(0, lam_q - c), non-increasing in q; keep
    // [lam_q, lam_{q+1}] with slope[q] > 0 >= slope[q+1]
    auto slope = [&](int q) { return sum[q] - vf - fmax(0.0, exp(llo + (lhi - llo) * q / double(OC_NL - 1)) - MMA_C); };
    int q = 0;
    while (q < OC_NL - 2 && slope(q + 1) > 0.0) ++q;
    const double step = (lhi - llo) / double(OC_NL - 1);
    st->log_lo = llo + step * q;
    st->log_hi = llo + step * (q + 1);
  });
}

__global__ void k_mma_apply(long long ne, const double* __restrict__ x, const double* __restrict__ low,
                            const double* __restrict__ upp, const double* __restrict__ df0,
                            const double* __restrict__ dv, double inv_n, double move, double xmin, double xmax,
                            const MMAState* st, double* __restrict__ xnew, double* lam_out) {
  const double lam = st->zero ? 0.0 : exp(0.5 * (st->log_lo + st->log_hi));
  if (lam_out && blockIdx.x == 0 && threadIdx.x == 0) *lam_out = lam;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne; e += (long long)gridDim.x * blockDim.x)
    xnew[e] = mma_x(mma_elem(x[e], low[e], upp[e], df0[e], dv[e] * inv_n, move, xmin, xmax), lam);
}

void launch_mma_update(int it, long long ne, const double* x, const double* x1, const double* x2, double* low,
                       double* upp, const double* df0, const double* dv, double vf, double move, double xmin,
                       double xmax, double* xnew, double* lam_out, void* state, double* partials, unsigned* counter,
                       int passes, hipStream_t s) {
  MMAState* st = (MMAState*)state;
  const dim3 g1d(grid1d(ne, 256, 65536)), b(256);
  const double inv_n = 1.0 / double(ne);
  hipLaunchKernelGGL(k_mma_asymptotes, g1d, b, 0, s, it, ne, x, x1, x2, low, upp, xmax - xmin);
  hipLaunchKernelGGL(k_mma_slope0, dim3(OC_BLOCKS), b, 0, s, ne, x, low, upp, df0, dv, inv_n, vf, move, xmin, xmax,
                     st, partials, counter);
  for (int p = 0; p < passes; ++p)
    hipLaunchKernelGGL(k_mma_slopes, dim3(OC_BLOCKS), b, 0, s, ne, x, low, upp, df0, dv, inv_n, vf, move, xmin,
                       xmax, st, partials, counter);
  hipLaunchKernelGGL(k_mma_apply, g1d, b, 0, s, ne, x, low, upp, df0, dv, inv_n, move, xmin, xmax, st, xnew,
                     lam_out);
}

// ---------------------------------------------------------------------------
// The same update with its scratch (block partials of the volume sweeps, the
// reduction counter, the multiplier bracket) in a fixed device array instead
// of a handle: nothing is allocated, so callers that may not allocate (graph
// capture, serving loops) can use it.  The array's size does not depend on the
// design size: the volume sweeps always run OC_BLOCKS workgroups.  Each device
// holds its own copy; calls on one device share it.
constexpr size_t OC_SCRATCH_COUNTER = 0, OC_SCRATCH_STATE = 256, OC_SCRATCH_PARTIALS = 512;
constexpr size_t OC_SCRATCH_BYTES = OC_SCRATCH_PARTIALS + sizeof(double) * OC_NL * OC_BLOCKS;
static __device__ __align__(256) unsigned char scratch[OC_SCRATCH_BYTES];

static_assert(sizeof(OCState) <= OC_SCRATCH_PARTIALS - OC_SCRATCH_STATE, "state slot");

// Device address of this device's scratch array, looked up once per device
// (the array's name is only a host-side stand-in).
constexpr int OC_MAX_DEVICES = 64;
static std::mutex oc_scratch_mutex;
static void* oc_scratch_addr[OC_MAX_DEVICES] = {};

hipError_t oc_scratch_device_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= OC_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(oc_scratch_mutex);
  if (!oc_scratch_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    oc_scratch_addr[dev] = p;
  }
  *out = oc_scratch_addr[dev];
  return hipSuccess;
}

size_t oc_scratch_bytes() { return OC_SCRATCH_BYTES; }

void launch_oc_update_scratch(long long ne, const double* x, const double* dc, const double* dv, double volume,
                              double move, double eta, double xmin, double* xnew, double* lam_out, void* scratch_ptr,
                              int passes, hipStream_t s) {
  char* base = static_cast<char*>(scratch_ptr);
  unsigned* counter = reinterpret_cast<unsigned*>(base + OC_SCRATCH_COUNTER);
  OCState* st = reinterpret_cast<OCState*>(base + OC_SCRATCH_STATE);
  double* partials = reinterpret_cast<double*>(base + OC_SCRATCH_PARTIALS);
  // the counter is cleared by a kernel (not a memset), so the sequence can be
  // captured in a graph
  hipLaunchKernelGGL(k_oc_init, dim3(1), dim3(1), 0, s, st, std::log(1e-40), std::log(1e40), counter);
  for (int it = 0; it < passes; ++it)
    hipLaunchKernelGGL(k_oc_volumes, dim3(OC_BLOCKS), dim3(256), 0, s, ne, x, dc, dv, move, eta, xmin, volume, st,
                       partials, counter);
  hipLaunchKernelGGL(k_oc_apply, dim3(grid1d(ne, 256, 65536)), dim3(256), 0, s, ne, x, dc, dv, move, eta, xmin, st,
                     xnew, lam_out);
}

}  // namespace msmg
