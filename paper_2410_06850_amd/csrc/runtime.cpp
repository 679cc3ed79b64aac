// Host runtime of the MsMG library: handle, hierarchy plan, memory plan,
// set-up orchestration, the PCG driver and the C ABI of include/msmg.h.
//
// The PCG loop keeps every scalar on the device; the host enqueues batches of
// iterations and polls one small status record between batches.  Kernels of a
// batch that start after convergence return immediately (device `done` flag).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../../include/msmg.h"
#include "internal.h"
#include "setup.h"

using namespace msmg;

static thread_local std::string g_last_error;

static int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess)                                                                    \
      return fail(MSMG_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));             \
  } while (0)

// The vectors, scalars and reduction scratch of one right-hand side's PCG.
struct VecSet {
  double *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr, *b = nullptr;
  float* xlo = nullptr;  // low part of the double-double iterate (|lo| <= ulp(hi) / 2, FP32)
  // V-cycle vectors (v_dt; v_r2 FP64) and coarse vectors
  void *v_r1 = nullptr, *v_r2 = nullptr, *v_res = nullptr;
  void *c_rc = nullptr, *c_x0 = nullptr, *c_t = nullptr, *c_x1 = nullptr, *c_d = nullptr;
  double *rcc = nullptr, *ecc = nullptr;
  double* rpart = nullptr;  // partial sums of the fused residual + restriction
  Scalars* sc = nullptr;
  Scalars* sc_host = nullptr;  // pinned
  double* partials = nullptr;
  unsigned* counter = nullptr;
};

struct msmg_handle {
  int device = 0;
  msmg_options opt{};
  Geo g{};
  Stencil st{};
  Hier hier{};
  int CX = 1;
  long long ntiles = 0;
  double lam_bound = 0.0;  // upper bound of the level-1 standard-form spectrum
  Material mat{};
  int rho_dt = DT_F64, kv_dt = DT_F64, v_dt = DT_F64, b_dt = DT_F64, a_dt = DT_F64, dv_dt = DT_F64;
  int rho_store_dt = DT_F64;  // storage of the canonical density copy
  bool mg = true;
  bool tpfa = false;                     // cell-centred two-point flux discretisation
  uint8_t* dface = nullptr;              // its Dirichlet face flags (one byte per cell)
  unsigned long long* fcount = nullptr;  // flag counts of the last set-up: valid, misplaced

  // density, mask, fixed values
  void* rho = nullptr;
  double* kc = nullptr;   // FP64 element conductivities (FP64 density only)
  void* kv = nullptr;     // element conductivities read by the cycle (kv_dt; may alias kc)
  uint32_t* bits = nullptr;
  double* tfix = nullptr;
  bool has_tfix = false;
  void* dinv = nullptr;

  // level 1 / 2
  double* Rc64 = nullptr;
  void* Rcs = nullptr;  // stored basis (aliases Rc64 for FP64)
  double* Ac64 = nullptr;
  void* Acv = nullptr;
  double* AcDinv64 = nullptr;
  void* AcDinvv = nullptr;
  double* G64 = nullptr;
  double* Rcc64 = nullptr;
  void* Rccv = nullptr;
  int* cc_ptr = nullptr;
  int* cc_dofs = nullptr;
  int* dof_cc = nullptr;
  int* dof_loc = nullptr;
  double* Acc = nullptr;  // becomes A_cc^-1 in place
  double* evals = nullptr;
  int* cell_status = nullptr;
  double* cc_evals = nullptr;
  int* cc_status = nullptr;
  int n_c = 0, n_cc = 0, max_cc_dofs = 0, max_cell_nodes = 0;
  std::vector<int> h_cc_ptr;

  // per right-hand side: vs[0] for every solve, vs[1] for the second side of
  // a batched pair (allocated with options.pair_rhs)
  VecSet vs[2];
  void *v_t0 = nullptr, *v_t1 = nullptr;  // Chebyshev scratch for degrees > 2 (side 0)
  int l1_blocks = 0;         // workgroups of the grid-synchronised coarse-level kernel (0: separate launches)
  unsigned* l1_bar = nullptr;  // its barrier words
  RestrictGeo rg{};          // fused residual + restriction of the cycle
  int red_blocks = 4096;
  long long march_resident = 2048;  // marching workgroups resident at once (queried at create)
  long long apply_resident = 768;   // the same for the LDS-queue apply
  bool has_basis = false;           // Rc64 holds the basis of the last completed set-up
  bool basis_live = false;          // lean memory: Rc64 not yet overwritten by PCG vectors
  long long partial_slots = 0;
  void* oc_state = nullptr;  // bracket of the OC multiplier

  SetupScratch scratch{};
  bool setup_done = false;
  double setup_ms = 0.0;
  int eig_unconverged = 0, cc_unconverged = 0, eig_ties = 0;
  TuneChoice tune[2]{};  // level-1 launch shapes per cell class
  std::vector<void*> allocs;
  std::vector<hipEvent_t> events;  // timing mode: 4 per timed iteration
  std::vector<hipEvent_t> setup_events;  // timing mode: set-up phases (SETUP_EVENTS)
  double setup_phase_ms[4] = {0, 0, 0, 0};
  double setup_dense_ms = 0.0, setup_dense_gflop = 0.0;
};

// coarse unknowns up to which levels 1 and 2 run as one grid-synchronised launch
static constexpr int kLevel1MaxCoarse = 1 << 18;

static size_t dt_size(int dt) { return dt == DT_F64 ? 8 : (dt == DT_F32 ? 4 : 2); }

// --------------------------------------------------------------------------
// plan

struct Plan {
  Hier h;
  int CX;
  long long ntiles;
  int n_c, n_cc, max_cell_nodes, max_cc_dofs;
  std::vector<int> cc_ptr;  // host, ncc+1
};

// extra = 1: unknowns are the nodes (n + 1 per axis); 0: the cells (TPFA)
static int make_plan(int nx, int ny, int nz, const msmg_options& o, Plan& P, int extra = 1) {
  if (nx < 1 || ny < 1 || nz < 1) return fail(MSMG_EINVAL, "mesh sizes must be positive");
  if (o.H < 2) return fail(MSMG_EINVAL, "H must be >= 2");
  if (o.H > 16) return fail(MSMG_EINVAL, "H must be <= 16");
  if (nx < o.H || ny < o.H || nz < o.H) return fail(MSMG_EINVAL, "each axis needs at least H elements (cells)");
  if (o.sd < 1) return fail(MSMG_EINVAL, "sd must be >= 1");
  if (o.Lc < 1 || o.Lc > LC_MAX) return fail(MSMG_EINVAL, "Lc must be in 1..8");
  if (o.Lcc < 1) return fail(MSMG_EINVAL, "Lcc must be >= 1");
  if (o.cheb_degree < 1 || o.cheb_degree > CHEB_MAX) return fail(MSMG_EINVAL, "cheb_degree must be in 1..16");
  if (!(o.cheb_hi > o.cheb_lo) || !(o.cheb_lo > 0.0)) return fail(MSMG_EINVAL, "need 0 < cheb_lo < cheb_hi");
  Hier& h = P.h;
  h.H = o.H;
  h.ncx = nx / o.H;
  h.ncy = ny / o.H;
  h.ncz = nz / o.H;
  h.ncells = h.ncx * h.ncy * h.ncz;
  h.Lc = o.Lc;
  h.sd = o.sd;
  h.nccx = std::max(1, h.ncx / o.sd);
  h.nccy = std::max(1, h.ncy / o.sd);
  h.nccz = std::max(1, h.ncz / o.sd);
  h.ncc = h.nccx * h.nccy * h.nccz;
  h.Lcc = o.Lcc;
  auto ext = [&](int c, int nc, int nn) { return cell_end(c, o.H, nc, nn) - cell_begin(c, o.H); };
  const int mx = ext(h.ncx - 1, h.ncx, nx + extra), my = ext(h.ncy - 1, h.ncy, ny + extra),
            mz = ext(h.ncz - 1, h.ncz, nz + extra);
  P.max_cell_nodes = mx * my * mz;
  if (mx > 16 || my > 16 || mz > 16) return fail(MSMG_EINVAL, "a coarse cell exceeds 16 nodes per axis");
  P.CX = std::max(1, 64 / o.H);
  P.ntiles = (long long)((h.ncx + P.CX - 1) / P.CX) * h.ncy * h.ncz;
  // cc cells: coarse dofs grouped; local order = cells of the group in x-fastest order, then l
  P.cc_ptr.assign(h.ncc + 1, 0);
  int maxd = 0;
  h.max_cc_cells = 0;
  for (int jz = 0; jz < h.nccz; ++jz)
    for (int jy = 0; jy < h.nccy; ++jy)
      for (int jx = 0; jx < h.nccx; ++jx) {
        const int J = (jz * h.nccy + jy) * h.nccx + jx;
        const int cxs = group_end(jx, h.sd, h.nccx, h.ncx) - group_begin(jx, h.sd);
        const int cys = group_end(jy, h.sd, h.nccy, h.ncy) - group_begin(jy, h.sd);
        const int czs = group_end(jz, h.sd, h.nccz, h.ncz) - group_begin(jz, h.sd);
        const int ncl = cxs * cys * czs;
        h.max_cc_cells = std::max(h.max_cc_cells, ncl);
        P.cc_ptr[J + 1] = ncl * h.Lc;
        maxd = std::max(maxd, ncl * h.Lc);
      }
  for (int J = 0; J < h.ncc; ++J) P.cc_ptr[J + 1] += P.cc_ptr[J];
  P.n_c = h.ncells * h.Lc;
  P.max_cc_dofs = maxd;
  int lcc_eff = 0;
  for (int J = 0; J < h.ncc; ++J) lcc_eff += std::min(h.Lcc, P.cc_ptr[J + 1] - P.cc_ptr[J]);
  (void)lcc_eff;
  if (h.Lcc > maxd) h.Lcc = maxd;
  P.n_cc = h.ncc * h.Lcc;
  if (P.n_cc > 72000) return fail(MSMG_EINVAL, "coarse-coarse dimension too large for the dense level-2 solve");
  if (o.lc_threshold > 0.0) {
    // an adaptive basis keeps at least one vector per coarse cell, so every
    // coarse-coarse cell must hold as many coarse cells as its subspace block
    // has vectors, or that block would be rank deficient
    int m = o.cc_block ? o.cc_block : std::min(32, h.Lcc + 15);
    if (m < h.Lcc + 1) m = std::min(32, h.Lcc + 1);
    const long long least = (long long)std::min(h.ncx, o.sd) * std::min(h.ncy, o.sd) * std::min(h.ncz, o.sd);
    if (least < m)
      return fail(MSMG_EINVAL, "an adaptive basis (lc_threshold > 0) needs at least " + std::to_string(m) +
                                   " coarse cells per coarse-coarse cell (sd >= 4 for L_cc = 17)");
    if (o.Lc > 7) return fail(MSMG_EINVAL, "an adaptive basis takes Lc <= 7");
  }
  return MSMG_OK;
}

static Geo make_geo(int nx, int ny, int nz, double lx, double ly, double lz, bool cells = false) {
  Geo g;
  g.nx = nx; g.ny = ny; g.nz = nz;
  // cell unknowns (TPFA): the "node" grid is the cell grid
  const int e = cells ? 0 : 1;
  g.nnx = nx + e; g.nny = ny + e; g.nnz = nz + e;
  g.nn = (long long)g.nnx * g.nny * g.nnz;
  g.ne = (long long)nx * ny * nz;
  g.hx = lx / nx; g.hy = ly / ny; g.hz = lz / nz;
  g.vol = g.hx * g.hy * g.hz;
  return g;
}

// Unit-k element matrix entries by the set of differing coordinates:
// K0[a][b] = wx S(dx)M(dy)M(dz) + wy M(dx)S(dy)M(dz) + wz M(dx)M(dy)S(dz),
// S(0)=1, S(1)=-1, M(0)=1/3, M(1)=1/6, wx = hy hz / hx (etc.).
static Stencil make_stencil(const Geo& g, double* lam_max_k0) {
  const double wx = g.hy * g.hz / g.hx, wy = g.hx * g.hz / g.hy, wz = g.hx * g.hy / g.hz;
  auto S = [](int d) { return d ? -1.0 : 1.0; };
  auto M = [](int d) { return d ? 1.0 / 6.0 : 1.0 / 3.0; };
  auto K = [&](int dx, int dy, int dz) {
    return wx * S(dx) * M(dy) * M(dz) + wy * M(dx) * S(dy) * M(dz) + wz * M(dx) * M(dy) * S(dz);
  };
  Stencil st;
  st.self = K(0, 0, 0);
  st.ax[0] = K(1, 0, 0);
  st.ax[1] = K(0, 1, 0);
  st.ax[2] = K(0, 0, 1);
  st.fd[0] = K(0, 1, 1);
  st.fd[1] = K(1, 0, 1);
  st.fd[2] = K(1, 1, 0);
  st.bd = K(1, 1, 1);
  const double sc = std::fabs(st.self);
  st.cubic = (std::fabs(st.ax[0]) <= 1e-14 * sc && std::fabs(st.ax[1]) <= 1e-14 * sc &&
              std::fabs(st.ax[2]) <= 1e-14 * sc) ? 1 : 0;
  if (st.cubic) st.ax[0] = st.ax[1] = st.ax[2] = 0.0;
  // eigenvalues of K0: tensor patterns, S has {0, 2}, M has {1/2, 1/6}
  double lm = 0.0;
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
    const double sx = ax ? 2.0 : 0.0, sy = ay ? 2.0 : 0.0, sz = az ? 2.0 : 0.0;
    const double mx = ax ? 1.0 / 6.0 : 0.5, my = ay ? 1.0 / 6.0 : 0.5, mz = az ? 1.0 / 6.0 : 0.5;
    lm = std::max(lm, wx * sx * my * mz + wy * mx * sy * mz + wz * mx * my * sz);
  }
  *lam_max_k0 = lm;
  return st;
}

static ChebCoef make_cheb(const msmg_options& o) {
  ChebCoef c{};
  c.degree = o.cheb_degree;
  const double theta = 0.5 * (o.cheb_hi + o.cheb_lo), delta = 0.5 * (o.cheb_hi - o.cheb_lo);
  const double sigma = theta / delta;
  c.inv_theta = 1.0 / theta;
  double rho_prev = 1.0 / sigma;
  for (int k = 1; k < o.cheb_degree; ++k) {
    const double rho = 1.0 / (2.0 * sigma - rho_prev);
    c.step_a[k] = rho * rho_prev;
    c.step_b[k] = 2.0 * rho / delta;
    if (k == 1) {
      c.c0 = 1.0 + rho * rho_prev;
      c.c1 = 2.0 * rho / delta;
    }
    rho_prev = rho;
  }
  return c;
}

static Ctx make_ctx(msmg_handle* h, int side = 0) {
  Ctx c{};
  c.g = h->g;
  c.st = h->st;
  c.h = h->hier;
  c.mat = h->mat;
  c.CX = h->CX;
  c.ntiles = h->ntiles;
  c.mg = make_march(h->g, h->march_resident);
  c.mgl = make_march(h->g, h->apply_resident, 8, LMX, LMY);
  c.rho = h->rho;
  c.rho_dt = h->rho_dt;
  c.kc = h->kc;
  c.kv = h->kv;
  c.kv_dt = h->kv_dt;
  c.bits = h->bits;
  c.dinv = h->dinv;
  c.v_dt = h->v_dt;
  c.Rc = h->Rcs;
  c.b_dt = h->b_dt;
  c.cheb = make_cheb(h->opt);
  c.sc = h->vs[side].sc;
  c.partials = h->vs[side].partials;
  c.counter = h->vs[side].counter;
  c.red_blocks = h->red_blocks;
  c.vc_t0 = h->v_t0;
  c.vc_t1 = h->v_t1;
  c.rg = h->rg;
  c.rpart = h->vs[side].rpart;
  c.cc.Ac = h->Acv;
  c.cc.AcDinv = h->AcDinvv;
  c.cc.a_dt = h->a_dt;
  c.cc.Rcc = h->Rccv;
  c.cc.cc_ptr = h->cc_ptr;
  c.cc.cc_dofs = h->cc_dofs;
  c.cc.dof_cc = h->dof_cc;
  c.cc.dof_loc = h->dof_loc;
  c.cc.AccInv = h->Acc;
  c.cc.n_c = h->n_c;
  c.cc.n_cc = h->n_cc;
  c.tpfa = h->tpfa ? 1 : 0;
  c.dface = h->dface;
  return c;
}

template <typename T>
static int dev_alloc(msmg_handle* h, T** p, size_t bytes) {
  void* q = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MSMG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  h->allocs.push_back(q);
  *p = reinterpret_cast<T*>(q);
  return MSMG_OK;
}

static void free_all(msmg_handle* h) {
  for (hipEvent_t e : h->events) (void)hipEventDestroy(e);
  h->events.clear();
  for (hipEvent_t e : h->setup_events) (void)hipEventDestroy(e);
  h->setup_events.clear();
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  for (VecSet& V : h->vs) {
    if (V.sc_host) (void)hipHostFree(V.sc_host);
    V.sc_host = nullptr;
  }
}

#define TRY(expr)                 \
  do {                            \
    int _r = (expr);              \
    if (_r != MSMG_OK) return _r; \
  } while (0)

// ---------------------------------------------------------------------------
// C ABI

extern "C" void msmg_default_options(msmg_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->H = 8;
  o->sd = 8;
  o->Lc = 4;
  o->Lcc = 17;
  o->cheb_degree = 2;
  o->cheb_lo = 0.15;
  o->cheb_hi = 1.5;
  o->vcycle_dtype = MSMG_F64;
  o->rho_v_dtype = MSMG_F64;
  o->basis_dtype = MSMG_F64;
  o->pc_kind = MSMG_PC_MULTIGRID;
  o->check_interval = 8;
  o->eig_block = 0;
  o->eig_degree = 0;
  o->eig_maxit = 60;
  o->eig_tol = 1e-12;
  o->cc_block = 0;
  o->cc_degree = 16;
  o->cc_maxit = 60;
  o->autotune = 1;
  o->tune_cache = nullptr;
  o->timing = 0;
  o->eig_warm_start = 0;
  o->rho_storage = MSMG_F64;
  o->lean_memory = 0;
  o->cc_group = 0;
  o->coarse_fused = 7;
  o->pair_rhs = 0;
  o->discretisation = MSMG_Q1;
  o->lc_threshold = 0.0;
}

extern "C" const char* msmg_last_error(void) { return g_last_error.c_str(); }

static int check_options(const msmg_options& o) {
  if (o.vcycle_dtype != MSMG_F64 && o.vcycle_dtype != MSMG_F32) return fail(MSMG_EINVAL, "vcycle_dtype must be F64 or F32");
  if (o.rho_v_dtype < 0 || o.rho_v_dtype > 2 || o.basis_dtype < 0 || o.basis_dtype > 2)
    return fail(MSMG_EINVAL, "bad storage dtype");
  if (o.vcycle_dtype == MSMG_F64 && o.rho_v_dtype != o.basis_dtype &&
      !(o.rho_v_dtype == MSMG_BF16 && o.basis_dtype == MSMG_F32))
    return fail(MSMG_EINVAL,
                "an FP64 cycle takes density and basis copies of one type (F64, F32 or BF16), or a BF16 density "
                "copy with an F32 basis");
  if (o.vcycle_dtype == MSMG_F32 && (o.rho_v_dtype == MSMG_F64 || o.basis_dtype == MSMG_F64))
    return fail(MSMG_EINVAL, "an FP32 cycle takes F32 or BF16 density and basis copies");
  if (o.pc_kind != MSMG_PC_MULTIGRID && o.pc_kind != MSMG_PC_SMOOTHER) return fail(MSMG_EINVAL, "bad pc_kind");
  if (o.check_interval < 1) return fail(MSMG_EINVAL, "check_interval must be >= 1");
  if (o.eig_block < 0 || o.eig_block > 16 || o.eig_degree < 0 || o.eig_maxit < 1 || !(o.eig_tol > 0))
    return fail(MSMG_EINVAL, "bad eigensolver options");
  if (o.cc_block < 0 || o.cc_block > 32 || o.cc_maxit < 1)
    return fail(MSMG_EINVAL, "bad coarse-coarse eigensolver options");
  if (o.rho_storage != MSMG_F64 && o.rho_storage != MSMG_F32) return fail(MSMG_EINVAL, "rho_storage must be F64 or F32");
  if (o.cc_group < 0) return fail(MSMG_EINVAL, "cc_group must be >= 0");
  if (o.pair_rhs && (o.pc_kind != MSMG_PC_MULTIGRID || o.cheb_degree != 2))
    return fail(MSMG_EINVAL, "pair_rhs needs the multigrid preconditioner with the degree-2 smoother");
  if (o.lean_memory && o.eig_warm_start)
    return fail(MSMG_EINVAL, "lean_memory keeps no basis between set-ups: eig_warm_start is not available");
  if (o.discretisation != MSMG_Q1 && o.discretisation != MSMG_TPFA) return fail(MSMG_EINVAL, "bad discretisation");
  if (!(o.lc_threshold >= 0.0) || !std::isfinite(o.lc_threshold)) return fail(MSMG_EINVAL, "lc_threshold must be >= 0");
  if (o.discretisation == MSMG_TPFA) {
    if (o.vcycle_dtype != MSMG_F64 || o.rho_v_dtype != MSMG_F64 || o.basis_dtype != MSMG_F64)
      return fail(MSMG_EINVAL, "the TPFA discretisation runs FP64 cycle vectors, density copy and basis");
    if (o.pair_rhs || o.lean_memory) return fail(MSMG_EINVAL, "the TPFA discretisation has no pair_rhs or lean_memory");
    if (!(o.cheb_hi >= 2.0))
      return fail(MSMG_EINVAL, "TPFA needs cheb_hi >= 2: the Jacobi-scaled TPFA matrix reaches close to 2");
  }
  return MSMG_OK;
}

// Device arrays of a handle.  With dry = true nothing is allocated and the
// bytes are summed into *total (the footprint msmg_query_plan reports).  With
// lean_memory the FP64 basis master shares the PCG work vectors r, p, q, z
// (it is only read during the set-up), the set-up-only Galerkin blocks of the
// coarse-coarse problem share the FP64 cycle iterate, and the diagnostic copy
// of A_cc is not kept.
static int alloc_arrays(msmg_handle* h, bool dry, size_t* total) {
  const msmg_options& o = h->opt;
  const long long nn = h->g.nn, ne = h->g.ne;
  const size_t vs = dt_size(h->v_dt);
  const bool lean = o.lean_memory != 0;
  int rc = MSMG_OK;
  size_t sum = 0;
  auto A = [&](auto** p, size_t bytes) {
    sum += bytes;
    if (!dry && rc == MSMG_OK) rc = dev_alloc(h, p, bytes);
  };
  A(&h->rho, ne * dt_size(h->rho_store_dt));
  // FP64 conductivities for the PCG apply when the density is FP64 (with an
  // FP32 density the apply forms them from it); the cycle's copy
  const bool kc64 = h->rho_store_dt == DT_F64 || h->tpfa;
  if (kc64) A(&h->kc, ne * 8);
  if (h->tpfa) {
    A(&h->dface, ne);
    A(&h->fcount, 16);
  }
  if (!(kc64 && h->kv_dt == DT_F64)) A(&h->kv, ne * dt_size(h->kv_dt));
  A(&h->bits, ((nn + 31) / 32) * 4);
  // Jacobi diagonal: FP64 only on the all-FP64 path (a fixed coefficient like rho)
  h->dv_dt = (h->v_dt == DT_F64 && h->b_dt == DT_F64) ? DT_F64 : DT_F32;
  A(&h->dinv, nn * dt_size(h->dv_dt));
  if (lean && h->mg) {
    // r, p, q, z in one block that also holds the FP64 basis during a set-up
    const long long nv = std::max<long long>(4, h->hier.Lc);
    double* blk = nullptr;
    A(&blk, (size_t)nv * nn * 8);
    if (blk) {
      h->vs[0].r = blk; h->vs[0].p = blk + nn; h->vs[0].q = blk + 2 * nn; h->vs[0].z = blk + 3 * nn;
      h->Rc64 = blk;
    }
  } else {
    A(&h->vs[0].r, nn * 8); A(&h->vs[0].p, nn * 8); A(&h->vs[0].q, nn * 8); A(&h->vs[0].z, nn * 8);
  }
  A(&h->vs[0].b, nn * 8);
  A(&h->vs[0].xlo, nn * 4);
  A(&h->vs[0].v_r1, nn * vs); A(&h->vs[0].v_res, nn * vs);
  if (o.cheb_degree > 2) { A(&h->v_t0, nn * vs); A(&h->v_t1, nn * vs); }
  // one slot per workgroup of any reducing launch (tiles, march, 1-D grids)
  h->partial_slots = std::max<long long>({h->ntiles + 8, 8192LL, make_march(h->g, h->march_resident).blocks,
                                          make_march(h->g, h->apply_resident, 8, LMX, LMY).blocks,
                                          (long long)h->red_blocks});
  A(&h->vs[0].partials, h->partial_slots * 2 * 8);
  A(&h->vs[0].counter, 64);
  A(&h->oc_state, 64);
  A(&h->vs[0].sc, sizeof(Scalars));
  if (h->mg) {
    A(&h->vs[0].v_r2, nn * 8);  // prolongated iterate: FP64 on every path
    if (!lean) A(&h->Rc64, nn * h->hier.Lc * 8);
    // the cycle's copy of the basis; the lean layout needs its own even in FP64,
    // since the master there is overwritten by the first solve
    if (h->b_dt != DT_F64 || lean) A(&h->Rcs, nn * h->hier.Lc * dt_size(h->b_dt));
    const size_t nblk = (size_t)h->hier.ncells * 27 * h->hier.Lc * h->hier.Lc;
    A(&h->Ac64, nblk * 8);
    if (lean && nblk <= (size_t)nn) h->G64 = (double*)h->vs[0].v_r2;
    else A(&h->G64, nblk * 8);
    A(&h->AcDinv64, (size_t)h->n_c * h->hier.Lc * 8);
    if (h->a_dt != DT_F64) {
      A(&h->Acv, nblk * 4);
      A(&h->AcDinvv, (size_t)h->n_c * h->hier.Lc * 4);
    }
    A(&h->Rcc64, (size_t)h->hier.Lcc * h->n_c * 8);
    A(&h->cc_ptr, (h->hier.ncc + 1) * 4);
    A(&h->cc_dofs, (size_t)h->n_c * 4);
    A(&h->dof_cc, (size_t)h->n_c * 4);
    A(&h->dof_loc, (size_t)h->n_c * 4);
    A(&h->Acc, (size_t)h->n_cc * h->n_cc * 8);
    A(&h->evals, (size_t)h->n_c * 8);
    A(&h->cell_status, (size_t)h->hier.ncells * 4);
    A(&h->cc_evals, (size_t)h->n_cc * 8);
    A(&h->cc_status, (size_t)h->hier.ncc * 4);
    A(&h->vs[0].c_rc, (size_t)h->n_c * 8); A(&h->vs[0].c_x0, (size_t)h->n_c * 8); A(&h->vs[0].c_t, (size_t)h->n_c * 8);
    A(&h->vs[0].c_x1, (size_t)h->n_c * 8); A(&h->vs[0].c_d, (size_t)h->n_c * 8);
    A(&h->vs[0].rcc, (size_t)h->n_cc * 8); A(&h->vs[0].ecc, (size_t)h->n_cc * 8);
    if (o.coarse_fused & 1) A(&h->l1_bar, (size_t)level1_barrier_words() * 4);
    if ((o.coarse_fused & 2) && restrict_fusable(h->hier) && !h->tpfa) {
      h->rg = make_restrict_geo(h->g, h->hier, h->march_resident);
      A(&h->vs[0].rpart, (size_t)h->rg.slots * h->hier.Lc * 8);
    }
    if ((o.coarse_fused & 2) && h->tpfa) {
      const Ctx c0 = make_ctx(h);
      if (tpfa_restrict_fusable(c0)) A(&h->vs[0].rpart, (size_t)tpfa_restrict_slots(c0) * h->hier.Lc * 8);
    }
    if (o.pair_rhs) {
      // the second side of a batched pair: its own PCG and cycle vectors
      VecSet& V = h->vs[1];
      A(&V.r, nn * 8); A(&V.p, nn * 8); A(&V.q, nn * 8); A(&V.z, nn * 8); A(&V.b, nn * 8);
      A(&V.xlo, nn * 4);
      A(&V.v_r1, nn * vs); A(&V.v_res, nn * vs); A(&V.v_r2, nn * 8);
      A(&V.partials, h->partial_slots * 2 * 8);
      A(&V.counter, 64);
      A(&V.sc, sizeof(Scalars));
      A(&V.c_rc, (size_t)h->n_c * 8); A(&V.c_x0, (size_t)h->n_c * 8); A(&V.c_t, (size_t)h->n_c * 8);
      A(&V.c_x1, (size_t)h->n_c * 8); A(&V.c_d, (size_t)h->n_c * 8);
      A(&V.rcc, (size_t)h->n_cc * 8); A(&V.ecc, (size_t)h->n_cc * 8);
      if (h->vs[0].rpart || (dry && (o.coarse_fused & 2) && restrict_fusable(h->hier)))
        A(&V.rpart, (size_t)h->rg.slots * h->hier.Lc * 8);
    }
    if (rc == MSMG_OK)
      rc = setup_scratch_alloc(h->g, h->hier, h->max_cc_dofs, h->n_cc, o, &h->scratch, [&](void** p, size_t bytes) {
        sum += bytes;
        return dry ? MSMG_OK : dev_alloc(h, p, bytes);
      });
  }
  if (total) *total = sum;
  return rc;
}

// Host-side fields of a handle that the plan and the options fix.
static void init_handle(msmg_handle* h, const msmg_options& o, const Plan& P, int nx, int ny, int nz, double lx,
                        double ly, double lz) {
  h->opt = o;
  h->tpfa = o.discretisation == MSMG_TPFA;
  h->g = make_geo(nx, ny, nz, lx, ly, lz, h->tpfa);
  double lmk0 = 0.0;
  h->st = make_stencil(h->g, &lmk0);
  h->lam_bound = 8.0 * lmk0 / h->g.vol;
  if (h->tpfa) {
    // Gershgorin bound of M^-1/2 K M^-1/2 for the TPFA local problems: per
    // face, T/m_K + T/sqrt(m_K m_L) <= (1 + sqrt 2) / h_d^2, two faces per axis
    const double s2 = 1.0 / (h->g.hx * h->g.hx) + 1.0 / (h->g.hy * h->g.hy) + 1.0 / (h->g.hz * h->g.hz);
    h->lam_bound = 2.0 * (1.0 + std::sqrt(2.0)) * s2;
  }
  h->hier = P.h;
  h->CX = P.CX;
  h->ntiles = P.ntiles;
  h->n_c = P.n_c;
  h->n_cc = P.n_cc;
  h->max_cc_dofs = P.max_cc_dofs;
  h->max_cell_nodes = P.max_cell_nodes;
  h->h_cc_ptr = P.cc_ptr;
  h->mg = (o.pc_kind == MSMG_PC_MULTIGRID);
  h->v_dt = o.vcycle_dtype;
  h->kv_dt = o.rho_v_dtype;
  h->b_dt = o.basis_dtype;
  h->rho_store_dt = o.rho_storage;
  // level-1 operator and level 2 stay FP64 on every path: an FP32 copy of A_c
  // costs ~10% more iterations at contrast 1e6
  h->a_dt = DT_F64;
}

extern "C" int msmg_query_plan(int nx, int ny, int nz, const msmg_options* opt, msmg_plan* out) {
  msmg_options o;
  if (opt) o = *opt; else msmg_default_options(&o);
  if (!out) return fail(MSMG_EINVAL, "out is NULL");
  TRY(check_options(o));
  Plan P;
  TRY(make_plan(nx, ny, nz, o, P, o.discretisation == MSMG_TPFA ? 0 : 1));
  out->ncx = P.h.ncx; out->ncy = P.h.ncy; out->ncz = P.h.ncz; out->ncells = P.h.ncells;
  out->nccx = P.h.nccx; out->nccy = P.h.nccy; out->nccz = P.h.nccz; out->ncc = P.h.ncc;
  out->n_c = P.n_c;
  out->n_cc = P.n_cc;
  out->max_cell_nodes = P.max_cell_nodes;
  out->max_cc_dofs = P.max_cc_dofs;
  const int e = o.discretisation == MSMG_TPFA ? 0 : 1;
  out->nodes = (long long)(nx + e) * (ny + e) * (nz + e);
  out->elements = (long long)nx * ny * nz;
  msmg_handle tmp;
  init_handle(&tmp, o, P, nx, ny, nz, 1.0, 1.0, 1.0);
  size_t bytes = 0;
  TRY(alloc_arrays(&tmp, true, &bytes));
  out->device_bytes = bytes;
  return MSMG_OK;
}

extern "C" int msmg_create(msmg_handle** out, int nx, int ny, int nz, double lx, double ly, double lz,
                           const msmg_options* opt) {
  if (!out) return fail(MSMG_EINVAL, "handle pointer is NULL");
  *out = nullptr;
  if (!(lx > 0) || !(ly > 0) || !(lz > 0)) return fail(MSMG_EINVAL, "box lengths must be positive");
  msmg_options o;
  if (opt) o = *opt; else msmg_default_options(&o);
  TRY(check_options(o));
  Plan P;
  TRY(make_plan(nx, ny, nz, o, P, o.discretisation == MSMG_TPFA ? 0 : 1));
  msmg_handle* h = new msmg_handle();
  init_handle(h, o, P, nx, ny, nz, lx, ly, lz);
  HIP_TRY(hipGetDevice(&h->device));
  if (h->tpfa && !tpfa_grid_fits(make_ctx(h))) {
    delete h;
    return fail(MSMG_EINVAL, "the TPFA stencil grid exceeds its workgroup budget (nx * ny too large)");
  }
  h->march_resident = march_resident_blocks();
  h->apply_resident = apply_resident_blocks();
  int rc = alloc_arrays(h, false, nullptr);
  // The one-launch coarse levels run one workgroup per compute unit: on small
  // coarse problems they save the launches and their gaps, on large ones too
  // few loads are in flight for the streams of A_c and the dense A_cc^-1
  // (measured per solve: 145 against 149 ms at 256^3, n_c = 131,072; 908
  // against 897 ms at 512^3; 16.9 against 14.8 s at 1024^3).
  if (rc == MSMG_OK && h->mg && h->l1_bar && h->a_dt == DT_F64 && h->hier.Lcc <= 64 && h->n_c <= kLevel1MaxCoarse)
    h->l1_blocks = level1_blocks();
  if (rc == MSMG_OK) {
    for (VecSet& V : h->vs) {
      if (!V.sc || rc != MSMG_OK) continue;
      hipError_t e = hipHostMalloc((void**)&V.sc_host, sizeof(Scalars), hipHostMallocDefault);
      if (e != hipSuccess) rc = fail(MSMG_ENOMEM, "pinned host allocation failed");
    }
  }
  if (rc != MSMG_OK) {
    free_all(h);
    delete h;
    return rc;
  }
  if (!h->kv) h->kv = h->kc;
  if (!h->Rcs) h->Rcs = h->Rc64;
  if (!h->Acv) h->Acv = h->Ac64;
  if (!h->AcDinvv) h->AcDinvv = h->AcDinv64;
  if (!h->Rccv) h->Rccv = h->Rcc64;
  for (VecSet& V : h->vs)
    if (V.counter) HIP_TRY(hipMemset(V.counter, 0, 64));
  if (h->l1_bar) HIP_TRY(hipMemset(h->l1_bar, 0, (size_t)level1_barrier_words() * 4));
  for (VecSet& V : h->vs)
    if (V.sc) HIP_TRY(hipMemset(V.sc, 0, sizeof(Scalars)));
  if (o.timing) {
    // events of the per-iteration and set-up timing (created here, outside any solve)
    h->events.resize(4 * 512);
    h->setup_events.resize(SETUP_EVENTS);
    for (auto& e : h->setup_events) {
      hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) {
        e = nullptr;
        msmg_destroy(h);
        return fail(MSMG_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(err));
      }
    }
    for (auto& e : h->events) {
      hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) {
        e = nullptr;
        msmg_destroy(h);
        return fail(MSMG_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(err));
      }
    }
  }
  if (h->mg) {
    // coarse-coarse dof maps (host-built, uploaded once)
    const Hier& hh = h->hier;
    std::vector<int> cc_dofs(h->n_c), dof_cc(h->n_c), dof_loc(h->n_c);
    for (int jz = 0; jz < hh.nccz; ++jz)
      for (int jy = 0; jy < hh.nccy; ++jy)
        for (int jx = 0; jx < hh.nccx; ++jx) {
          const int J = (jz * hh.nccy + jy) * hh.nccx + jx;
          int d = h->h_cc_ptr[J];
          for (int cz = group_begin(jz, hh.sd); cz < group_end(jz, hh.sd, hh.nccz, hh.ncz); ++cz)
            for (int cy = group_begin(jy, hh.sd); cy < group_end(jy, hh.sd, hh.nccy, hh.ncy); ++cy)
              for (int cx = group_begin(jx, hh.sd); cx < group_end(jx, hh.sd, hh.nccx, hh.ncx); ++cx) {
                const int cell = (cz * hh.ncy + cy) * hh.ncx + cx;
                for (int l = 0; l < hh.Lc; ++l) {
                  const int gd = cell * hh.Lc + l;
                  cc_dofs[d] = gd;
                  dof_cc[gd] = J;
                  dof_loc[gd] = d - h->h_cc_ptr[J];
                  ++d;
                }
              }
        }
    HIP_TRY(hipMemcpy(h->cc_ptr, h->h_cc_ptr.data(), (hh.ncc + 1) * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(h->cc_dofs, cc_dofs.data(), (size_t)h->n_c * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(h->dof_cc, dof_cc.data(), (size_t)h->n_c * 4, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(h->dof_loc, dof_loc.data(), (size_t)h->n_c * 4, hipMemcpyHostToDevice));
  }
  *out = h;
  return MSMG_OK;
}

extern "C" void msmg_destroy(msmg_handle* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  free_all(h);
  delete h;
}

static double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

extern "C" int msmg_setup(msmg_handle* h, const void* rho, msmg_dtype rho_dtype, double kmin, double kmax, int p,
                          const uint8_t* mask, const double* fixed_values, hipStream_t s) {
  if (!h || !rho || !mask) return fail(MSMG_EINVAL, "NULL argument");
  if (rho_dtype != MSMG_F64 && rho_dtype != MSMG_F32) return fail(MSMG_EINVAL, "rho must be F64 or F32");
  if (h->rho_store_dt == DT_F32 && rho_dtype != MSMG_F32)
    return fail(MSMG_EINVAL, "this handle stores the density in FP32 (rho_storage): pass F32 densities");
  if (!(kmin > 0.0) || !(kmax >= kmin) || !std::isfinite(kmax)) return fail(MSMG_EINVAL, "need 0 < k_min <= k_max");
  if (p < 1 || p > 16) return fail(MSMG_EINVAL, "p must be in 1..16");
  const double t0 = now_ms();
  h->setup_done = false;
  h->mat.kmin = kmin;
  h->mat.kmax = kmax;
  h->mat.p = p;
  h->rho_dt = h->rho_store_dt;
  const long long nn = h->g.nn, ne = h->g.ne;
  launch_convert(rho, rho_dtype, h->rho, h->rho_store_dt, ne, s);
  if (h->tpfa) {
    // Dirichlet face flags: copied and checked; no unknown is fixed
    Ctx c0 = make_ctx(h);
    unsigned long long cnt[2] = {0, 0};
    HIP_TRY(hipMemsetAsync(h->fcount, 0, 16, s));
    launch_tpfa_flags(c0, mask, h->dface, h->fcount, s);
    HIP_TRY(hipMemsetAsync(h->bits, 0, ((nn + 31) / 32) * 4, s));
    HIP_TRY(hipMemcpyAsync(cnt, h->fcount, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (cnt[1]) return fail(MSMG_EINVAL, "a Dirichlet face flag sits on an internal face (or outside bits 0..5)");
    if (cnt[0] == 0) return fail(MSMG_ESINGULAR, "no Dirichlet face: the operator is singular");
    if (fixed_values) {
      if (!h->tfix) TRY(dev_alloc(h, &h->tfix, nn * 8));
      launch_convert(fixed_values, DT_F64, h->tfix, DT_F64, nn, s);
      h->has_tfix = true;
    } else {
      h->has_tfix = false;
    }
  } else {
  launch_pack_mask(mask, h->bits, nn, s);
  if (fixed_values) {
    if (!h->tfix) TRY(dev_alloc(h, &h->tfix, nn * 8));
    // tfix = values on fixed nodes, 0 elsewhere
    Ctx c0 = make_ctx(h);
    launch_convert(fixed_values, DT_F64, h->tfix, DT_F64, nn, s);
    launch_zero_free(c0, h->tfix, s);
    h->has_tfix = true;
  } else {
    h->has_tfix = false;
  }
  // mask must hold a fixed node (else A is singular)
  {
    Ctx c = make_ctx(h);
    int nfixed = 0;
    TRY(count_fixed(c, &nfixed, s));
    if (nfixed == 0) return fail(MSMG_ESINGULAR, "the Dirichlet mask is empty: the operator is singular");
  }
  }
  Ctx c = make_ctx(h);
  if (h->kc) launch_conductivity(c, h->rho, h->rho_dt, h->kc, DT_F64, s);
  if (h->kv != h->kc) launch_conductivity(c, h->rho, h->rho_dt, h->kv, h->kv_dt, s);
  if (h->tpfa) launch_tpfa_diag_inv(c, (double*)h->dinv, s);
  else launch_diag_inv(c, h->rho, h->rho_dt, h->dinv, h->dv_dt, s);
  HIP_TRY(hipGetLastError());
  if (h->mg) {
    SetupArgs a{};
    a.lam_bound = h->lam_bound;
    a.Rc64 = h->Rc64;
    a.Rcs = h->Rcs;
    a.b_dt = h->b_dt;
    a.Ac64 = h->Ac64;
    a.Acv = h->Acv;
    a.AcDinv64 = h->AcDinv64;
    a.AcDinvv = h->AcDinvv;
    a.a_dt = h->a_dt;
    a.G64 = h->G64;
    a.Rcc64 = h->Rcc64;
    a.Rccv = h->Rccv;
    a.Acc = h->Acc;
    a.evals = h->evals;
    a.cell_status = h->cell_status;
    a.cc_evals = h->cc_evals;
    a.cc_status = h->cc_status;
    a.n_c = h->n_c;
    a.n_cc = h->n_cc;
    a.max_cell_nodes = h->max_cell_nodes;
    a.max_cc_dofs = h->max_cc_dofs;
    a.cc_ptr = h->cc_ptr;
    a.h_cc_ptr = h->h_cc_ptr.data();
    a.cc_dofs = h->cc_dofs;
    a.dof_cc = h->dof_cc;
    a.dof_loc = h->dof_loc;
    a.opt = &h->opt;
    a.warm = (h->opt.eig_warm_start && h->has_basis) ? 1 : 0;
    h->has_basis = false;
    a.tune = h->tune;
    a.ev = h->setup_events.empty() ? nullptr : h->setup_events.data();
    SetupReport rep{};
    const int r = run_setup(c, a, &h->scratch, &rep, s);
    if (r != MSMG_OK) return fail(r, std::string("set-up failed: ") + rep.msg);
    h->eig_unconverged = rep.eig_unconverged;
    h->cc_unconverged = rep.cc_unconverged;
    h->eig_ties = rep.eig_ties;
    if (a.ev) {
      HIP_TRY(hipEventSynchronize(a.ev[4]));
      for (int k = 0; k < 4; ++k) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, a.ev[k], a.ev[k + 1]));
        h->setup_phase_ms[k] = ms;
      }
      h->setup_dense_ms = rep.dense_ms;
      h->setup_dense_gflop = rep.dense_gflop;
    }
  }
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipGetLastError());
  h->setup_ms = now_ms() - t0;
  h->setup_done = true;
  h->has_basis = (h->mg != 0) && !h->opt.lean_memory;
  h->basis_live = (h->mg != 0);
  return MSMG_OK;
}

// Polls of one bounded barrier wait in the grid-synchronised coarse-level kernel
// (each poll sleeps ~60 ns): about a quarter of a second, far beyond any
// legitimate wait, after which the solve reports MSMG_ETIMEOUT.
static constexpr unsigned LEVEL1_SPIN_LIMIT = 1u << 22;

// Levels 1 and 2 of Algorithm 1 and the prolongation to level 0:
// v_r2 = r1 + R_c^T e_c from the restricted residual c_rc.
// Levels 1 and 2 of Algorithm 1 and the prolongation r2 = r1 + R_c^T e_c.
// With e1 given, the prolongation is left to the caller: e_c = *e1 + *e2
// (*e2 may be null).
static void coarse_correction(msmg_handle* h, const Ctx& c, VecSet& V, hipStream_t s, const double** e1 = nullptr,
                              const double** e2 = nullptr) {
  if (h->l1_blocks > 0) {
    // every coarse step in one grid-synchronised launch; c_x0 ends as e_c
    if (launch_level1(c, h->l1_blocks, (const double*)V.c_rc, (double*)V.c_x0, (double*)V.c_t, V.rcc,
                      h->l1_bar, LEVEL1_SPIN_LIMIT, s) == hipSuccess) {
      if (e1) {
        *e1 = (const double*)V.c_x0;
        *e2 = nullptr;
        return;
      }
      launch_prolong(c, V.v_r1, V.c_x0, nullptr, V.v_r2, s);
      return;
    }
    // the launch failed: one launch per step from now on
    (void)hipGetLastError();
    h->l1_blocks = 0;
  }
  launch_gs_sweep(c, V.c_rc, V.c_x0, true, s);                    // rc0 = S_c^-1 rc
  launch_ac_residual(c, V.c_rc, V.c_x0, V.c_t, s);               // rc - A_c rc0
  launch_cc_restrict(c, V.c_t, V.rcc, s);                         // rcc = R_cc (...)
  launch_acc_solve(c, V.rcc, V.ecc, s);                           // ecc = A_cc^-1 rcc
  launch_cc_prolong(c, V.c_x0, V.ecc, V.c_x1, s);                // rc1 = rc0 + R_cc^T ecc
  launch_ac_residual(c, V.c_rc, V.c_x1, V.c_t, s);               // rc - A_c rc1
  launch_gs_sweep(c, V.c_t, V.c_d, false, s);                     // S_c^-T (...)
  if (e1) {
    *e1 = (const double*)V.c_x1;
    *e2 = (const double*)V.c_d;
    return;
  }
  launch_prolong(c, V.v_r1, V.c_x1, V.c_d, V.v_r2, s);          // r2 = r1 + R_c^T ec (FP64)
}

// Algorithm 1 on the cell unknowns of the two-point flux discretisation:
// the level-0 steps as separate launches, levels 1 and 2 shared with Q1.
static void precondition_tpfa(msmg_handle* h, const Ctx& c, VecSet& V, const double* r, double* z, const double* q,
                              int mode, hipStream_t s) {
  double* r1 = (double*)V.v_r1;
  double* res = (double*)V.v_res;
  launch_tpfa_smooth(c, r, r1, s);  // r1 = S^-1 r0
  if (!h->mg) {
    launch_vc_output(c, r1, true, nullptr, z, r, q, mode, s);
    return;
  }
  if (V.rpart) {
    launch_tpfa_vresidual_restrict(c, r, r1, V.rpart, (double*)V.c_rc, s);  // rc = R_c (r0 - A r1)
  } else {
    launch_tpfa_vresidual(c, r, r1, res, s);           // r0 - A r1
    launch_tpfa_restrict(c, res, (double*)V.c_rc, s);  // rc = R_c (r0 - A r1)
  }
  const double *e1 = nullptr, *e2 = nullptr;
  coarse_correction(h, c, V, s, &e1, &e2);                  // e_c
  launch_tpfa_prolong(c, r1, e1, e2, (double*)V.v_r2, s);  // r2 = r1 + R_c^T e_c
  launch_tpfa_vresidual(c, r, (const double*)V.v_r2, res, s);  // r0 - A r2
  if (c.cheb.degree == 2) {
    launch_tpfa_smooth_output(c, res, (const double*)V.v_r2, z, r, q, mode, s);  // y = r2 + S^-T (...)
    return;
  }
  launch_tpfa_smooth(c, res, r1, s);                           // S^-T (...)
  launch_vc_output(c, V.v_r2, true, r1, z, r, q, mode, s);     // y = r2 + ...
}

// One preconditioner application r (FP64) -> z (FP64) with the PCG reduction
// mode (0 init, 1 iteration, 2 none).
static void precondition(msmg_handle* h, const Ctx& c, VecSet& V, const double* r, double* z, const double* q,
                         int mode, hipStream_t s) {
  if (c.tpfa) {
    precondition_tpfa(h, c, V, r, z, q, mode, s);
    return;
  }
  const bool v64 = (h->v_dt == DT_F64);
  const bool fused = smooth_output_fused(c);
  if (!h->mg) {
    if (fused) {
      launch_smooth_output(c, r, true, nullptr, z, r, q, mode, s);
      return;
    }
    launch_smooth(c, r, true, V.v_r1, s);
    launch_vc_output(c, V.v_r1, v64, nullptr, z, r, q, mode, s);
    return;
  }
  launch_smooth(c, r, true, V.v_r1, s);                            // r1 = S^-1 r0
  if (V.rpart) {
    launch_vresidual_restrict(c, r, V.v_r1, (double*)V.c_rc, s);  // rc = R_c (r0 - A r1)
  } else {
    launch_vresidual(c, r, true, V.v_r1, v64, V.v_res, s);        // r0 - A r1
    launch_restrict(c, V.v_res, V.c_rc, s);                       // rc = R_c (r0 - A r1)
  }
  if (h->opt.coarse_fused & 4) {
    const double *e1 = nullptr, *e2 = nullptr;
    coarse_correction(h, c, V, s, &e1, &e2);                           // e_c
    launch_vresidual_prolong(c, r, V.v_r1, e1, e2, V.v_res, (double*)V.v_r2, s);  // r2 = r1 + R_c^T e_c, r0 - A r2
  } else {
    coarse_correction(h, c, V, s);                                     // r2 = r1 + R_c^T e_c
    launch_vresidual(c, r, true, V.v_r2, true, V.v_res, s);       // r0 - A r2
  }
  if (fused) {
    launch_smooth_output(c, V.v_res, false, (const double*)V.v_r2, z, r, q, mode, s);  // y = r2 + S^-T (...)
    return;
  }
  launch_smooth(c, V.v_res, false, V.v_r1, s);                    // S^-T (...)
  launch_vc_output(c, V.v_r2, true, V.v_r1, z, r, q, mode, s);    // y = r2 + ...
}

// The PCG's products with A on either discretisation: q = A p with the step
// length reduction, and b - A x (x + xlo) with the true-residual reduction.
static void op_apply_pcg(const Ctx& c, const double* p, double* q, hipStream_t s) {
  if (c.tpfa) launch_tpfa_apply(c, p, q, true, s);
  else launch_apply(c, p, q, 1, s);
}
static void op_residual(const Ctx& c, const double* b, const double* x, const float* xlo, double* y, bool reduce,
                        hipStream_t s) {
  if (c.tpfa) launch_tpfa_residual(c, b, x, xlo, y, reduce, s);
  else launch_residual(c, b, x, xlo, y, reduce, s);
}

static int read_scalars(VecSet& V, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(V.sc_host, V.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return MSMG_OK;
}

extern "C" int msmg_precondition(msmg_handle* h, const double* r, double* z, hipStream_t s) {
  if (!h || !r || !z) return fail(MSMG_EINVAL, "NULL argument");
  if (!h->setup_done) return fail(MSMG_ESTATE, "msmg_setup has not completed");
  Ctx c = make_ctx(h);
  if (h->opt.lean_memory) h->basis_live = false;
  launch_sc_reset(c, 0, 0, s);
  launch_zero_fixed_copy(c, r, h->vs[0].r, s);
  precondition(h, c, h->vs[0], h->vs[0].r, z, nullptr, 2, s);
  HIP_TRY(hipGetLastError());
  if (h->l1_blocks > 0) {
    // the grid-synchronised coarse-level kernel reports a failed wait in the scalars
    TRY(read_scalars(h->vs[0], s));
    if (h->vs[0].sc_host->status == ST_SYNC_TIMEOUT)
      return fail(MSMG_ETIMEOUT, "a grid-wide wait of the coarse-level kernel exceeded its limit");
  }
  return MSMG_OK;
}

extern "C" int msmg_apply(msmg_handle* h, const double* x, double* y, hipStream_t s) {
  if (!h || !x || !y) return fail(MSMG_EINVAL, "NULL argument");
  if (!h->setup_done) return fail(MSMG_ESTATE, "msmg_setup has not completed");
  if (x == y) return fail(MSMG_EINVAL, "x and y must not alias");
  Ctx c = make_ctx(h);
  if (h->tpfa) {
    launch_tpfa_apply(c, x, y, false, s);
    HIP_TRY(hipGetLastError());
    return MSMG_OK;
  }
  // the march stages x with zero fixed entries (handle scratch q, which the
  // lean layout shares with the exported basis)
  if (h->opt.lean_memory) h->basis_live = false;
  launch_zero_fixed_copy(c, x, h->vs[0].q, s);
  launch_apply(c, h->vs[0].q, y, 2, s, x);
  HIP_TRY(hipGetLastError());
  return MSMG_OK;
}

extern "C" int msmg_sensitivity(msmg_handle* h, const double* T, const double* lam, double* dc, hipStream_t s) {
  if (!h || !T || !dc) return fail(MSMG_EINVAL, "NULL argument");
  if (!h->setup_done) return fail(MSMG_ESTATE, "msmg_setup has not completed");
  Ctx c = make_ctx(h);
  if (h->tpfa) launch_tpfa_sensitivity(c, T, lam, h->has_tfix ? h->tfix : nullptr, 0.0, false, dc, s);
  else launch_sensitivity(c, T, lam, dc, s);
  HIP_TRY(hipGetLastError());
  return MSMG_OK;
}

extern "C" int msmg_sensitivity_heat_source(msmg_handle* h, const double* T, const double* lam, double f0, double* dc,
                                            hipStream_t s) {
  if (!h || !T || !lam || !dc) return fail(MSMG_EINVAL, "NULL argument");
  if (!std::isfinite(f0)) return fail(MSMG_EINVAL, "f0 must be finite");
  if (!h->setup_done) return fail(MSMG_ESTATE, "msmg_setup has not completed");
  Ctx c = make_ctx(h);
  if (h->tpfa) launch_tpfa_sensitivity(c, T, lam, h->has_tfix ? h->tfix : nullptr, f0, true, dc, s);
  else launch_sensitivity_heat_source(c, T, lam, f0, dc, s);
  HIP_TRY(hipGetLastError());
  return MSMG_OK;
}

extern "C" int msmg_heat_source_load(msmg_handle* h, double f0, double* f, hipStream_t s) {
  if (!h || !f) return fail(MSMG_EINVAL, "NULL argument");
  if (!std::isfinite(f0)) return fail(MSMG_EINVAL, "f0 must be finite");
  if (!h->setup_done) return fail(MSMG_ESTATE, "msmg_setup has not completed");
  Ctx c = make_ctx(h);
  if (h->tpfa) launch_tpfa_heat_source_load(c, f0, f, s);
  else launch_heat_source_load(c, f0, f, s);
  HIP_TRY(hipGetLastError());
  return MSMG_OK;
}

extern "C" int msmg_element_load(msmg_handle* h, const double* src, double sconst, double* f, hipStream_t s) {
  if (!h || !f) return fail(MSMG_EINVAL, "NULL argument");
  if (h->tpfa) launch_tpfa_cell_load(make_ctx(h), src, sconst, f, s);
  else launch_element_load(h->g, src, sconst, f, s);
  HIP_TRY(hipGetLastError());
  return MSMG_OK;
}

extern "C" int msmg_time_apply(msmg_handle* h, const double* x, int reps, double* ms, hipStream_t s) {
  if (!h || !x || !ms) return fail(MSMG_EINVAL, "NULL argument");
  if (reps < 1) return fail(MSMG_EINVAL, "reps must be >= 1");
  if (!h->setup_done) return fail(MSMG_ESTATE, "msmg_setup has not completed");
  Ctx c = make_ctx(h);
  VecSet& V = h->vs[0];
  if (h->opt.lean_memory) h->basis_live = false;
  // p = x (zero fixed entries), r^T z = p^T p > 0, so that every launch of the
  // PCG's apply runs its step reduction and leaves the iteration undone
  launch_sc_reset(c, 1, 1 << 30, s);
  launch_zero_fixed_copy(c, x, V.p, s);
  launch_vc_output(c, V.p, true, nullptr, V.z, V.p, nullptr, 0, s);
  op_apply_pcg(c, V.p, V.q, s);  // warm-up
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t err = hipEventCreate(&e1);
  if (err == hipSuccess) err = hipEventRecord(e0, s);
  for (int r = 0; r < reps && err == hipSuccess; ++r) op_apply_pcg(c, V.p, V.q, s);
  if (err == hipSuccess) err = hipEventRecord(e1, s);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float t = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(MSMG_EHIP, std::string("apply timing: ") + hipGetErrorString(err));
  TRY(read_scalars(V, s));
  if (V.sc_host->done) return fail(MSMG_EINVAL, "x gives p^T A p <= 0 (zero or non-finite input)");
  *ms = double(t) / reps;
  return MSMG_OK;
}

extern "C" int msmg_stream_ceiling(const double* x, const double* k, double* y, long long nn, long long ne, int reps,
                                   double* ms, hipStream_t s) {
  if (!x || !k || !y || !ms) return fail(MSMG_EINVAL, "NULL argument");
  if (nn < 2 || ne < 2 || ne > nn || (nn & 1) || (ne & 1) || reps < 1)
    return fail(MSMG_EINVAL, "need even sizes 2 <= ne <= nn and reps >= 1");
  if (x == y || k == y) return fail(MSMG_EINVAL, "y must not alias x or k");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  hipError_t err = hipEventCreate(&e1);
  if (err != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(MSMG_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(err));
  }
  launch_stream_ceiling(x, k, y, nn, ne, s);  // warm-up
  err = hipEventRecord(e0, s);
  for (int r = 0; r < reps && err == hipSuccess; ++r) launch_stream_ceiling(x, k, y, nn, ne, s);
  if (err == hipSuccess) err = hipEventRecord(e1, s);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float t = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(MSMG_EHIP, std::string("stream ceiling: ") + hipGetErrorString(err));
  *ms = double(t) / reps;
  return MSMG_OK;
}

extern "C" int msmg_prolong_nodal(int nx, int ny, int nz, const double* tc, double* tf, hipStream_t s) {
  if (nx < 1 || ny < 1 || nz < 1 || !tc || !tf) return fail(MSMG_EINVAL, "bad arguments");
  launch_prolong_nodal(nx, ny, nz, tc, tf, s);
  HIP_TRY(hipGetLastError());
  return MSMG_OK;
}

extern "C" int msmg_prolong_element(int nx, int ny, int nz, const void* rc, void* rf, msmg_dtype dt, hipStream_t s) {
  if (nx < 1 || ny < 1 || nz < 1 || !rc || !rf || dt < 0 || dt > 2) return fail(MSMG_EINVAL, "bad arguments");
  launch_prolong_element(nx, ny, nz, rc, rf, dt, s);
  HIP_TRY(hipGetLastError());
  return MSMG_OK;
}

static void fill_setup_timing(const msmg_handle* h, msmg_info* info) {
  for (int k = 0; k < 4; ++k) info->setup_phase_ms[k] = h->setup_phase_ms[k];
  info->setup_dense_ms = h->setup_dense_ms;
  info->setup_dense_gflop = h->setup_dense_gflop;
}

// PCG driver shared by the state and adjoint solves.  `homogeneous` solves
// with zero fixed values (the adjoint system), ignoring the set-up's values.
static int solve_impl(msmg_handle* h, const double* f, double* T, double* T_lo, int use_x0, double rtol, int maxit,
                      msmg_info* info, hipStream_t s, bool homogeneous) {
  if (!h || !f || !T) return fail(MSMG_EINVAL, "NULL argument");
  if (!h->setup_done) return fail(MSMG_ESTATE, "msmg_setup has not completed");
  if (!(rtol >= 0.0) || maxit < 0) return fail(MSMG_EINVAL, "need rtol >= 0 and maxit >= 0");
  if (f == T || (T_lo && (T_lo == T || T_lo == f))) return fail(MSMG_EINVAL, "f, T and T_lo must not alias");
  const double t0 = now_ms();
  Ctx c = make_ctx(h);
  VecSet& V = h->vs[0];
  if (h->opt.lean_memory) h->basis_live = false;
  const double* lift = (h->has_tfix && !homogeneous) ? h->tfix : nullptr;
  double* x = T;
  // b = f - A t_fix on free rows (0 on fixed rows); TPFA: b = f plus the
  // Dirichlet faces' 2 k_K |F| / h_d T_D
  if (c.tpfa) launch_tpfa_lift(c, f, lift, V.b, s);
  else if (lift) launch_residual(c, f, lift, nullptr, V.b, false, s);
  else launch_zero_fixed_copy(c, f, V.b, s);
  // x: free entries of the guess (or 0), fixed entries 0 during the iteration
  if (use_x0) launch_zero_fixed_copy(c, T, x, s);
  else launch_fill(c, x, 0.0, s);
  launch_fill(c, V.p, 0.0, s);
  launch_sc_reset(c, 1, maxit, s);
  launch_norm2(c, V.b, 0, rtol * rtol, s);  // bb, tol2
  HIP_TRY(hipMemsetAsync(V.xlo, 0, sizeof(float) * size_t(c.g.nn), s));
  if (use_x0) op_residual(c, V.b, x, nullptr, V.r, false, s);
  else launch_copy(c, V.b, V.r, s);
  launch_norm2(c, V.r, 1, 0.0, s);  // rr
  TRY(read_scalars(V, s));
  int restarts = 0;
  int status = MSMG_OK;
  double rel = 0.0;
  const double bb = V.sc_host->bb;
  if (!(bb > 0.0)) {
    // zero right-hand side: the solution is the lift alone
    launch_fill(c, x, 0.0, s);
    launch_finish_solution_dd(c, T, V.xlo, T_lo, lift, s);
    HIP_TRY(hipStreamSynchronize(s));
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->status = MSMG_OK;
      info->solve_ms = now_ms() - t0;
      info->setup_ms = h->setup_ms;
      info->n_c = h->n_c;
      info->n_cc = h->n_cc;
    }
    return MSMG_OK;
  }
  bool converged = V.sc_host->rr <= V.sc_host->tol2;
  if (converged) rel = std::sqrt(V.sc_host->rr / bb);
  int iters = 0;
  int timed_total = 0;
  if (!converged && maxit > 0) {
    precondition(h, c, V, V.r, V.z, nullptr, 0, s);
    launch_update_px(c, x, V.xlo, V.p, V.z, s);
    const int batch = h->opt.check_interval;
    const int max_timed = int(h->events.size() / 4);
    int launched = 0;
    while (true) {
      for (int it = 0; it < batch; ++it) {
        const bool tm = h->opt.timing && launched < max_timed;
        if (tm) HIP_TRY(hipEventRecord(h->events[4 * launched + 0], s));
        op_apply_pcg(c, V.p, V.q, s);
        if (tm) HIP_TRY(hipEventRecord(h->events[4 * launched + 1], s));
        launch_update_r(c, V.r, V.q, s);
        if (tm) HIP_TRY(hipEventRecord(h->events[4 * launched + 2], s));
        precondition(h, c, V, V.r, V.z, V.q, 1, s);
        if (tm) HIP_TRY(hipEventRecord(h->events[4 * launched + 3], s));
        launch_update_px(c, x, V.xlo, V.p, V.z, s);  // also x += alpha p of this step
        ++launched;
      }
      timed_total = std::min(launched, max_timed);
      TRY(read_scalars(V, s));
      const Scalars& S = *V.sc_host;
      if (!S.done) continue;
      // the step that stopped the iteration skipped the direction update:
      // add its alpha p to the iterate before x is read
      launch_update_x_pending(c, x, V.xlo, V.p, s);
      iters = S.iters;
      if (S.status == ST_CONV_RECURSIVE) {
        // confirm with the true residual
        op_residual(c, V.b, x, V.xlo, V.q, true, s);
        TRY(read_scalars(V, s));
        const double trr = V.sc_host->true_rr;
        if (trr <= V.sc_host->tol2) {
          converged = true;
          rel = std::sqrt(trr / bb);
          break;
        }
        if (V.sc_host->iters >= maxit || restarts >= 16) {
          status = MSMG_MAXIT;
          rel = std::sqrt(trr / bb);
          break;
        }
        // residual replacement and restart of the search direction
        ++restarts;
        launch_copy(c, V.q, V.r, s);
        launch_sc_reset(c, 0, 0, s);
        launch_fill(c, V.p, 0.0, s);
        precondition(h, c, V, V.r, V.z, nullptr, 0, s);
        launch_update_px(c, x, V.xlo, V.p, V.z, s);
        continue;
      }
      if (S.status == ST_SYNC_TIMEOUT)
        return fail(MSMG_ETIMEOUT, "a grid-wide wait of the coarse-level kernel exceeded its limit");
      status = (S.status == ST_MAXIT) ? MSMG_MAXIT : (S.status == ST_BREAKDOWN ? MSMG_BREAKDOWN : MSMG_NONFINITE);
      op_residual(c, V.b, x, V.xlo, V.q, true, s);
      TRY(read_scalars(V, s));
      rel = std::sqrt(V.sc_host->true_rr / bb);
      break;
    }
  } else if (!converged) {
    status = MSMG_MAXIT;
    rel = std::sqrt(V.sc_host->rr / bb);
  }
  launch_finish_solution_dd(c, T, V.xlo, T_lo, lift, s);
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipGetLastError());
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = status;
    info->iterations = iters;
    info->restarts = restarts;
    info->rel_res = rel;
    info->solve_ms = now_ms() - t0;
    info->setup_ms = h->setup_ms;
    fill_setup_timing(h, info);
    info->n_c = h->n_c;
    info->n_cc = h->n_cc;
    info->eig_unconverged = h->eig_unconverged;
    info->cc_unconverged = h->cc_unconverged;
    info->eig_ties = h->eig_ties;
    if (h->opt.timing) {
      // iterations after convergence return at once; average over the real ones
      const int nt = std::min(timed_total, iters);
      double ta = 0.0, tp = 0.0;
      for (int k = 0; k < nt; ++k) {
        float a = 0.f, p = 0.f;
        HIP_TRY(hipEventElapsedTime(&a, h->events[4 * k + 0], h->events[4 * k + 1]));
        HIP_TRY(hipEventElapsedTime(&p, h->events[4 * k + 2], h->events[4 * k + 3]));
        ta += a;
        tp += p;
      }
      info->timed = nt;
      info->apply_ms = nt ? ta / nt : 0.0;
      info->precond_ms = nt ? tp / nt : 0.0;
    }
  }
  if (status != MSMG_OK) g_last_error = "solve stopped before convergence";
  return status;
}

// Levels 0-2 of Algorithm 1 for the two right-hand sides of a batched pair:
// every kernel that reads the operator's coefficients (the conductivity copy,
// the Jacobi diagonal, the basis R_c, A_c, R_cc, A_cc^-1) runs once for both
// sides; a side whose solve has stopped skips its share.
static void precondition_pair(msmg_handle* h, const Ctx& c0, const Ctx& c1, VecSet& V0, VecSet& V1,
                              const double* q0, const double* q1, int mode, hipStream_t s) {
  launch_smooth_pair(c0, c1, V0.r, V1.r, V0.v_r1, V1.v_r1, s);                         // r1 = S^-1 r0
  if (V0.rpart && V1.rpart) {
    launch_vresidual_restrict_pair(c0, c1, V0.r, V1.r, V0.v_r1, V1.v_r1, (double*)V0.c_rc, (double*)V1.c_rc, s);
  } else {
    const bool v64 = (h->v_dt == DT_F64);
    launch_vresidual(c0, V0.r, true, V0.v_r1, v64, V0.v_res, s);
    launch_restrict(c0, V0.v_res, V0.c_rc, s);
    launch_vresidual(c1, V1.r, true, V1.v_r1, v64, V1.v_res, s);
    launch_restrict(c1, V1.v_res, V1.c_rc, s);
  }
  bool coarse_done = false;
  if (h->l1_blocks > 0) {
    if (launch_level1_pair(c0, c1, h->l1_blocks, (const double*)V0.c_rc, (const double*)V1.c_rc, (double*)V0.c_x0,
                           (double*)V1.c_x0, (double*)V0.c_t, (double*)V1.c_t, V0.rcc, V1.rcc, h->l1_bar,
                           LEVEL1_SPIN_LIMIT, s) == hipSuccess) {
      launch_prolong_pair(c0, c1, V0.v_r1, V1.v_r1, V0.c_x0, V1.c_x0, V0.v_r2, V1.v_r2, s);
      coarse_done = true;
    } else {
      (void)hipGetLastError();
      h->l1_blocks = 0;
    }
  }
  if (!coarse_done) {
    coarse_correction(h, c0, V0, s);
    coarse_correction(h, c1, V1, s);
  }
  launch_vresidual_pair(c0, c1, V0.r, V1.r, (const double*)V0.v_r2, (const double*)V1.v_r2, V0.v_res, V1.v_res, s);
  launch_smooth_output_pair(c0, c1, V0.v_res, V1.v_res, (const double*)V0.v_r2, (const double*)V1.v_r2, V0.z, V1.z,
                            V0.r, V1.r, q0, q1, mode, s);
}

// One side of a batched pair: its system, iterate and outcome.
struct PairSide {
  VecSet* V;
  Ctx c;
  const double* f;
  double* x;
  double* x_lo;
  const double* lift;
  double bb = 0.0;
  bool finished = false;
  int status = MSMG_OK, iters = 0, restarts = 0;
  double rel = 0.0;
};

// The state solve A T = f (with the set-up's fixed values) and the adjoint
// solve A_FF lambda = g (zero fixed values) of one set-up, as two PCG
// recurrences advanced together: each iteration's operator apply and
// preconditioner run once for both (precondition_pair); the vector updates,
// scalars, stopping tests and residual replacements stay per side.
static int solve_pair_impl(msmg_handle* h, const double* f, double* T, double* T_lo, const double* g, double* lam,
                           double* lam_lo, double rtol, int maxit, msmg_info* info_T, msmg_info* info_lam,
                           hipStream_t s) {
  if (!h || !f || !T || !g || !lam) return fail(MSMG_EINVAL, "NULL argument");
  if (!h->setup_done) return fail(MSMG_ESTATE, "msmg_setup has not completed");
  if (!h->vs[1].sc) return fail(MSMG_ESTATE, "the handle was created without options.pair_rhs");
  if (!(rtol >= 0.0) || maxit < 1) return fail(MSMG_EINVAL, "need rtol >= 0 and maxit >= 1");
  {
    const void* ps[] = {f, T, T_lo, g, lam, lam_lo};
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j)
        if (ps[i] && ps[i] == ps[j]) return fail(MSMG_EINVAL, "f, T, T_lo, g, lambda and lambda_lo must not alias");
  }
  const double t0 = now_ms();
  if (h->opt.lean_memory) h->basis_live = false;
  PairSide S[2];
  S[0].V = &h->vs[0];
  S[0].c = make_ctx(h, 0);
  S[0].f = f;
  S[0].x = T;
  S[0].x_lo = T_lo;
  S[0].lift = h->has_tfix ? h->tfix : nullptr;
  S[1].V = &h->vs[1];
  S[1].c = make_ctx(h, 1);
  S[1].f = g;
  S[1].x = lam;
  S[1].x_lo = lam_lo;
  S[1].lift = nullptr;
  bool trivial = false;
  for (PairSide& P : S) {
    VecSet& V = *P.V;
    const Ctx& c = P.c;
    if (P.lift) launch_residual(c, P.f, P.lift, nullptr, V.b, false, s);
    else launch_zero_fixed_copy(c, P.f, V.b, s);
    launch_fill(c, P.x, 0.0, s);
    launch_fill(c, V.p, 0.0, s);
    launch_sc_reset(c, 1, maxit, s);
    launch_norm2(c, V.b, 0, rtol * rtol, s);
    HIP_TRY(hipMemsetAsync(V.xlo, 0, sizeof(float) * size_t(c.g.nn), s));
    launch_copy(c, V.b, V.r, s);
    launch_norm2(c, V.r, 1, 0.0, s);
    TRY(read_scalars(V, s));
    P.bb = V.sc_host->bb;
    if (!(P.bb > 0.0) || V.sc_host->rr <= V.sc_host->tol2) trivial = true;
  }
  if (trivial) {
    // a zero or already converged right-hand side: two ordinary solves
    int r0 = solve_impl(h, f, T, T_lo, 0, rtol, maxit, info_T, s, false);
    if (r0 < 0) return r0;
    int r1 = solve_impl(h, g, lam, lam_lo, 0, rtol, maxit, info_lam, s, true);
    if (r1 < 0) return r1;
    return r0 != MSMG_OK ? r0 : r1;
  }
  precondition_pair(h, S[0].c, S[1].c, *S[0].V, *S[1].V, nullptr, nullptr, 0, s);
  for (PairSide& P : S) launch_update_px(P.c, P.x, P.V->xlo, P.V->p, P.V->z, s);
  const int batch = h->opt.check_interval;
  while (!(S[0].finished && S[1].finished)) {
    // once one side has stopped, the other runs the single-side kernels (the
    // pair kernels would still stage the stopped side's share in places)
    PairSide* alone = S[0].finished ? &S[1] : (S[1].finished ? &S[0] : nullptr);
    for (int it = 0; it < batch; ++it) {
      if (alone) {
        VecSet& V = *alone->V;
        launch_apply(alone->c, V.p, V.q, 1, s);
        launch_update_r(alone->c, V.r, V.q, s);
        precondition(h, alone->c, V, V.r, V.z, V.q, 1, s);
        launch_update_px(alone->c, alone->x, V.xlo, V.p, V.z, s);
        continue;
      }
      launch_apply_pair(S[0].c, S[1].c, S[0].V->p, S[1].V->p, S[0].V->q, S[1].V->q, s);
      for (PairSide& P : S) launch_update_r(P.c, P.V->r, P.V->q, s);
      precondition_pair(h, S[0].c, S[1].c, *S[0].V, *S[1].V, S[0].V->q, S[1].V->q, 1, s);
      for (PairSide& P : S) launch_update_px(P.c, P.x, P.V->xlo, P.V->p, P.V->z, s);
    }
    for (PairSide& P : S) {
      if (P.finished) continue;
      VecSet& V = *P.V;
      const Ctx& c = P.c;
      TRY(read_scalars(V, s));
      const Scalars Sc = *V.sc_host;
      if (!Sc.done) continue;
      launch_update_x_pending(c, P.x, V.xlo, V.p, s);
      P.iters = Sc.iters;
      if (Sc.status == ST_SYNC_TIMEOUT)
        return fail(MSMG_ETIMEOUT, "a grid-wide wait of the coarse-level kernel exceeded its limit");
      if (Sc.status == ST_CONV_RECURSIVE) {
        launch_residual(c, V.b, P.x, V.xlo, V.q, true, s);
        TRY(read_scalars(V, s));
        const double trr = V.sc_host->true_rr;
        if (trr <= V.sc_host->tol2) {
          P.finished = true;
          P.rel = std::sqrt(trr / P.bb);
          continue;
        }
        if (V.sc_host->iters >= maxit || P.restarts >= 16) {
          P.finished = true;
          P.status = MSMG_MAXIT;
          P.rel = std::sqrt(trr / P.bb);
          continue;
        }
        // residual replacement and restart of this side's direction (its
        // first preconditioner application runs alone); the next batch
        // takes it up again with the other side
        ++P.restarts;
        launch_copy(c, V.q, V.r, s);
        launch_sc_reset(c, 0, 0, s);
        launch_fill(c, V.p, 0.0, s);
        precondition(h, c, V, V.r, V.z, nullptr, 0, s);
        launch_update_px(c, P.x, V.xlo, V.p, V.z, s);
        continue;
      }
      P.finished = true;
      P.status = (Sc.status == ST_MAXIT) ? MSMG_MAXIT : (Sc.status == ST_BREAKDOWN ? MSMG_BREAKDOWN : MSMG_NONFINITE);
      launch_residual(c, V.b, P.x, V.xlo, V.q, true, s);
      TRY(read_scalars(V, s));
      P.rel = std::sqrt(V.sc_host->true_rr / P.bb);
    }
  }
  for (PairSide& P : S) launch_finish_solution_dd(P.c, P.x, P.V->xlo, P.x_lo, P.lift, s);
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipGetLastError());
  const double ms = now_ms() - t0;
  msmg_info* infos[2] = {info_T, info_lam};
  for (int k = 0; k < 2; ++k) {
    if (!infos[k]) continue;
    msmg_info* in = infos[k];
    std::memset(in, 0, sizeof(*in));
    in->status = S[k].status;
    in->iterations = S[k].iters;
    in->restarts = S[k].restarts;
    in->rel_res = S[k].rel;
    in->solve_ms = ms;
    in->setup_ms = h->setup_ms;
    fill_setup_timing(h, in);
    in->n_c = h->n_c;
    in->n_cc = h->n_cc;
    in->eig_unconverged = h->eig_unconverged;
    in->cc_unconverged = h->cc_unconverged;
    in->eig_ties = h->eig_ties;
  }
  const int st = S[0].status != MSMG_OK ? S[0].status : S[1].status;
  if (st != MSMG_OK) g_last_error = "a solve of the pair stopped before convergence";
  return st;
}

extern "C" int msmg_solve_pair(msmg_handle* h, const double* f, double* T, double* T_lo, const double* g,
                               double* lambda, double* lambda_lo, double rtol, int maxit, msmg_info* info_T,
                               msmg_info* info_lambda, hipStream_t s) {
  return solve_pair_impl(h, f, T, T_lo, g, lambda, lambda_lo, rtol, maxit, info_T, info_lambda, s);
}

extern "C" int msmg_solve(msmg_handle* h, const double* f, double* T, double* T_lo, int use_x0, double rtol,
                          int maxit, msmg_info* info, hipStream_t s) {
  return solve_impl(h, f, T, T_lo, use_x0, rtol, maxit, info, s, false);
}

extern "C" int msmg_solve_adjoint(msmg_handle* h, const double* g, double* lambda, double* lambda_lo, int use_x0,
                                  double rtol, int maxit, msmg_info* info, hipStream_t s) {
  return solve_impl(h, g, lambda, lambda_lo, use_x0, rtol, maxit, info, s, true);
}

extern "C" int msmg_export(msmg_handle* h, int what, void* host_out, size_t bytes) {
  if (!h || !host_out) return fail(MSMG_EINVAL, "NULL argument");
  if (!h->setup_done) return fail(MSMG_ESTATE, "msmg_setup has not completed");
  if (!h->mg) return fail(MSMG_ESTATE, "no coarse spaces with the smoother-only preconditioner");
  const Hier& hh = h->hier;
  const void* src = nullptr;
  size_t need = 0;
  switch (what) {
    case 0: src = h->evals; need = (size_t)h->n_c * 8; break;
    case 1:
      if (!h->basis_live) return fail(MSMG_EINVAL, "lean_memory: the FP64 basis was overwritten by a solve, apply or preconditioner call");
      src = h->Rc64; need = (size_t)h->g.nn * hh.Lc * 8; break;
    case 2: src = h->Ac64; need = (size_t)hh.ncells * 27 * hh.Lc * hh.Lc * 8; break;
    case 3: src = h->cc_evals; need = (size_t)h->n_cc * 8; break;
    case 4:
      if (!h->scratch.acc_copy) return fail(MSMG_EINVAL, "lean_memory: no copy of A_cc is kept");
      src = h->scratch.acc_copy; need = (size_t)h->n_cc * h->n_cc * 8; break;
    case 5: src = h->cell_status; need = (size_t)hh.ncells * 4; break;
    default: return fail(MSMG_EINVAL, "unknown export id");
  }
  if (bytes < need) return fail(MSMG_EINVAL, "output buffer too small: need " + std::to_string(need) + " bytes");
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(host_out, src, need, hipMemcpyDeviceToHost));
  return MSMG_OK;
}

// ---------------------------------------------------------------------------
// Design update helpers of the optimisation loop.

extern "C" int msmg_density_filter(int nx, int ny, int nz, double radius, const double* in, double* out,
                                   int transpose, hipStream_t s) {
  if (nx < 1 || ny < 1 || nz < 1) return fail(MSMG_EINVAL, "mesh sizes must be >= 1");
  if (!(radius > 1.0) || radius > 4.0) return fail(MSMG_EINVAL, "filter radius must be in (1, 4] elements");
  if (!in || !out) return fail(MSMG_EINVAL, "NULL argument");
  if (in == out) return fail(MSMG_EINVAL, "in and out must not alias");
  launch_density_filter(nx, ny, nz, radius, in, out, transpose != 0, s);
  HIP_TRY(hipGetLastError());
  return MSMG_OK;
}

extern "C" int msmg_oc_update(msmg_handle* h, const double* x, const double* dc, const double* dv,
                              double volume_fraction, double move, double eta, double x_min, double* x_new,
                              double* lambda, hipStream_t s) {
  if (!h || !x || !dc || !dv || !x_new) return fail(MSMG_EINVAL, "NULL argument");
  if (x_new == x || x_new == dc || x_new == dv) return fail(MSMG_EINVAL, "x_new must not alias the inputs");
  if (!(volume_fraction > 0.0 && volume_fraction <= 1.0)) return fail(MSMG_EINVAL, "volume fraction in (0, 1]");
  if (!(move > 0.0) || !(eta > 0.0) || !(x_min >= 0.0 && x_min < 1.0))
    return fail(MSMG_EINVAL, "need move > 0, eta > 0, 0 <= x_min < 1");
  const long long ne = h->g.ne;
  launch_oc_update(ne, x, dc, dv, volume_fraction * double(ne), move, eta, x_min, x_new, lambda, h->oc_state,
                   h->vs[0].partials, h->vs[0].counter, 8, s);
  HIP_TRY(hipGetLastError());
  return MSMG_OK;
}

extern "C" int msmg_dot(msmg_handle* h, const double* a, const double* b, long long n, double* out, hipStream_t s) {
  if (!h || !a || !b || !out) return fail(MSMG_EINVAL, "NULL argument");
  if (n < 0 || n > h->g.nn) return fail(MSMG_EINVAL, "need 0 <= n <= the handle's unknowns");
  launch_dot(a, b, n, out, h->vs[0].partials, h->vs[0].counter, h->red_blocks, s);
  HIP_TRY(hipGetLastError());
  return MSMG_OK;
}

extern "C" int msmg_scale(const double* x, long long n, double c, const double* s_dev, double* y, hipStream_t s) {
  if (!x || !y || n < 0) return fail(MSMG_EINVAL, "bad arguments");
  launch_scale(x, n, c, s_dev, y, s);
  HIP_TRY(hipGetLastError());
  return MSMG_OK;
}

extern "C" int msmg_mma_update(msmg_handle* h, int iter, const double* x, const double* xold1, const double* xold2,
                               double* low, double* upp, const double* df0, const double* dv, double volume_fraction,
                               double move, double x_min, double* x_new, double* lambda, hipStream_t s) {
  if (!h || !x || !xold1 || !xold2 || !low || !upp || !df0 || !dv || !x_new) return fail(MSMG_EINVAL, "NULL argument");
  if (iter < 0) return fail(MSMG_EINVAL, "iter must be >= 0");
  if (x_new == x || x_new == xold1 || x_new == xold2 || x_new == low || x_new == upp || x_new == df0 || x_new == dv ||
      low == upp)
    return fail(MSMG_EINVAL, "x_new, low and upp must not alias the other arrays");
  if (!(volume_fraction > 0.0 && volume_fraction <= 1.0)) return fail(MSMG_EINVAL, "volume fraction in (0, 1]");
  if (!(move > 0.0) || !(x_min >= 0.0 && x_min < 1.0)) return fail(MSMG_EINVAL, "need move > 0 and 0 <= x_min < 1");
  launch_mma_update(iter, h->g.ne, x, xold1, xold2, low, upp, df0, dv, volume_fraction, move, x_min, 1.0, x_new,
                    lambda, h->oc_state, h->vs[0].partials, h->vs[0].counter, 8, s);
  HIP_TRY(hipGetLastError());
  return MSMG_OK;
}

// Largest design the allocation-free update takes (its scratch does not grow
// with the design; the bound keeps element indices and volumes exact).
static constexpr long long OC_NOALLOC_MAX_ELEMENTS = 1LL << 40;

extern "C" int msmg_oc_update_noalloc(int nx, int ny, int nz, const double* x, const double* dc, const double* dv,
                                      double volume_fraction, double move, double eta, double x_min, double* x_new,
                                      double* lambda, hipStream_t s) {
  if (nx < 1 || ny < 1 || nz < 1) return fail(MSMG_EINVAL, "mesh sizes must be >= 1");
  const long long ne = (long long)nx * ny * nz;
  if (ne > OC_NOALLOC_MAX_ELEMENTS)
    return fail(MSMG_EINVAL, "design has " + std::to_string(ne) + " elements; the allocation-free update takes at most " +
                                 std::to_string(OC_NOALLOC_MAX_ELEMENTS));
  if (!x || !dc || !dv || !x_new) return fail(MSMG_EINVAL, "NULL argument");
  if (x_new == x || x_new == dc || x_new == dv) return fail(MSMG_EINVAL, "x_new must not alias the inputs");
  if (!(volume_fraction > 0.0 && volume_fraction <= 1.0)) return fail(MSMG_EINVAL, "volume fraction in (0, 1]");
  if (!(move > 0.0) || !(eta > 0.0) || !(x_min >= 0.0 && x_min < 1.0))
    return fail(MSMG_EINVAL, "need move > 0, eta > 0, 0 <= x_min < 1");
  void* scratch = nullptr;
  HIP_TRY(oc_scratch_device_ptr(&scratch));
  launch_oc_update_scratch(ne, x, dc, dv, volume_fraction * double(ne), move, eta, x_min, x_new, lambda, scratch, 8, s);
  HIP_TRY(hipGetLastError());
  return MSMG_OK;
}
