// Internal declarations shared by the kernel files and the runtime.
#pragma once

#include <algorithm>

#include "common.h"
#include "march.h"

namespace msmg {

enum DType { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };

constexpr int LC_MAX = 8;     // basis vectors per coarse cell (upper bound)
constexpr int CHEB_MAX = 16;  // Chebyshev degree upper bound

struct ChebCoef {
  int degree;
  double inv_theta;  // 1/theta
  double c0, c1;     // fused first two steps: out = c0 z1 + c1 D^-1 (r - A z1)
  double step_a[CHEB_MAX], step_b[CHEB_MAX];
};

// Level-1 / level-2 data layout shared with the kernels.
struct CoarseCtx {
  const void* Ac;        // [ncells][27][Lc][Lc]  (a_dt)
  const void* AcDinv;    // [ncells][Lc][Lc]      (a_dt)
  int a_dt;
  const void* Rcc;       // per cc cell J: [Lcc][nd_J] at offset Lcc * cc_ptr[J]   (v_dt)
  const int* cc_ptr;     // [ncc + 1] offsets of cc-local dofs
  const int* cc_dofs;    // [n_c] global coarse dof of each cc-local dof
  const int* dof_cc;     // [n_c] cc cell of each coarse dof
  const int* dof_loc;    // [n_c] local index of each coarse dof in its cc cell
  const double* AccInv;  // [n_cc][n_cc] FP64 inverse of A_cc
  int n_c, n_cc;
};

// Partial sums of the restriction fused into the cycle's first residual: the
// march runs on z chunks of whole coarse cells (czc of them, the last chunk
// also takes the remainder planes of the last cell); a workgroup's MX x MY
// column block meets at most nlx x nly coarse cells per z-cell, so each
// workgroup owns nlx * nly * nlz slots of L_c sums.
struct RestrictGeo {
  March m;            // cell-aligned march: zc = czc * H, nzc = ceil(ncz / czc)
  int czc;
  int nlx, nly, nlz;  // local coarse cells per workgroup along x, y, z
  long long slots;    // workgroups x local cells (each slot holds L_c doubles)
};
RestrictGeo make_restrict_geo(const Geo& g, const Hier& h, long long resident);
// The fused residual + restriction covers cell sizes that divide the march's
// tile rows into whole lane groups: H in {2, 4, 8, 16}.
inline bool restrict_fusable(const Hier& h) { return h.H == 2 || h.H == 4 || h.H == 8 || h.H == 16; }

struct Ctx {
  Geo g;
  Stencil st;
  Hier h;
  Material mat;
  int CX;             // coarse cells per tile along x
  long long ntiles;
  March mg;           // plane-march decomposition of the fine stencil kernels
  March mgl;          // the same for the LDS-queue apply (its own tile shape)
  const void* rho;    // canonical density (rho_dt)
  int rho_dt;
  const double* kc;   // FP64 element conductivities for an FP64 density (null for FP32:
                      // the apply forms them from rho)
  const void* kv;     // element conductivities read by the cycle (kv_dt; may alias kc)
  int kv_dt;
  const uint32_t* bits;
  void* dinv;         // Jacobi D^-1, V-cycle type
  int v_dt;           // V-cycle vector type
  void* Rc;           // [nn][Lc] basis, b_dt
  int b_dt;
  ChebCoef cheb;
  Scalars* sc;
  double* partials;
  unsigned* counter;
  int red_blocks;
  void* vc_t0;        // V-cycle scratch vectors (v_dt)
  void* vc_t1;
  RestrictGeo rg;     // fused residual + restriction (when restrict_fusable)
  double* rpart;      // its per-workgroup partial sums, rg.slots * Lc doubles
  CoarseCtx cc;
  // cell-centred two-point flux discretisation: unknowns are the cells (g.nn =
  // g.ne, g.nnx = g.nx, ...), kc holds the FP64 cell conductivities, dface the
  // Dirichlet face flags of each cell (bit 0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z)
  int tpfa;
  const uint8_t* dface;
};

// PCG scalars after a preconditioner application: tt = (z^T r, z^T q).
MSMG_DEV void vc_finish(Scalars* sc, const double* tt, int mode) {
  sc->zr = tt[0];
  sc->zq = tt[1];
  if (!(tt[0] > 0.0)) {
    sc->status = (tt[0] == tt[0]) ? ST_BREAKDOWN : ST_NONFINITE;
    sc->done = 1;
    return;
  }
  if (mode == 0) {
    sc->beta = 0.0;
  } else {
    // beta = z^T (r_new - r_old) / rz_old with r_old = r_new + alpha q
    sc->beta = -sc->alpha * tt[1] / sc->rz;
  }
  sc->rz = tt[0];
}

// Slots of the handle's 16-word counter block (zero between kernels unless
// noted): the ticket of grid_reduce, the fixed-node count of a set-up (left
// holding the count).
constexpr int CTR_REDUCE = 0, CTR_FIXED = 8;

// 1-D launch size: one thread per item, at most `cap` workgroups (grid-stride loops)
inline int grid1d(long long n, int bs, int cap = 4096) {
  long long b = (n + bs - 1) / bs;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return int(b);
}

// design update (density filter, optimality criteria)
void launch_density_filter(int nx, int ny, int nz, double r, const double* in, double* out, bool transpose,
                           hipStream_t s);
void launch_oc_update(long long ne, const double* x, const double* dc, const double* dv, double volume, double move,
                      double eta, double xmin, double* xnew, double* lam_out, void* state, double* partials,
                      unsigned* counter, int passes, hipStream_t s);
// method of moving asymptotes for one volume constraint: low, upp in/out
void launch_mma_update(int it, long long ne, const double* x, const double* x1, const double* x2, double* low,
                       double* upp, const double* df0, const double* dv, double vf, double move, double xmin,
                       double xmax, double* xnew, double* lam_out, void* state, double* partials, unsigned* counter,
                       int passes, hipStream_t s);
// the same with the scratch in a fixed per-device array (no allocation)
hipError_t oc_scratch_device_ptr(void** out);
size_t oc_scratch_bytes();
void launch_oc_update_scratch(long long ne, const double* x, const double* dc, const double* dv, double volume,
                              double move, double eta, double xmin, double* xnew, double* lam_out, void* scratch_ptr,
                              int passes, hipStream_t s);

// objective values and chain-rule scalings: *out = a^T b (fixed order, the
// handle's reduction scratch), y = c * (*sdev) * x (sdev may be null: y = c x)
void launch_dot(const double* a, const double* b, long long n, double* out, double* partials, unsigned* counter,
                int max_blocks, hipStream_t s);
void launch_scale(const double* x, long long n, double c, const double* sdev, double* y, hipStream_t s);

// fine level
long long march_resident_blocks();  // marching workgroups the device runs at once
long long apply_resident_blocks();  // the same for the LDS-queue apply
void launch_pack_mask(const uint8_t* mask, uint32_t* bits, long long nn, hipStream_t s);
void launch_convert(const void* in, int din, void* out, int dout, long long n, hipStream_t s);
void launch_conductivity(const Ctx& c, const void* rho, int rdt, void* kc, int kdt, hipStream_t s);
void launch_diag_inv(const Ctx& c, const void* rho, int rdt, void* dinv, int vdt, hipStream_t s);
void launch_zero_fixed_copy(const Ctx& c, const double* in, double* out, hipStream_t s);
void launch_finish_solution(const Ctx& c, double* T, const double* tfix, hipStream_t s);
void launch_norm2(const Ctx& c, const double* v, int what, double rtol2, hipStream_t s);
void launch_update_r(const Ctx& c, double* r, const double* q, hipStream_t s);
void launch_update_x_pending(const Ctx& c, double* x, float* xlo, const double* p, hipStream_t s);
void launch_finish_solution_dd(const Ctx& c, double* T, const float* xlo, double* tlo, const double* tfix, hipStream_t s);
void launch_update_px(const Ctx& c, double* x, float* xlo, double* p, const double* z, hipStream_t s);
// y = A x (mode 0), with p^T A p -> alpha (mode 1), or P A P xraw + (I - P) xraw
// (mode 2, x = xraw with zero fixed entries).  x is zero on fixed nodes.
void launch_apply(const Ctx& c, const double* x, double* y, int mode, hipStream_t s, const double* xraw = nullptr);
void launch_residual(const Ctx& c, const double* b, const double* x, const float* xlo, double* y, bool reduce,
                     hipStream_t s);
void launch_smooth(const Ctx& c, const void* in, bool in_is_f64, void* out, hipStream_t s);
void launch_restrict(const Ctx& c, const void* r, void* rc, hipStream_t s);
void launch_prolong(const Ctx& c, const void* base, const void* e1, const void* e2, void* out, hipStream_t s);
void launch_vresidual(const Ctx& c, const void* r, bool r_is_f64, const void* x, bool x_is_f64, void* out,
                      hipStream_t s);
// out = r - A x2 with x2 = base + R_c^T (e1 + e2) formed in the march (e2 may
// be null); x2 is written too.  The prolongation and the residual of the two
// separate launches, bit for bit.
void launch_vresidual_prolong(const Ctx& c, const double* r, const void* base, const double* e1, const double* e2,
                              void* out, double* x2, hipStream_t s);
// rc = R_c (r - A x) without storing the residual (r FP64, x of the cycle's
// vector type): the fused march writes per-workgroup partials, a second kernel
// adds them per coarse cell in a fixed order.  Only when restrict_fusable.
void launch_vresidual_restrict(const Ctx& c, const double* r, const void* x, double* rc, hipStream_t s);
void launch_vc_output(const Ctx& c, const void* a, bool a_is_f64, const void* b, double* z, const double* r,
                      const double* q, int mode, hipStream_t s);
// Degree-2 post-smoother fused with the output: z = base + S^-1 in (base may be
// null) with the PCG reduction `mode`; only when smooth_output_fused(c).
bool smooth_output_fused(const Ctx& c);
void launch_smooth_output(const Ctx& c, const void* in, bool in_is_f64, const double* base, double* z,
                          const double* r, const double* q, int mode, hipStream_t s);
// The same kernels for the two right-hand sides of a batched pair (a and b:
// contexts of the two sides; the coefficients are a's, shared).  The
// smoother, the residual after the coarse correction and the fused output are
// the degree-2 forms; inputs and outputs as in the single-side launchers.
void launch_apply_pair(const Ctx& a, const Ctx& b, const double* xa, const double* xb, double* ya, double* yb,
                       hipStream_t s);
void launch_smooth_pair(const Ctx& a, const Ctx& b, const double* ina, const double* inb, void* outa, void* outb,
                        hipStream_t s);
void launch_vresidual_restrict_pair(const Ctx& a, const Ctx& b, const double* ra, const double* rb, const void* xa,
                                    const void* xb, double* rca, double* rcb, hipStream_t s);
void launch_prolong_pair(const Ctx& a, const Ctx& b, const void* basea, const void* baseb, const void* ea,
                         const void* eb, void* outa, void* outb, hipStream_t s);
void launch_vresidual_pair(const Ctx& a, const Ctx& b, const double* ra, const double* rb, const double* xa,
                           const double* xb, void* outa, void* outb, hipStream_t s);
void launch_smooth_output_pair(const Ctx& a, const Ctx& b, const void* ina, const void* inb, const double* basea,
                               const double* baseb, double* za, double* zb, const double* ra, const double* rb,
                               const double* qa, const double* qb, int mode, hipStream_t s);
void launch_sensitivity(const Ctx& c, const double* T, const double* lam, double* dc, hipStream_t s);
void launch_sensitivity_heat_source(const Ctx& c, const double* T, const double* lam, double f0, double* dc,
                                    hipStream_t s);
void launch_heat_source_load(const Ctx& c, double f0, double* f, hipStream_t s);
void launch_element_load(const Geo& g, const double* src, double sconst, double* f, hipStream_t s);
void launch_prolong_nodal(int nx, int ny, int nz, const double* tc, double* tf, hipStream_t s);
void launch_prolong_element(int nx, int ny, int nz, const void* rc, void* rf, int dt, hipStream_t s);
// one read of x (nn) and k (ne <= nn) and one write of y (nn), coalesced: the
// operator apply's traffic without its stencil (nn, ne even)
void launch_stream_ceiling(const double* x, const double* k, double* y, long long nn, long long ne, hipStream_t s);

// cell-centred two-point flux operator (Ctx.tpfa): FP64 vectors, FP64 basis
bool tpfa_grid_fits(const Ctx& c);  // the stencil grid fits the reduction's block budget
void launch_tpfa_apply(const Ctx& c, const double* x, double* y, bool reduce, hipStream_t s);
void launch_tpfa_residual(const Ctx& c, const double* b, const double* x, const float* xlo, double* y, bool reduce,
                          hipStream_t s);
void launch_tpfa_vresidual(const Ctx& c, const double* r, const double* x, double* out, hipStream_t s);
void launch_tpfa_smooth(const Ctx& c, const double* in, double* out, hipStream_t s);
// degree-2 post-smoother fused with the output z = base + S^-1 res (PCG reduction `mode`)
void launch_tpfa_smooth_output(const Ctx& c, const double* res, const double* base, double* z, const double* r,
                               const double* q, int mode, hipStream_t s);
void launch_tpfa_restrict(const Ctx& c, const double* v, double* rc, hipStream_t s);
// rc = R_c (r - A x) without storing the residual: per-(coarse cell, row)
// partials in part (tpfa_restrict_slots(c) * Lc doubles), then a fixed-order
// sum; only when tpfa_restrict_fusable(c) (H in {4, 8, 16} dividing every axis)
bool tpfa_restrict_fusable(const Ctx& c);
long long tpfa_restrict_slots(const Ctx& c);
void launch_tpfa_vresidual_restrict(const Ctx& c, const double* r, const double* x, double* part, double* rc,
                                    hipStream_t s);
void launch_tpfa_prolong(const Ctx& c, const double* base, const double* e1, const double* e2, double* out,
                         hipStream_t s);
void launch_tpfa_diag_inv(const Ctx& c, double* dinv, hipStream_t s);
void launch_tpfa_lift(const Ctx& c, const double* f, const double* td, double* b, hipStream_t s);
void launch_tpfa_flags(const Ctx& c, const uint8_t* in, uint8_t* out, unsigned long long* counts, hipStream_t s);
void launch_tpfa_cell_load(const Ctx& c, const double* src, double sconst, double* f, hipStream_t s);
void launch_tpfa_heat_source_load(const Ctx& c, double f0, double* f, hipStream_t s);
int launch_tpfa_galerkin(const Ctx& c, const void* R, int b_dt, int drop_cc, double* out, hipStream_t s);
// design sensitivities: lam null = the compliance (lam = T), td null = zero
// Dirichlet values, source: the heat source's term with f0
void launch_tpfa_sensitivity(const Ctx& c, const double* T, const double* lam, const double* td, double f0,
                             bool source, double* dc, hipStream_t s);

// coarse levels (V-cycle)
void launch_gs_sweep(const Ctx& c, const void* b, void* x, bool forward, hipStream_t s);
void launch_ac_residual(const Ctx& c, const void* b, const void* x, void* t, hipStream_t s);
void launch_cc_restrict(const Ctx& c, const void* t, double* rcc, hipStream_t s);
void launch_acc_solve(const Ctx& c, const double* rcc, double* ecc, hipStream_t s);
void launch_cc_prolong(const Ctx& c, const void* base, const double* ecc, void* out, hipStream_t s);
// Levels 1 and 2 of Algorithm 1 (coarse sweeps, coarse-coarse restriction,
// direct solve, prolongation) in one launch of `blocks` workgroups with
// grid-wide barriers between the steps (level1_blocks(): one per compute unit,
// within the device's co-resident capacity; 0 when that cannot be had).
// Input rc; output x = e_c, the coarse correction; t and rcc are its scratch;
// bar: level1_barrier_words() zeroed words.  FP64 A_c only.
hipError_t launch_level1_pair(const Ctx& c0, const Ctx& c1, int blocks, const double* rc0, const double* rc1,
                              double* x0, double* x1, double* t0, double* t1, double* rcc0, double* rcc1,
                              unsigned* bar, unsigned spin_limit, hipStream_t s);
int level1_blocks();
int level1_barrier_words();  // size of its barrier buffer (unsigned words)
hipError_t launch_level1(const Ctx& c, int blocks, const double* rc, double* x, double* t, double* rcc,
                         unsigned* bar, unsigned spin_limit, hipStream_t s);

}  // namespace msmg
