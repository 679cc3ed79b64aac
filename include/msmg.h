/*
 * msmg.h -- C ABI of the MI355X multiscale-multigrid PCG solver for SIMP
 * steady heat conduction on structured Q1 hexahedral meshes.
 *
 * Problem (paper section 2): -div(k(rho) grad T) = f on the box
 * [0,lx] x [0,ly] x [0,lz] cut into nx * ny * nz trilinear hexahedra, with
 * k = k_min + rho^p (k_max - k_min) per element (section 2.1, eq. material),
 * fixed temperatures on a nodal mask and adiabatic boundaries elsewhere.  The
 * discrete system A T = f (section 2.2, eq. new linear system; here nodal Q1
 * instead of the paper's two-point flux volumes) is solved by preconditioned
 * CG whose preconditioner is the three-grid cycle of Algorithm 1 with coarse
 * spaces from the local spectral problems eq. (spepb) and eq. (spectral cc)
 * (section 3).  Sensitivities follow the adjoint of section 2.3.
 *
 * Conventions
 *   - Node n = (k*(ny+1) + j)*(nx+1) + i, element e = (k*ny + j)*nx + i
 *     (x fastest).  Nodal arrays hold (nx+1)(ny+1)(nz+1) entries, element
 *     arrays nx*ny*nz.
 *   - Every array argument is a HIP device pointer unless stated otherwise.
 *     The caller owns it; the library never keeps it past the call except
 *     where stated.  The library owns the handle and all its device memory.
 *   - Work is enqueued on the given stream; one handle is used from one
 *     stream at a time.  msmg_solve blocks until the solve ends.
 *   - Return codes: 0 success; > 0 solve ended without convergence (result
 *     still written); < 0 error (nothing useful written), see msmg_last_error.
 */
#ifndef MSMG_H
#define MSMG_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct msmg_handle msmg_handle;

typedef enum { MSMG_F64 = 0, MSMG_F32 = 1, MSMG_BF16 = 2 } msmg_dtype;

typedef enum { MSMG_PC_MULTIGRID = 0, MSMG_PC_SMOOTHER = 1 } msmg_pc_kind;

/* Discretisation of the heat equation.
 *   MSMG_Q1:   trilinear (Q1) elements; unknowns are the (nx+1)(ny+1)(nz+1)
 *              mesh nodes, Dirichlet data live on fixed nodes.
 *   MSMG_TPFA: the paper's cell-centred two-point flux finite volumes
 *              (section 2.2, eq. flux and eq. new linear system); unknowns
 *              are the nx*ny*nz cells (numbered like the elements), the face
 *              conductivity is the harmonic mean of the two cells', and
 *              Dirichlet data live on flagged boundary faces, each closing
 *              its cell's balance over half a cell (2 k_K |F| / h_d). */
typedef enum { MSMG_Q1 = 0, MSMG_TPFA = 1 } msmg_discretisation;

enum {
  MSMG_OK = 0,
  MSMG_MAXIT = 1,       /* iteration limit reached                      */
  MSMG_BREAKDOWN = 2,   /* p^T A p <= 0 or r^T z <= 0                    */
  MSMG_NONFINITE = 3,   /* NaN / Inf in the iteration                    */
  MSMG_EINVAL = -1,     /* invalid argument                               */
  MSMG_ENOMEM = -2,     /* device allocation failed                       */
  MSMG_EHIP = -3,       /* HIP runtime error                              */
  MSMG_ESETUP = -4,     /* coarse-space construction failed               */
  MSMG_ESINGULAR = -5,  /* no fixed-temperature node: A is singular       */
  MSMG_ESTATE = -6,     /* call order violated (e.g. solve before setup)  */
  MSMG_ETIMEOUT = -7    /* a bounded device-side wait gave up (the
                           coarse-level kernel's grid-wide barrier)       */
};

/* Solver options (section 4 of the paper fixes sd, L_c, L_cc as tunables;
 * the smoother choice and precision are this library's). */
typedef struct msmg_options {
  int H;               /* coarse cell size in elements per axis (>= 2)          [8]    */
  int sd;              /* coarse cells per coarse-coarse cell per axis (>= 1)   [8]    */
  int Lc;              /* eigenvectors per coarse cell, 1..8 (eq. spepb)        [4]    */
  int Lcc;             /* eigenvectors per coarse-coarse cell (eq. spectral cc) [17]   */
  int cheb_degree;     /* level-0 Chebyshev-Jacobi steps, 1..16                 [2]    */
  double cheb_lo;      /* smoothing interval on D^-1 A                          [0.15] */
  double cheb_hi;      /*                                                        [1.5]  */
  int vcycle_dtype;    /* MSMG_F64 or MSMG_F32 vectors inside the cycle         [F64]  */
  int rho_v_dtype;     /* conductivity copy read by the cycle: F64/F32/BF16     [F64]
                          (the FP64 k = k_min + rho^p (k_max - k_min) of each
                          element, rounded once per set-up; rho itself is kept
                          at its canonical precision)                             */
  int basis_dtype;     /* storage of R_c: F64/F32/BF16                          [F64]  */
                       /* (an FP64 cycle takes equal copy types, or BF16 + F32)        */
  int pc_kind;         /* MSMG_PC_MULTIGRID or MSMG_PC_SMOOTHER (level 0 only)  [MG]   */
  int check_interval;  /* PCG iterations between host convergence polls        [8]    */
  int eig_block;       /* level-1 subspace block size (0 = tuned)               [0]    */
  int eig_degree;      /* level-1 filter degree (0 = tuned)                     [0]    */
  int eig_maxit;       /* outer subspace iterations per cell                    [60]   */
  double eig_tol;      /* residual tolerance relative to the spectral bound     [1e-12]*/
  int cc_block;        /* coarse-coarse subspace block size (0 = Lcc + guard)   [0]    */
  int cc_degree;       /* unused (kept for the layout of this struct)           [16]   */
  int cc_maxit;        /* coarse-coarse outer iterations                        [60]   */
  int autotune;        /* 1: tune the level-1 launch shape on first setup       [1]    */
  const char* tune_cache; /* host path of the tuning cache file, or NULL       [NULL] */
  int timing;          /* 1: time the operator apply and the preconditioner of  [0]
                          every PCG iteration with HIP events on the solve stream */
  int eig_warm_start;  /* 1: start the level-1 eigensolver of a set-up from the  [0]
                          previous set-up's basis (designs that change little
                          between set-ups, e.g. an optimisation loop)            */
  int rho_storage;     /* MSMG_F64 or MSMG_F32: storage of the canonical density [F64]
                          copy; F32 storage takes F32 densities only             */
  int lean_memory;     /* 1: the FP64 basis master shares the PCG work vectors   [0]
                          (read only during a set-up; msmg_export of it works
                          until the next solve, apply or preconditioner call),
                          set-up-only coarse-coarse blocks share the cycle's
                          FP64 iterate, and no copy of A_cc is kept (export 4
                          fails).  Excludes eig_warm_start.  For the largest
                          grids (1024^3 on one GPU).                             */
  int cc_group;        /* coarse-coarse cells whose dense shifted matrices the   [0]
                          set-up holds at once (0 = as many as fit in 24 GB)     */
  int coarse_fused;    /* bit 0: levels 1 and 2 of each cycle in one launch      [7]
                          (one workgroup per compute unit, grid-wide barriers
                          between the steps; taken while n_c <= 262,144, larger
                          coarse levels run one launch per step); bit 1: the restriction fused into the cycle's
                          first residual (H = 2, 4, 8 or 16); bit 2: the
                          prolongation fused into the residual after the coarse
                          correction.  Cleared bits run one launch per step.
                          The same arithmetic up to the order of the sums.       */
  int pair_rhs;        /* 1: allocate a second set of PCG and cycle vectors     [0]
                          for msmg_solve_pair (about 11 nodal vectors more;
                          needs the multigrid kind with cheb_degree 2)           */
  int discretisation;  /* MSMG_Q1 or MSMG_TPFA                                  [Q1]
                          TPFA: FP64 cycle vectors, density copy and basis
                          (the dtype options at F64), no pair_rhs, no
                          lean_memory, and cheb_hi >= 2 (the Jacobi-scaled
                          TPFA matrix reaches close to 2; [0.2, 2] suits it).
                          Vectors ("nodal" below) then hold one value per
                          cell; coarse cells group H^3 cells (remainders join
                          the last); coarse_fused bit 1 fuses the restriction
                          into the first residual when H is 4, 8 or 16 and
                          divides every axis; bit 2 does not apply.             */
  double lc_threshold; /* > 0: adaptive local basis size l_c^i per coarse cell  [0]
                          (section 3 allows one per cell): cell i keeps its
                          eigenpairs of eq. spepb with lambda <= lc_threshold *
                          (pi / (H h_max))^2, at least one and at most Lc (Lc
                          is then the maximum; Lc <= 7).  The coarse levels
                          keep Lc slots per cell, unused ones decoupled.       */
} msmg_options;

/* Solve report. */
typedef struct msmg_info {
  int status;              /* return code of msmg_solve                          */
  int iterations;          /* PCG iterations                                     */
  int restarts;            /* residual replacements after a failed true check    */
  double rel_res;          /* final true ||b - A T||_2 / ||b||_2 on free nodes   */
  double solve_ms;         /* wall time of the solve, host side                  */
  double setup_ms;         /* wall time of the last msmg_setup                   */
  int n_c, n_cc;           /* coarse and coarse-coarse dimensions                */
  int eig_unconverged;     /* level-1 cells that hit eig_maxit                   */
  int cc_unconverged;      /* coarse-coarse cells that hit cc_maxit              */
  int eig_ties;            /* level-1 cells whose cutoff gap is below 1e-8 bound */
  int timed;               /* iterations timed (options.timing)                  */
  double apply_ms;         /* mean duration of the PCG operator apply kernel     */
  double precond_ms;       /* mean duration of one preconditioner application    */
  double setup_phase_ms[4]; /* timing: the last set-up's phases (HIP events):    */
                            /* local spectral problems, Galerkin A_c, the        */
                            /* coarse-coarse problems, A_cc and its inverse      */
  double setup_dense_ms;    /* timing: of these, the dense Gauss-Jordan inverses */
  double setup_dense_gflop; /* their flop count, n^3 per n x n inverse           */
} msmg_info;

/* Hierarchy sizes for a mesh and options; host only, no GPU needed. */
typedef struct msmg_plan {
  int ncx, ncy, ncz, ncells;   /* coarse cells                                */
  int nccx, nccy, nccz, ncc;   /* coarse-coarse cells                         */
  int n_c, n_cc;               /* padded coarse dimension, cc dimension       */
  int max_cell_nodes;          /* largest owned-node box of a coarse cell     */
  int max_cc_dofs;             /* largest coarse-coarse local dimension       */
  long long nodes, elements;
  long long device_bytes;      /* device memory the handle will hold          */
} msmg_plan;

/* Fill *opt with the defaults listed above. */
void msmg_default_options(msmg_options* opt);

/* Hierarchy plan for nx*ny*nz elements (host only).  Returns MSMG_EINVAL when
 * the sizes or options cannot be used. */
int msmg_query_plan(int nx, int ny, int nz, const msmg_options* opt, msmg_plan* out);

/* Allocate a handle for an nx*ny*nz mesh of the box lx*ly*lz (opt NULL =
 * defaults).  Allocates all device memory up front on the current device. */
int msmg_create(msmg_handle** h, int nx, int ny, int nz, double lx, double ly, double lz,
                const msmg_options* opt);

/* Per-design set-up (paper flowchart: form the coefficient field, solve the
 * spectral problems on every coarse and coarse-coarse element, build the
 * preconditioner).  rho: element densities in [0,1] of dtype MSMG_F64 or
 * MSMG_F32 (copied; this copy defines the operator).  k_min > 0,
 * k_max >= k_min, p >= 1.  mask: nodal uint8, nonzero = fixed temperature
 * (must contain at least one node).  fixed_values: nodal FP64 temperatures
 * read on fixed nodes, or NULL for zero.  Call again whenever rho changes.
 * TPFA: mask holds one byte per cell, its Dirichlet faces (bit 0 the -x
 * face, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z); only faces on the domain boundary may
 * be flagged (MSMG_EINVAL otherwise) and at least one must be
 * (MSMG_ESINGULAR otherwise).  fixed_values: one FP64 temperature per cell,
 * imposed on every flagged face of that cell, or NULL for zero.  All device
 * pointers. */
int msmg_setup(msmg_handle* h, const void* rho, msmg_dtype rho_dtype, double k_min, double k_max, int p,
               const uint8_t* mask, const double* fixed_values, hipStream_t stream);

/* Solve A T = f by PCG (Polak-Ribiere beta) with the configured preconditioner.
 * f: nodal FP64 load (entries on fixed nodes are ignored).  T: nodal FP64 output;
 * when use_x0 != 0 its free entries are the initial guess.  Stops when the true
 * relative residual ||(f - A T)_F|| / ||b_F|| <= rtol (b = f minus the fixed-value
 * lift), or after maxit iterations.  info may be NULL (host pointer).
 * The iterate is kept in double-double precision: at high conductivity contrast
 * T reaches ~1/k_min and a binary64 T alone cannot reach residuals near 1e-8.
 * T_lo (nullable, nodal FP64 output): when given, T receives the high part and
 * T_lo the low part of the iterate (T + T_lo); when NULL, T = round(T + T_lo). */
int msmg_solve(msmg_handle* h, const double* f, double* T, double* T_lo, int use_x0, double rtol, int maxit,
               msmg_info* info, hipStream_t stream);

/* Adjoint solve of the sensitivity analysis (section 2.3, eq. adjoint): A_FF u_F = g_F
 * with zero fixed entries (u = lambda), whatever fixed values the set-up was given,
 * reusing the set-up of the last msmg_setup.  Arguments, outputs and return codes as
 * for msmg_solve (g: nodal FP64, entries on fixed nodes ignored; lambda: nodal FP64,
 * zero on fixed nodes; lambda_lo nullable). */
int msmg_solve_adjoint(msmg_handle* h, const double* g, double* lambda, double* lambda_lo, int use_x0, double rtol,
                       int maxit, msmg_info* info, hipStream_t stream);

/* The state solve and the adjoint solve of one set-up together (the paper's
 * LS1 and LS2 of section 4, sharing the set-up as in its tables; section 2.3,
 * eq. adjoint): A T = f with the set-up's fixed values (as msmg_solve from a
 * zero guess) and A_FF lambda = g with zero fixed entries (as
 * msmg_solve_adjoint), by two PCG recurrences advanced together.  Every
 * kernel that reads the operator's coefficients (the operator apply, the
 * smoothers, the fused residual and restriction, levels 1 and 2, the
 * prolongation) runs once for both right-hand sides, the two sides'
 * workgroups side by side on one XCD; scalars, stopping tests and residual
 * replacements stay per side, and a side that has stopped drops out.
 * f, g: nodal FP64 loads; T, lambda: nodal FP64 outputs; T_lo, lambda_lo:
 * nullable low parts as for msmg_solve; info_T, info_lambda: nullable host
 * reports (solve_ms is the pair's wall time).  Needs a handle created with
 * options.pair_rhs = 1 (MSMG_ESTATE otherwise).  Returns the first non-zero
 * outcome of the two solves, or an error < 0. */
int msmg_solve_pair(msmg_handle* h, const double* f, double* T, double* T_lo, const double* g, double* lambda,
                    double* lambda_lo, double rtol, int maxit, msmg_info* info_T, msmg_info* info_lambda,
                    hipStream_t stream);

/* Element sensitivities dc/drho_e = -p rho_e^(p-1) (k_max - k_min) lambda_e^T K0 T_e
 * (evaluated as -sum_{a<b} K0_ab (lambda_a - lambda_b)(T_a - T_b), exact for zero-row-sum K0)
 * (section 2.3 with a design-independent load).  lambda: nodal adjoint with zero
 * fixed entries, or NULL for the compliance case lambda = T (free entries of T;
 * valid for zero fixed values).  dc: element FP64 output.
 * TPFA: per cell, dc/drho_K = lambda^T (db/drho_K - dA/drho_K T) with the
 * harmonic faces' dT_F/dk_K = w_d 2 k_L^2 / (k_K + k_L)^2 and the Dirichlet
 * faces' 2 w_d k_K (diagonal and T_D lift, T_D from the set-up), times
 * dk/drho. */
int msmg_sensitivity(msmg_handle* h, const double* T, const double* lambda, double* dc, hipStream_t stream);

/* Element sensitivities of an objective with the design-dependent heat source of
 * section 2.1 eq. (material), f_e = f0 (1 - rho_e^p) (section 2.3):
 *   dc/drho_e = lambda^T (df/drho_e - dA/drho_e T)
 *             = -p rho_e^(p-1) [ (k_max - k_min) lambda_e^T K0 T_e + f0 (V/8) sum_{a in e} lambda_a ],
 * rho, p, k_min, k_max from the last msmg_setup.  T: nodal FP64 state including its
 * fixed values; lambda: nodal FP64 adjoint with zero fixed entries (required, the
 * source term makes the problem non-self-adjoint); dc: element FP64 output.  f0 = 0
 * gives msmg_sensitivity's value.  MSMG_EINVAL for NULL pointers or a non-finite
 * f0, MSMG_ESTATE before the first msmg_setup.  TPFA: msmg_sensitivity's cell
 * value plus lambda_K (-f0 p rho_K^(p-1)) |K|. */
int msmg_sensitivity_heat_source(msmg_handle* h, const double* T, const double* lambda, double f0, double* dc,
                                 hipStream_t stream);

/* Nodal load of the design-dependent heat source of section 2.1 eq. (material):
 * f_n = sum_{e ni n} f0 (1 - rho_e^p) V/8 with rho and p of the last msmg_setup
 * (TPFA: the cell integral f_K = f0 (1 - rho_K^p) |K|).
 * f: nodal FP64 output, written on every node (the solves ignore fixed entries).
 * MSMG_EINVAL for a NULL pointer or a non-finite f0, MSMG_ESTATE before the first
 * msmg_setup.  The mean-temperature objective of section 2.3 eq. (cost function),
 * (1/|Omega|) int T, has the weights msmg_element_load(src = NULL, 1/|Omega|). */
int msmg_heat_source_load(msmg_handle* h, double f0, double* f, hipStream_t stream);

/* y = P A P x + (I - P) x with P the projection on free nodes (FP64, nodal).
 * TPFA: y = A x over the cells (no unknown is fixed). */
int msmg_apply(msmg_handle* h, const double* x, double* y, hipStream_t stream);

/* z = M^-1 r: one preconditioner application (Algorithm 1 for the multigrid
 * kind).  Entries of r on fixed nodes are ignored; z is zero there.  With the
 * one-launch coarse levels (options.coarse_fused bit 0) the call waits for the
 * result and returns MSMG_ETIMEOUT if a barrier wait of that kernel gave up. */
int msmg_precondition(msmg_handle* h, const double* r, double* z, hipStream_t stream);

/* Consistent nodal load of an element-wise constant source: f_n = sum_{e ni n} s_e V/8,
 * with s_e = src[e], or s_e = src_const when src is NULL (TPFA: the cell
 * integral f_K = s_K |K|). */
int msmg_element_load(msmg_handle* h, const double* src, double src_const, double* f, hipStream_t stream);

/* Measurement aid: the memory traffic of the operator apply (msmg_apply reads
 * x on nn nodes and k on ne elements and writes y on nn nodes) without its
 * stencil.  Runs y = x (+ k on the first ne entries) reps times, coalesced,
 * one read or write per value, and returns the mean kernel time in *ms (host
 * pointer); 8 (2 nn + ne) bytes over that time is the bandwidth this access mix
 * reaches, the practical ceiling of the apply.  x, k, y: FP64 device arrays
 * (y must not alias x or k), nn and ne even, 2 <= ne <= nn.  Blocks until
 * done. */
int msmg_stream_ceiling(const double* x, const double* k, double* y, long long nn, long long ne, int reps, double* ms,
                        hipStream_t stream);

/* Measurement aid: the PCG's operator-apply kernel (q = A p with its step
 * reduction, the kernel of every PCG iteration) launched reps times back to
 * back on p = x after the last msmg_setup; *ms (host pointer) receives the
 * mean time per launch from HIP events around the batch, so per-launch
 * dispatch gaps are amortised rather than counted once each.  x: nodal FP64
 * device array (cells for TPFA), not zero on free entries.  Uses the
 * handle's PCG work vectors and scalars (do not overlap with a solve on the
 * handle).  Blocks until done. */
int msmg_time_apply(msmg_handle* h, const double* x, int reps, double* ms, hipStream_t stream);

/* Interpolation step between resolutions (section 3, interpolation technique):
 * Tc on the (nx,ny,nz) mesh -> Tf on the (2nx,2ny,2nz) mesh, the coarse trilinear
 * function evaluated at the fine nodes (no handle needed). */
int msmg_prolong_nodal(int nx, int ny, int nz, const double* Tc, double* Tf, hipStream_t stream);

/* Element injection (nx,ny,nz) -> (2nx,2ny,2nz) of an element field of dtype dt
 * (each child takes its parent's value). */
int msmg_prolong_element(int nx, int ny, int nz, const void* rc, void* rf, msmg_dtype dt, hipStream_t stream);

/* Density filter of the optimisation loop (a design-variable filter: the
 * paper's MMA loop of section 4 works on filtered densities; the weights are
 * the usual linear hat): w(e,f) = max(0, radius - |c_e - c_f|) with element
 * centres in element units, summed over elements inside the nx*ny*nz mesh.
 *   transpose = 0: out_e = sum_f w(e,f) in_f / W_e,  W_e = sum_f w(e,f)
 *   transpose != 0: out_f = sum_e w(e,f) in_e / W_e (its adjoint, for chain-rule
 *                   sensitivities)
 * in, out: element FP64 device arrays (caller-owned, must not alias).
 * radius in (1, 4]; MSMG_EINVAL otherwise. */
int msmg_density_filter(int nx, int ny, int nz, double radius, const double* in, double* out, int transpose,
                        hipStream_t stream);

/* Optimality-criteria design update (a stand-in for the MMA step of section
 * 2.3): x_new_e = clamp(x_e (-dc_e / (lambda dv_e))^eta, max(x_min, x_e - move),
 * min(1, x_e + move)) with the multiplier lambda > 0 found on the device so that
 * sum_e x_new_e = volume_fraction * elements.  x, dc, dv, x_new: element FP64
 * device arrays of the handle's mesh (dv > 0; x_new must not alias the inputs).
 * lambda: nullable device pointer receiving the multiplier.  Uses the handle's
 * reduction scratch (do not overlap with other calls on the handle). */
int msmg_oc_update(msmg_handle* h, const double* x, const double* dc, const double* dv, double volume_fraction,
                   double move, double eta, double x_min, double* x_new, double* lambda, hipStream_t stream);

/* Method of moving asymptotes (MMA; Svanberg 1987), the optimiser of the
 * paper's section 2.3, for one volume constraint f1(x) = dv . x / N - vf <= 0
 * and x_min <= x <= 1 on the handle's N elements: update number iter (0-based)
 * moves the asymptotes by the signs of the last two steps (the first two
 * updates place them at x -/+ 0.5 (1 - x_min)), builds the separable convex
 * approximation of the objective (gradient df0) and the constraint, limits the
 * step to max(x_min, L + 0.1 (x - L), x - move (1 - x_min)) ..
 * min(1, U - 0.1 (U - x), x + move (1 - x_min)), and solves the approximate
 * problem (elastic variable with c = 1000, d = 1) through its dual, the
 * multiplier found on the device.  x, xold1, xold2 (the designs of the two
 * previous updates; any values for iter < 2), df0, dv, x_new: element FP64
 * device arrays; low, upp: element FP64 in/out (the previous asymptotes in,
 * this update's out); lambda: nullable device pointer receiving the
 * multiplier.  Uses the handle's reduction scratch. */
int msmg_mma_update(msmg_handle* h, int iter, const double* x, const double* xold1, const double* xold2, double* low,
                    double* upp, const double* df0, const double* dv, double volume_fraction, double move,
                    double x_min, double* x_new, double* lambda, hipStream_t stream);

/* msmg_oc_update without a handle and without any allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc).  Same update, same kernels and the
 * same result as msmg_oc_update on an nx*ny*nz design; x, dc, dv, x_new:
 * element FP64 device arrays (x_new must not alias the inputs), lambda
 * nullable.  The scratch (block partials of the volume sweeps, a counter and
 * the multiplier bracket, about 66 KB) is a fixed array that each device holds
 * from the first call until the process ends; its size does not depend on the
 * design.  Designs above 2^40 elements are rejected with MSMG_EINVAL.  Every
 * call on one device uses that device's array, so calls that overlap on one
 * device (other streams, other threads) race; serialise them.  The counter is
 * cleared by a kernel at the start of every call (no memset). */
int msmg_oc_update_noalloc(int nx, int ny, int nz, const double* x, const double* dc, const double* dv,
                           double volume_fraction, double move, double eta, double x_min, double* x_new,
                           double* lambda, hipStream_t stream);

/* Objective values of the optimisation loop (section 2.3: the compliance
 * c = f^T T, the mean temperature of eq. cost function c = w^T T): *out = a^T b
 * over n <= the handle's unknowns, summed in a fixed order (bitwise
 * reproducible).  a, b: FP64 device arrays; out: one FP64 device value.  Uses
 * the handle's reduction scratch (do not overlap with other calls on the
 * handle). */
int msmg_dot(msmg_handle* h, const double* a, const double* b, long long n, double* out, hipStream_t stream);

/* Chain-rule scaling of a gradient (section 2.3): y = c * s * x over n entries,
 * with s = *s_dev read on the device (an upstream gradient; s_dev NULL: s = 1).
 * x, y: FP64 device arrays (y may alias x). */
int msmg_scale(const double* x, long long n, double c, const double* s_dev, double* y, hipStream_t stream);

/* Diagnostics of the last set-up, copied to host memory (blocking):
 *   what = 0: level-1 eigenvalues, ncells*Lc doubles (padded entries 0)
 *   what = 1: R_c in FP64, nodes*Lc doubles, node-major
 *   what = 2: A_c blocks, ncells*27*Lc*Lc doubles
 *   what = 3: coarse-coarse eigenvalues, ncc*Lcc doubles
 *   what = 4: A_cc, n_cc*n_cc doubles
 *   what = 5: per-cell level-1 status, ncells ints (outer iterations; < 0 = not converged)
 * `bytes` is the capacity of `host_out`.  Returns MSMG_EINVAL if too small. */
int msmg_export(msmg_handle* h, int what, void* host_out, size_t bytes);

/* Release the handle and its device memory (NULL is ignored). */
void msmg_destroy(msmg_handle* h);

/* Message of the last error on the calling thread ("" if none). */
const char* msmg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MSMG_H */
