// Set-up of the coarse spaces (paper section 3): per-cell spectral problems
// eq. (spepb), Galerkin coarse operators, coarse-coarse spectral problems
// eq. (spectral cc), the coarse-coarse operator and its inverse.
#pragma once

#include <functional>

#include "../../include/msmg.h"
#include "internal.h"

namespace msmg {

// Pivot block of the batched symmetric Gauss-Jordan (sweep) inverse and its
// workspace: per matrix the inverted pivot block (GJ_NB^2) and the pivot row
// panel (GJ_NB x n).
constexpr int GJ_NB = 128;  // pivot columns per sweep step (64-deep halves per tile)
inline size_t gj_workspace_doubles(int n, int batch) {
  return (size_t)batch * ((size_t)GJ_NB * GJ_NB + (size_t)GJ_NB * n);
}
// Device memory for the dense shifted coarse-coarse matrices: the cc cells are
// solved in groups whose matrices fit in this many bytes.
constexpr size_t CC_GROUP_BYTES = size_t(24) << 30;
constexpr int CC_GRAM_SLICES = 8;  // workgroups per cc cell of the Gram products
int gj_inverse(int n, int batch, double* A, double* work, hipStream_t s);

// Launch shape of the level-1 eigensolver chosen by the tuner.
struct TuneChoice {
  int valid;
  int bs;       // threads per block
  int m;        // subspace block size
  int degree;   // filter degree
  int blocks_per_cu;
  double ms;    // measured time of the tuned launch
};

struct SetupScratch {
  // coarse-coarse subspace iteration, vectors laid out per cc cell as [m][nd_J]
  double* Y = nullptr;   // current block
  double* Yp = nullptr;  // previous block (filter recurrence)
  double* Z = nullptr;   // operator image / next block
  double* small = nullptr;  // per cc cell: 3 matrices of mcc x mcc
  double* gpart = nullptr;  // per cc cell of a group: CC_GRAM_SLICES partial Gram matrices
  double* ccpar = nullptr;  // per cc cell filter parameters
  int* ccflag = nullptr;    // per cc cell: converged iteration or -1; then per cc cell: Cholesky failed
  double* acc_copy = nullptr;  // A_cc before inversion (diagnostics)
  double* gj = nullptr;        // Gauss-Jordan panels (batched)
  double* Gd = nullptr;        // dense shifted coarse-coarse matrices, then their inverses
  unsigned* work = nullptr;    // work-queue counter
  int* cells = nullptr;        // level-1 cells by shape class: the regular (H^3-node) cells, then the rest
  int n_regular = -1;          // regular cells in `cells` (-1: list not built yet)
  int mcc = 0;
  int cc_group = 0;            // cc cells whose dense shifted matrices are held at once
};

struct SetupArgs {
  double lam_bound;
  double* Rc64;
  void* Rcs;
  int b_dt;
  double* Ac64;
  void* Acv;
  double* AcDinv64;
  void* AcDinvv;
  int a_dt;
  double* G64;
  double* Rcc64;
  void* Rccv;
  double* Acc;
  double* evals;
  int* cell_status;
  double* cc_evals;
  int* cc_status;
  int n_c, n_cc;
  int max_cell_nodes;
  int max_cc_dofs;
  const int* cc_ptr;
  const int* h_cc_ptr;
  const int* cc_dofs;
  const int* dof_cc;
  const int* dof_loc;
  const msmg_options* opt;
  int warm;  // level-1 solver starts from the basis left in Rc64 by the previous set-up
  TuneChoice* tune;  // per level-1 cell class: [0] regular cells, [1] the rest
  // timing (null: none): SETUP_EVENTS events; the phase boundaries are
  // recorded in ev[0 .. 4], ev[5], ev[6] bracket each dense inversion
  hipEvent_t* ev;
};
constexpr int SETUP_EVENTS = 7;

struct SetupReport {
  int eig_unconverged;
  int cc_unconverged;
  int eig_ties;
  double dense_ms;     // with timing: the dense Gauss-Jordan inversions
  double dense_gflop;  // and their flop count (n^3 per n x n sweep inverse)
  char msg[256];
};
// time one dense batched inversion (n x n, batch of them) into rep when the
// set-up is timed
int timed_gj_inverse(const SetupArgs& sa, SetupReport* rep, int n, int batch, double* A, double* work, hipStream_t s);

int setup_scratch_alloc(const Geo& g, const Hier& h, int max_cc_dofs, int n_cc, const msmg_options& o, SetupScratch* s,
                        const std::function<int(void**, size_t)>& alloc);

int run_setup(const Ctx& c, const SetupArgs& a, SetupScratch* s, SetupReport* rep, hipStream_t st);

// level-1 eigensolver launch over cells[first .. first + count) of the class
// list, with LDS for cells of up to nl nodes (used by the tuner and the set-up)
int launch_local_eigen(const Ctx& c, const SetupArgs& a, SetupScratch* s, int bs, int m, int degree,
                       int blocks, hipStream_t st, int first, int count, int nl);
size_t local_lds_bytes(int M, int nl);

// utilities implemented with the fine kernels
void launch_fill(const Ctx& c, double* x, double v, hipStream_t s);
void launch_copy(const Ctx& c, const double* a, double* b, hipStream_t s);
void launch_zero_free(const Ctx& c, double* x, hipStream_t s);
void launch_sc_reset(const Ctx& c, int full, int maxit, hipStream_t s);
int count_fixed(const Ctx& c, int* nfixed, hipStream_t s);

}  // namespace msmg
