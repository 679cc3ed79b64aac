// Set-up driver: orders the coarse-space construction for one density field
// (paper flowchart: coefficient field -> spectral problems on the coarse
// cells -> spectral problems on the coarse-coarse cells -> preconditioner),
// and the launch-shape tuner of the batched per-cell eigensolver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "setup.h"

namespace msmg {

int launch_galerkin(const Ctx& c, const void* R, int b_dt, int drop_cc, double* out, hipStream_t s);
void launch_block_inverse(const Ctx& c, double* Ac, double* Dinv, hipStream_t s);
int run_cc_eigen(const Ctx& c, const SetupArgs& sa, SetupScratch* sc, const double* G, int* n_unconv, SetupReport* rep,
                 hipStream_t s);
int build_acc(const Ctx& c, const SetupArgs& sa, double* u, hipStream_t s);
void launch_convert(const void* in, int din, void* out, int dout, long long n, hipStream_t s);

int setup_scratch_alloc(const Geo& g, const Hier& h, int max_cc_dofs, int n_cc, const msmg_options& o, SetupScratch* s,
                        const std::function<int(void**, size_t)>& alloc) {
  (void)g;
  int m = o.cc_block ? o.cc_block : std::min(32, h.Lcc + 15);
  if (m < h.Lcc + 1) m = std::min(32, h.Lcc + 1);
  s->mcc = m;
  const size_t nvec = (size_t)m * h.ncells * h.Lc;
  int r;
  if ((r = alloc((void**)&s->Y, nvec * 8))) return r;
  if ((r = alloc((void**)&s->Yp, nvec * 8))) return r;
  if ((r = alloc((void**)&s->Z, nvec * 8))) return r;
  if ((r = alloc((void**)&s->small, (size_t)h.ncc * 4 * m * m * 8))) return r;
  if ((r = alloc((void**)&s->ccpar, (size_t)h.ncc * (8 + m + 1) * 8))) return r;
  if ((r = alloc((void**)&s->ccflag, (size_t)h.ncc * 2 * 4))) return r;  // convergence flags, Cholesky failures
  if (!o.lean_memory && (r = alloc((void**)&s->acc_copy, (size_t)n_cc * n_cc * 8))) return r;
  const size_t ndm = (size_t)std::max(max_cc_dofs, 1);
  s->cc_group = (int)std::max<size_t>(1, std::min<size_t>(h.ncc, CC_GROUP_BYTES / (ndm * ndm * 8)));
  if (o.cc_group > 0) s->cc_group = std::min(s->cc_group, o.cc_group);
  const size_t gj_single = gj_workspace_doubles(n_cc, 1);
  const size_t gj_batch = gj_workspace_doubles(int(ndm), s->cc_group);
  if ((r = alloc((void**)&s->gj, std::max(gj_single, gj_batch) * 8))) return r;
  if ((r = alloc((void**)&s->Gd, (size_t)s->cc_group * ndm * ndm * 8))) return r;
  if ((r = alloc((void**)&s->gpart, (size_t)s->cc_group * CC_GRAM_SLICES * m * m * 8))) return r;
  if ((r = alloc((void**)&s->work, 64))) return r;
  if ((r = alloc((void**)&s->cells, (size_t)h.ncells * 4))) return r;
  s->n_regular = -1;
  return MSMG_OK;
}

static int hip_ok(hipError_t e, SetupReport* rep, const char* what) {
  if (e == hipSuccess) return MSMG_OK;
  std::snprintf(rep->msg, sizeof(rep->msg), "%s: %s", what, hipGetErrorString(e));
  return MSMG_EHIP;
}

// ---- tuner cache ----------------------------------------------------------
static std::string tune_key(const Ctx& c, int nl) {
  hipDeviceProp_t p;
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipGetDeviceProperties(&p, dev);
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s H%d L%d nl%d rho%d cells%d%s", p.gcnArchName, c.h.H, c.h.Lc, nl, c.rho_dt,
                c.h.ncells, c.tpfa ? " tpfa" : "");
  return buf;
}

static bool cache_lookup(const char* path, const std::string& key, TuneChoice* t) {
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof(line), f)) {
    char* bar = std::strchr(line, '|');
    if (!bar) continue;
    *bar = 0;
    if (key == line) {
      TuneChoice c{};
      if (std::sscanf(bar + 1, "%d %d %d %d %lf", &c.bs, &c.m, &c.degree, &c.blocks_per_cu, &c.ms) == 5) {
        c.valid = 1;
        *t = c;
        found = true;
      }
    }
  }
  std::fclose(f);
  return found;
}

static void cache_store(const char* path, const std::string& key, const TuneChoice& t) {
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s|%d %d %d %d %.4f\n", key.c_str(), t.bs, t.m, t.degree, t.blocks_per_cu, t.ms);
  std::fclose(f);
}

static int count_unconverged(const SetupArgs& sa, int ncells, int* unconv, int* ties, hipStream_t s) {
  std::vector<int> st(ncells);
  if (hipMemcpyAsync(st.data(), sa.cell_status, sizeof(int) * ncells, hipMemcpyDeviceToHost, s) != hipSuccess) return MSMG_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return MSMG_EHIP;
  int u = 0, t = 0;
  for (int v : st) {
    u += (v >> 28) & 1;
    t += (v >> 29) & 1;
  }
  *unconv = u;
  *ties = t;
  return MSMG_OK;
}

// Time the level-1 eigensolver over a few launch shapes on the first cells of
// one class (cells[first .. first + count), LDS for nl nodes) and keep the
// fastest one with the fewest unconverged cells.  Two workgroups per CU are
// tried where their LDS fits (regular cells of H = 8: 512 nodes, 76 KB).
static int tune_local(const Ctx& c, const SetupArgs& sa, SetupScratch* sc, int cus, int first, int count, int nl,
                      hipStream_t s, TuneChoice* best) {
  struct Cand { int bs, m, degree, bpc; };
  std::vector<Cand> cands = {{256, 8, 12, 1}, {512, 8, 12, 1}, {768, 8, 8, 1}, {768, 8, 12, 1},
                             {768, 8, 20, 1}, {1024, 8, 12, 1}, {256, 8, 12, 2}, {512, 8, 12, 2},
                             {512, 8, 8, 2}, {512, 8, 20, 2}};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MSMG_EHIP;
  best->valid = 0;
  int best_unconv = 1 << 30;
  // candidates are timed on the first cells only (a few rounds of workgroups)
  const int lim = std::min(count, 64 * cus);
  for (const Cand& cd : cands) {
    if (cd.m < c.h.Lc + 1) continue;
    if (cd.bpc > 1 && size_t(cd.bpc) * local_lds_bytes(cd.m, nl) > 160 * 1024) continue;
    const int blocks = std::max(1, std::min(lim, cd.bpc * cus));
    (void)hipEventRecord(e0, s);
    const int r = launch_local_eigen(c, sa, sc, cd.bs, cd.m, cd.degree, blocks, s, first, lim, nl);
    (void)hipEventRecord(e1, s);
    if (r != MSMG_OK) continue;
    if (hipEventSynchronize(e1) != hipSuccess) return MSMG_EHIP;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    int un = 0, ti = 0;
    if (count_unconverged(sa, c.h.ncells, &un, &ti, s) != MSMG_OK) return MSMG_EHIP;
    const bool better = (un < best_unconv) || (un == best_unconv && ms < best->ms);
    if (!best->valid || better) {
      best->valid = 1;
      best->bs = cd.bs;
      best->m = cd.m;
      best->degree = cd.degree;
      best->blocks_per_cu = cd.bpc;
      best->ms = ms;
      best_unconv = un;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best->valid ? MSMG_OK : MSMG_ESETUP;
}

// The level-1 cells in two shape classes: the regular cells (H nodes along
// every axis) first, then the cells that keep a remainder, with their count.
static int build_cell_classes(const Hier& h, const Geo& g, SetupScratch* sc, hipStream_t s) {
  std::vector<int> reg, rest;
  reg.reserve(h.ncells);
  for (int cz = 0; cz < h.ncz; ++cz)
    for (int cy = 0; cy < h.ncy; ++cy)
      for (int cx = 0; cx < h.ncx; ++cx) {
        const int cell = (cz * h.ncy + cy) * h.ncx + cx;
        const bool regular = cell_end(cx, h.H, h.ncx, g.nnx) - cell_begin(cx, h.H) == h.H &&
                             cell_end(cy, h.H, h.ncy, g.nny) - cell_begin(cy, h.H) == h.H &&
                             cell_end(cz, h.H, h.ncz, g.nnz) - cell_begin(cz, h.H) == h.H;
        (regular ? reg : rest).push_back(cell);
      }
  const int n0 = int(reg.size());
  reg.insert(reg.end(), rest.begin(), rest.end());
  if (hipMemcpyAsync(sc->cells, reg.data(), sizeof(int) * reg.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    return MSMG_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return MSMG_EHIP;
  sc->n_regular = n0;
  return MSMG_OK;
}

int timed_gj_inverse(const SetupArgs& sa, SetupReport* rep, int n, int batch, double* A, double* work, hipStream_t s) {
  if (sa.ev && hipEventRecord(sa.ev[5], s) != hipSuccess) return MSMG_EHIP;
  const int r = gj_inverse(n, batch, A, work, s);
  if (r != MSMG_OK || !sa.ev) return r;
  float ms = 0.f;
  if (hipEventRecord(sa.ev[6], s) != hipSuccess || hipEventSynchronize(sa.ev[6]) != hipSuccess ||
      hipEventElapsedTime(&ms, sa.ev[5], sa.ev[6]) != hipSuccess)
    return MSMG_EHIP;
  rep->dense_ms += ms;
  rep->dense_gflop += double(batch) * double(n) * double(n) * double(n) * 1e-9;
  return MSMG_OK;
}

int run_setup(const Ctx& c, const SetupArgs& sa, SetupScratch* sc, SetupReport* rep, hipStream_t s) {
  std::memset(rep, 0, sizeof(*rep));
  // phase boundaries for the timing mode: 0 start, 1 after the local problems,
  // 2 after A_c, 3 after the coarse-coarse problems, 4 after A_cc^-1
  auto mark = [&](int k) {
    if (sa.ev) (void)hipEventRecord(sa.ev[k], s);
  };
  mark(0);
  const Hier& h = c.h;
  const msmg_options& o = *sa.opt;
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);

  // 1. local spectral problems eq. (spepb) -> R_c (FP64), one launch per cell
  // shape class, each with its own tuned shape and LDS size
  int r;
  if (sc->n_regular < 0 && (r = build_cell_classes(h, c.g, sc, s))) return hip_ok(hipGetLastError(), rep, "cell classes");
  const int nclass[2] = {sc->n_regular, h.ncells - sc->n_regular};
  const int first[2] = {0, sc->n_regular};
  const int nlc[2] = {h.H * h.H * h.H, sa.max_cell_nodes};
  for (int k = 0; k < 2; ++k) {
    if (nclass[k] == 0) continue;
    TuneChoice& tc = sa.tune[k];
    if (o.eig_block > 0 || o.eig_degree > 0 || !o.autotune) {
      tc.valid = 1;
      tc.bs = nlc[k] <= 256 ? 256 : 768;
      tc.blocks_per_cu = 1;
      tc.m = o.eig_block > 0 ? o.eig_block : 8;
      tc.degree = o.eig_degree > 0 ? o.eig_degree : 12;
    } else if (!tc.valid) {
      const std::string key = tune_key(c, nlc[k]);
      if (!cache_lookup(o.tune_cache, key, &tc)) {
        r = tune_local(c, sa, sc, cus, first[k], nclass[k], nlc[k], s, &tc);
        if (r != MSMG_OK) {
          std::snprintf(rep->msg, sizeof(rep->msg), "level-1 eigensolver tuning failed");
          return r;
        }
        cache_store(o.tune_cache, key, tc);
      }
    }
    const int blocks = std::max(1, std::min(nclass[k], tc.blocks_per_cu * cus));
    r = launch_local_eigen(c, sa, sc, tc.bs, tc.m, tc.degree, blocks, s, first[k], nclass[k], nlc[k]);
    if (r != MSMG_OK) {
      std::snprintf(rep->msg, sizeof(rep->msg), "level-1 eigensolver launch failed (block %d)", tc.m);
      return r;
    }
  }
  if ((r = count_unconverged(sa, h.ncells, &rep->eig_unconverged, &rep->eig_ties, s))) return r;

  mark(1);
  // 2. stored copy of R_c, Galerkin A_c from the stored values
  const long long nb = c.g.nn * h.Lc;
  if (sa.Rcs != (void*)sa.Rc64) launch_convert(sa.Rc64, DT_F64, sa.Rcs, sa.b_dt, nb, s);
  auto galerkin = [&](const void* R, int bdt, int drop_cc, double* out) {
    return c.tpfa ? launch_tpfa_galerkin(c, R, bdt, drop_cc, out, s) : launch_galerkin(c, R, bdt, drop_cc, out, s);
  };
  if ((r = galerkin(sa.Rcs, sa.b_dt, 0, sa.Ac64))) return hip_ok(hipGetLastError(), rep, "Galerkin A_c");
  launch_block_inverse(c, sa.Ac64, sa.AcDinv64, s);
  const long long nblk = (long long)h.ncells * 27 * h.Lc * h.Lc;
  if (sa.a_dt != DT_F64) {
    launch_convert(sa.Ac64, DT_F64, sa.Acv, sa.a_dt, nblk, s);
    launch_convert(sa.AcDinv64, DT_F64, sa.AcDinvv, sa.a_dt, (long long)sa.n_c * h.Lc, s);
  }

  mark(2);
  // 3. coarse-coarse spectral problems eq. (spectral cc) on the FP64 basis
  if ((r = galerkin(sa.Rc64, DT_F64, 1, sa.G64))) return hip_ok(hipGetLastError(), rep, "Galerkin G");
  if ((r = run_cc_eigen(c, sa, sc, sa.G64, &rep->cc_unconverged, rep, s))) {
    std::snprintf(rep->msg, sizeof(rep->msg), "coarse-coarse eigensolver failed");
    return r;
  }
  if (sa.Rccv != sa.Rcc64) launch_convert(sa.Rcc64, DT_F64, sa.Rccv, DT_F32, (long long)h.Lcc * sa.n_c, s);

  mark(3);
  // 4. A_cc = R_cc A_c R_cc^T from the cycle's copies, then its inverse
  if ((r = build_acc(c, sa, sc->Y, s))) return hip_ok(hipGetLastError(), rep, "A_cc");
  const size_t nn2 = (size_t)sa.n_cc * sa.n_cc * 8;
  if (sc->acc_copy &&
      (r = hip_ok(hipMemcpyAsync(sc->acc_copy, sa.Acc, nn2, hipMemcpyDeviceToDevice, s), rep, "A_cc copy")))
    return r;
  if ((r = timed_gj_inverse(sa, rep, sa.n_cc, 1, sa.Acc, sc->gj, s))) return hip_ok(hipGetLastError(), rep, "A_cc inverse");
  mark(4);
  return hip_ok(hipGetLastError(), rep, "set-up");
}

}  // namespace msmg
