// Problem state: host maps, device views into the caller's workspace, and
// the V-cycle / CG drivers.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "../../include/gmg.h"
#include "dispatch.hpp"
#include "host/esttables.hpp"
#include "host/maps.hpp"

namespace gmg {

struct DevLevel {
  LevelView v;
  int64_t off = 0;     // offset in the concatenated level vectors
  int64_t n_S = 0, n_I = 0;
  const int32_t* ilist = nullptr;
  double lam = 1.0;    // lambda_max estimate of D^{-1} A^S
};

// Work memory of one V-cycle: level vectors x, g, t, d (concatenated over
// levels, mg precision), operator slots of the level passes, restricted
// parent-cell values of the fine families of one level.
struct VWork {
  void *lx = nullptr, *lg = nullptr, *lt = nullptr, *ld = nullptr;
  double* E = nullptr;
  char* rbuf = nullptr;
};

// state of an asynchronous CG solve
struct CgState {
  bool running = false, pending = false, timed = false;
  int it = 0;            // iterations done
  int status = 0;
  double nb = 0.0;       // ||b||
  double* u = nullptr;
  hipStream_t stream = nullptr;
  std::vector<double> hist;
};

struct Problem {
  gmg_options opt{};
  std::shared_ptr<const Maps> maps;   // shared by clones (read-only after creation)
  const KernelTable* kt = nullptr;
  MatsH<float> m32{};
  MatsH<double> m64{};

  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t ws_need = 0;     // workspace bytes, fixed at creation
  bool bound = false;
  int device = -1;

  std::vector<DevLevel> lv;
  LeafView leaf;
  int64_t n_total = 0;   // sum of level DoFs
  int64_t n_dir = 0;
  const int32_t* copy = nullptr;
  void *lx = nullptr, *lg = nullptr, *lt = nullptr, *ld = nullptr, *ldinv = nullptr;
  double *cx = nullptr, *cr = nullptr, *cz = nullptr, *cp = nullptr, *cq = nullptr, *cb = nullptr;
  double* E = nullptr;     // slots of the two-pass operators (used as float or double)
  char* rbuf = nullptr;    // restricted parent-cell values of fine families (mg precision)
  double *scal = nullptr, *part = nullptr;
  double* ainv = nullptr;
  const int32_t* cidx = nullptr;
  int n0 = 0;
  double* eig = nullptr;   // 5 FP64 vectors of the largest level
  int64_t max_level_dofs = 0;
  int64_t e_levels = 0;    // operator slots the level passes need (E holds at least these)
  int64_t fam_max = 0;     // largest family count of a level >= 1
  double* host = nullptr;  // pinned scalars
  hipGraphExec_t graph = nullptr;
  hipStream_t graph_stream = nullptr;
  double timing[3] = {0, 0, 0};
  CgState cg;
  std::vector<hipEvent_t> ev;
  // error estimator: face tables (built on first use) and the workspace
  // they were last uploaded to
  std::shared_ptr<const EstTables> est;
  mutable const char* est_uploaded = nullptr;

  ~Problem();
};

size_t plan_workspace(Problem& P, char* base);
void bind_problem(Problem& P, void* ws, size_t bytes, hipStream_t s);
// E: the operator slots to use (null: the problem's own, in its workspace)
void apply_leaf(Problem& P, const double* x, double* y, bool mass, hipStream_t s, double* E = nullptr);
// doubles of operator slots the leaf operator needs
int64_t leaf_slots(const Problem& P);
void vcycle(Problem& P, const double* r, double* z, hipStream_t s);
// V-cycle with its work memory in the library's fixed device scratch array
// (no allocation); GMG_E_INVAL when the problem needs more than it holds
void vcycle_noalloc(Problem& P, const double* r, double* z, hipStream_t s);
// one V-cycle for each problem of a batch (same dimension, degree, precision,
// smoother), the level sweeps of all of them batched; d_table (device,
// 256-byte aligned, table_bytes) receives the launch tables, *need their
// size; with d_table null only *need is computed; h_stage: optional pinned
// host staging buffer of at least *need bytes; dot_rz: the partial sums of
// r.z into each problem's dot partials (CG)
void vcycle_batch(const std::vector<Problem*>& ps, const double* const* r, double* const* z, char* d_table,
                  size_t table_bytes, size_t* need, char* h_stage, hipStream_t s, bool dot_rz,
                  hipEvent_t staged = nullptr);
int solve(Problem& P, const double* b, double* u, int32_t* iters, double* hist, hipStream_t s);
void cg_start(Problem& P, const double* b, double* u, hipStream_t s, bool timed);
bool cg_poll(Problem& P, bool block);
// the state machine split for callers that enqueue the preconditioner
// themselves (batched): cg_check returns 0 (busy), 1 (finished) or 2 (next
// iteration due); cg_enqueue_tail enqueues the iteration after z = B r
int cg_check(Problem& P, bool block);
void cg_enqueue_tail(Problem& P, hipStream_t s);
void cg_enqueue_iteration(Problem& P);  // preconditioner and tail on the CG stream
// residual error estimator and marking (Sec. 4.3), device work memory in a
// caller-owned workspace of est_workspace_bytes(P) bytes
size_t est_workspace_bytes(Problem& P);
void estimate(Problem& P, const double* u, const double* f, char* ws, size_t bytes, double* eta, hipStream_t s);
void mark(Problem& P, const double* eta, double fraction, uint8_t* flags, char* ws, size_t bytes, hipStream_t s);
// marking kernels (mark.hip): flags of the m largest of eta[0..n) (ties in
// index order) through a stable descending key sort
size_t mark_temp_bytes(int64_t n);
void mark_top(const double* eta, int64_t n, int64_t m, double* keys_out, int32_t* idx_in, int32_t* idx_out,
              void* temp, size_t temp_bytes, uint8_t* flags, hipStream_t s);
// The next CG iteration of every problem of ps (each with its iteration due,
// cg_check having returned 2), each step one launch over all of them on s:
// the batched V-cycle z = B r, then the rest of the iteration; each
// problem's iteration event is recorded on s.  Tables as vcycle_batch.
void cg_iteration_batch(const std::vector<Problem*>& ps, char* d_table, size_t table_bytes, size_t* need,
                        char* h_stage, hipStream_t s, hipEvent_t staged = nullptr);
void set_constant(double* p, int64_t n, double v, hipStream_t s);
void apply_level_hook(Problem& P, int level, int variant, const void* x, void* y, hipStream_t s);

}  // namespace gmg

struct gmg_problem_s {
  gmg::Problem P;
};
