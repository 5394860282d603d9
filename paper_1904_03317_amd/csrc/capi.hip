// extern "C" boundary of the library (declared in include/gmg.h).  Every
// entry point catches C++ exceptions and turns them into status codes plus a
// thread-local message.
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>

#include "../../include/gmg.h"
#include "host/forest.hpp"
#include "host/maps.hpp"
#include "problem.hpp"

struct gmg_mesh_s {
  std::unique_ptr<gmg::Forest> f;
};

namespace gmg {
namespace {
thread_local std::string g_last_error;
}
void set_last_error(const std::string& m) { g_last_error = m; }
}  // namespace gmg

namespace {

template <typename F>
int guard(F&& f) {
  try {
    return f();
  } catch (const gmg::Error& e) {
    gmg::set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    gmg::set_last_error("host allocation failed");
    return GMG_E_NOMEM_HOST;
  } catch (const std::exception& e) {
    gmg::set_last_error(e.what());
    return GMG_E_INVAL;
  } catch (...) {
    gmg::set_last_error("unknown error");
    return GMG_E_INVAL;
  }
}

#define REQUIRE(c, msg) \
  if (!(c)) gmg::fail(GMG_E_INVAL, msg)

}  // namespace

extern "C" {

void gmg_options_default(gmg_options* o) {
  if (!o) return;
  o->degree = 2;
  o->mg_precision = 32;
  o->cheb_degree = 4;
  o->cheb_lo = 0.08;
  o->cheb_hi = 1.2;
  o->eig_iters = 10;
  o->rtol = 1e-10;
  o->max_iter = 100;
  o->use_graph = 1;
  o->op_variant = 0;
  o->smoother = GMG_SMOOTHER_CHEBYSHEV;
  o->relax = 1.0;
}

const char* gmg_last_error(void) { return gmg::g_last_error.c_str(); }

int gmg_mesh_create(int dim, int n_coarse, const int32_t* origins, gmg_mesh* out) {
  return guard([&] {
    REQUIRE(out && origins, "null argument");
    auto m = std::make_unique<gmg_mesh_s>();
    m->f = std::make_unique<gmg::Forest>(dim, n_coarse, origins);
    *out = m.release();
    return 0;
  });
}

int gmg_mesh_refine(gmg_mesh m, const uint8_t* flags, int64_t* n_after) {
  return guard([&] {
    REQUIRE(m && flags, "null argument");
    int64_t n = m->f->refine(flags);
    if (n_after) *n_after = n;
    return 0;
  });
}

int gmg_mesh_num_leaves(gmg_mesh m, int64_t* n) {
  return guard([&] {
    REQUIRE(m && n, "null argument");
    *n = (int64_t)m->f->leaves().size();
    return 0;
  });
}

int gmg_mesh_dim(gmg_mesh m, int* dim) {
  return guard([&] {
    REQUIRE(m && dim, "null argument");
    *dim = m->f->dim();
    return 0;
  });
}

int gmg_mesh_leaves(gmg_mesh m, int8_t* level, int64_t* anchor) {
  return guard([&] {
    REQUIRE(m, "null argument");
    const auto& L = m->f->leaves();
    const int d = m->f->dim();
    for (size_t i = 0; i < L.size(); ++i) {
      if (level) level[i] = L[i].c.level;
      if (anchor)
        for (int a = 0; a < d; ++a) anchor[i * d + a] = L[i].c.a[a];
    }
    return 0;
  });
}

int gmg_mesh_destroy(gmg_mesh m) {
  delete m;
  return 0;
}

int gmg_problem_create(gmg_mesh m, const gmg_options* opts, const double* coeff, gmg_problem* out) {
  return guard([&] {
    REQUIRE(m && opts && out, "null argument");
    REQUIRE(opts->degree >= 1 && opts->degree <= 4, "degree must be 1..4");
    REQUIRE(opts->mg_precision == 32 || opts->mg_precision == 64, "mg_precision must be 32 or 64");
    REQUIRE(opts->cheb_degree >= 1 && opts->cheb_degree <= 64, "cheb_degree must be 1..64");
    REQUIRE(opts->cheb_lo > 0 && opts->cheb_hi > opts->cheb_lo, "0 < cheb_lo < cheb_hi required");
    REQUIRE(opts->eig_iters >= 1 && opts->eig_iters <= 100, "eig_iters must be 1..100");
    REQUIRE(opts->rtol > 0 && opts->max_iter >= 1, "rtol > 0 and max_iter >= 1 required");
    REQUIRE(m->f->max_level() < 24, "too many levels");
    REQUIRE(opts->op_variant == 0, "op_variant must be 0");
    REQUIRE(opts->smoother == GMG_SMOOTHER_CHEBYSHEV || opts->smoother == GMG_SMOOTHER_JACOBI, "unknown smoother");
    REQUIRE(opts->relax > 0 && opts->relax <= 2, "0 < relax <= 2 required");
    auto p = std::make_unique<gmg_problem_s>();
    gmg::Problem& P = p->P;
    P.opt = *opts;
    P.kt = gmg::kernel_table(m->f->dim(), opts->degree);
    REQUIRE(P.kt, "no kernels for this dimension/degree");
    P.maps = std::make_shared<const gmg::Maps>(gmg::build_maps(*m->f, opts->degree, coeff));
    const gmg::FE1D& fe = P.maps->fe;
    for (int i = 0; i < 25; ++i) {
      P.m64.M[i] = fe.M[i];
      P.m64.K[i] = fe.K[i];
      P.m32.M[i] = (float)fe.M[i];
      P.m32.K[i] = (float)fe.K[i];
    }
    for (int i = 0; i < 45; ++i) {
      P.m64.E[i] = fe.E[i];
      P.m32.E[i] = (float)fe.E[i];
    }
    P.ws_need = gmg::plan_workspace(P, nullptr);
    *out = p.release();
    return 0;
  });
}

int gmg_problem_clone(gmg_problem src, const gmg_options* opts, gmg_problem* out) {
  return guard([&] {
    REQUIRE(src && opts && out, "null argument");
    REQUIRE(opts->degree == src->P.maps->k, "clone must keep the degree");
    REQUIRE(opts->mg_precision == 32 || opts->mg_precision == 64, "mg_precision must be 32 or 64");
    REQUIRE(opts->cheb_degree >= 1 && opts->cheb_degree <= 64, "cheb_degree must be 1..64");
    REQUIRE(opts->cheb_lo > 0 && opts->cheb_hi > opts->cheb_lo, "0 < cheb_lo < cheb_hi required");
    REQUIRE(opts->eig_iters >= 1 && opts->eig_iters <= 100, "eig_iters must be 1..100");
    REQUIRE(opts->rtol > 0 && opts->max_iter >= 1, "rtol > 0 and max_iter >= 1 required");
    REQUIRE(opts->smoother == GMG_SMOOTHER_CHEBYSHEV || opts->smoother == GMG_SMOOTHER_JACOBI, "unknown smoother");
    REQUIRE(opts->relax > 0 && opts->relax <= 2, "0 < relax <= 2 required");
    auto p = std::make_unique<gmg_problem_s>();
    gmg::Problem& P = p->P;
    P.opt = *opts;
    P.kt = src->P.kt;
    P.maps = src->P.maps;
    P.m32 = src->P.m32;
    P.m64 = src->P.m64;
    P.ws_need = gmg::plan_workspace(P, nullptr);
    *out = p.release();
    return 0;
  });
}

int gmg_problem_info(gmg_problem p, gmg_info* o) {
  return guard([&] {
    REQUIRE(p && o, "null argument");
    const gmg::Maps& M = *p->P.maps;
    std::memset(o, 0, sizeof(*o));
    o->dim = M.dim;
    o->degree = M.k;
    o->n_levels = (int32_t)M.levels.size();
    o->mg_precision = p->P.opt.mg_precision;
    o->n_dofs = M.n_dofs;
    o->n_hanging = M.n_hanging;
    o->n_leaves = M.n_leaves;
    int64_t nf = 0;
    for (auto d : M.dirichlet) nf += d == 0;
    o->n_free = nf;
    for (size_t l = 0; l < M.levels.size() && l < 24; ++l) {
      o->level_dofs[l] = M.levels[l].n_dofs;
      o->level_cells[l] = M.levels[l].n_cells;
      o->lambda_max[l] = l < p->P.lv.size() ? p->P.lv[l].lam : 0.0;
    }
    o->workspace_bytes = p->P.ws_need;
    return 0;
  });
}

int gmg_problem_array(gmg_problem p, int which, int level, const void** ptr, int64_t* count) {
  return guard([&] {
    REQUIRE(p && ptr && count, "null argument");
    const gmg::Maps& M = *p->P.maps;
    auto lev = [&]() -> const gmg::LevelData& {
      REQUIRE(level >= 0 && level < (int)M.levels.size(), "level out of range");
      return M.levels[level];
    };
    switch (which) {
      case GMG_ARR_LEAF_CELLMAP: *ptr = M.leaf_cellmap.data(); *count = (int64_t)M.leaf_cellmap.size(); break;
      case GMG_ARR_LEAF_DIRICHLET: *ptr = M.dirichlet.data(); *count = (int64_t)M.dirichlet.size(); break;
      case GMG_ARR_CON_OFFSETS: *ptr = M.con_off.data(); *count = (int64_t)M.con_off.size(); break;
      case GMG_ARR_CON_MASTERS: *ptr = M.con_mas.data(); *count = (int64_t)M.con_mas.size(); break;
      case GMG_ARR_CON_WEIGHTS: *ptr = M.con_w.data(); *count = (int64_t)M.con_w.size(); break;
      case GMG_ARR_COPY_LEVEL: *ptr = M.copy_level.data(); *count = (int64_t)M.copy_level.size(); break;
      case GMG_ARR_COPY_INDEX: *ptr = M.copy_index.data(); *count = (int64_t)M.copy_index.size(); break;
      case GMG_ARR_LEVEL_CELLMAP: *ptr = lev().cellmap.data(); *count = (int64_t)lev().cellmap.size(); break;
      case GMG_ARR_LEVEL_FLAGS: *ptr = lev().flags.data(); *count = (int64_t)lev().flags.size(); break;
      case GMG_ARR_LEVEL_PARENT: *ptr = lev().parent.data(); *count = (int64_t)lev().parent.size(); break;
      case GMG_ARR_LEAF_CELLMAP_PARENT:
        *ptr = M.leaf_cellmap_parent.data();
        *count = (int64_t)M.leaf_cellmap_parent.size();
        break;
      case GMG_ARR_LEAF_MASK: *ptr = M.leaf_mask.data(); *count = (int64_t)M.leaf_mask.size(); break;
      case GMG_ARR_LEVEL_PERM:
        lev();
        *ptr = M.layouts[level].perm.data();
        *count = (int64_t)M.layouts[level].perm.size();
        break;
      default: gmg::fail(GMG_E_INVAL, "unknown array");
    }
    return 0;
  });
}

int gmg_problem_workspace_bytes(gmg_problem p, size_t* bytes) {
  return guard([&] {
    REQUIRE(p && bytes, "null argument");
    *bytes = p->P.ws_need;
    return 0;
  });
}

int gmg_problem_bind(gmg_problem p, void* ws, size_t bytes, hipStream_t s) {
  return guard([&] {
    REQUIRE(p && ws, "null argument");
    gmg::bind_problem(p->P, ws, bytes, s);
    return 0;
  });
}

int gmg_problem_destroy(gmg_problem p) {
  delete p;
  return 0;
}

int gmg_rhs(gmg_problem p, const double* f, double* b, hipStream_t s) {
  return guard([&] {
    REQUIRE(p && f && b, "null argument");
    REQUIRE(p->P.bound, "problem not bound");
    gmg::apply_leaf(p->P, f, b, true, s);
    return 0;
  });
}

int gmg_solve_rhs(gmg_problem p, const double* b, double* u, int32_t* iters, double* hist, hipStream_t s) {
  return guard([&] {
    REQUIRE(p && b && u && iters, "null argument");
    return gmg::solve(p->P, b, u, iters, hist, s);
  });
}

int gmg_solve(gmg_problem p, const double* f, double* u, int32_t* iters, double* hist, hipStream_t s) {
  return guard([&] {
    REQUIRE(p && u && iters, "null argument");
    gmg::Problem& P = p->P;
    REQUIRE(P.bound, "problem not bound");
    const double* src = f;
    if (!f) {
      gmg::set_constant(P.cx, P.maps->n_dofs, 1.0, s);
      src = P.cx;
    }
    gmg::apply_leaf(P, src, P.cb, true, s);
    return gmg::solve(P, P.cb, u, iters, hist, s);
  });
}

int gmg_apply_leaf(gmg_problem p, const double* x, double* y, hipStream_t s) {
  return guard([&] {
    REQUIRE(p && x && y, "null argument");
    REQUIRE(p->P.bound, "problem not bound");
    gmg::apply_leaf(p->P, x, y, false, s);
    return 0;
  });
}

int gmg_apply_level(gmg_problem p, int level, int variant, const void* x, void* y, hipStream_t s) {
  return guard([&] {
    REQUIRE(p && x && y, "null argument");
    REQUIRE(variant >= 0 && variant <= 2, "variant must be 0, 1 or 2");
    gmg::apply_level_hook(p->P, level, variant, x, y, s);
    return 0;
  });
}

int gmg_vcycle(gmg_problem p, const double* r, double* z, hipStream_t s) {
  return guard([&] {
    REQUIRE(p && r && z, "null argument");
    gmg::vcycle(p->P, r, z, s);
    return 0;
  });
}

int gmg_vcycle_batch(const gmg_problem* ps, int n, const double* const* r, double* const* z, void* table,
                     size_t* table_bytes, hipStream_t s) {
  return guard([&] {
    REQUIRE(ps && n >= 1 && table_bytes, "null argument");
    std::vector<gmg::Problem*> pv(n);
    for (int i = 0; i < n; ++i) {
      REQUIRE(ps[i], "null problem");
      pv[i] = &ps[i]->P;
    }
    if (table) {
      REQUIRE(r && z, "null argument");
      for (int i = 0; i < n; ++i) REQUIRE(r[i] && z[i], "null vector");
    }
    size_t need = 0;
    gmg::vcycle_batch(pv, r, z, (char*)table, *table_bytes, &need, nullptr, s, false);
    *table_bytes = need;
    if (table) {
      hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) gmg::fail(GMG_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    }
    return 0;
  });
}

int gmg_estimator_workspace_bytes(gmg_problem p, size_t* bytes) {
  return guard([&] {
    REQUIRE(p && bytes, "null argument");
    *bytes = gmg::est_workspace_bytes(p->P);
    return 0;
  });
}

int gmg_estimate(gmg_problem p, const double* u, const double* f, void* ws, size_t bytes, double* eta,
                 hipStream_t s) {
  return guard([&] {
    REQUIRE(p && u && f && eta, "null argument");
    gmg::estimate(p->P, u, f, (char*)ws, bytes, eta, s);
    return 0;
  });
}

int gmg_mark(gmg_problem p, const double* eta, double fraction, uint8_t* flags, void* ws, size_t bytes,
             hipStream_t s) {
  return guard([&] {
    REQUIRE(p && eta && flags, "null argument");
    gmg::mark(p->P, eta, fraction, flags, (char*)ws, bytes, s);
    return 0;
  });
}

int gmg_vcycle_noalloc(gmg_problem p, const double* r, double* z, hipStream_t s) {
  return guard([&] {
    REQUIRE(p && r && z, "null argument");
    gmg::vcycle_noalloc(p->P, r, z, s);
    return 0;
  });
}

int gmg_problem_last_timing(gmg_problem p, double* out3) {
  return guard([&] {
    REQUIRE(p && out3, "null argument");
    for (int i = 0; i < 3; ++i) out3[i] = p->P.timing[i];
    return 0;
  });
}

}  // extern "C"
