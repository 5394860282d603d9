// Device setup, V-cycle with local smoothing (Alg. 2, Sec. 2.3) and
// FP64 preconditioned CG (Sec. 1, 4.1) on one GPU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>

#define GMG_SOLVER_TU
#include "famkernels.hpp"
#include "kernels.hpp"
#include "problem.hpp"

namespace gmg {

#define HIPCHECK(x)                                                                  \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) fail(GMG_E_HIP, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------- table registry
namespace {
const KernelTable* g_tables[2][5] = {};
}
void register_table(int dim, int k, const KernelTable* t) { g_tables[dim - 2][k] = t; }
const KernelTable* kernel_table(int dim, int k) {
  if (dim < 2 || dim > 3 || k < 1 || k > 4) return nullptr;
  return g_tables[dim - 2][k];
}

Problem::~Problem() {
  if (graph) (void)hipGraphExecDestroy(graph);
  for (auto e : ev) (void)hipEventDestroy(e);
  if (host) (void)hipHostFree(host);
}

static unsigned grid1(int64_t n) {
  int64_t g = (n + dev::kBlock - 1) / dev::kBlock;
  return (unsigned)std::max<int64_t>(1, g);
}
// grid of the kernels fused with a dot product (one partial per block)
static unsigned fuse_grid(int64_t n) {
  const int64_t per = (int64_t)dev::kBlock * dev::kFuseNPT;
  return (unsigned)std::max<int64_t>(1, (n + per - 1) / per);
}
static unsigned p2_grid(int64_t n) {
  const int64_t per = (int64_t)dev::kBlock * dev::kP2NPT;
  return (unsigned)std::max<int64_t>(1, (n + per - 1) / per);
}
static unsigned dot_grid(int64_t n) {
  return (unsigned)std::min<int64_t>(dev::kDotBlocks, std::max<int64_t>(1, (n + dev::kBlock - 1) / dev::kBlock));
}

template <typename T>
static void fill_dev(T* p, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = (unsigned)std::min<int64_t>(4096, grid1(n));
  hipLaunchKernelGGL(dev::fill<T>, dim3(g), dim3(dev::kBlock), 0, s, n, p, v);
}

void set_constant(double* p, int64_t n, double v, hipStream_t s) { fill_dev(p, n, v, s); }

template <typename T>
static const LevelOps<T>& ops(Problem& P);
template <>
const LevelOps<float>& ops<float>(Problem& P) { return P.kt->f32; }
template <>
const LevelOps<double>& ops<double>(Problem& P) { return P.kt->f64; }
template <typename T>
static const MatsH<T>& mats(Problem& P);
template <>
const MatsH<float>& mats<float>(Problem& P) { return P.m32; }
template <>
const MatsH<double>& mats<double>(Problem& P) { return P.m64; }

// y = A_l x on every row of level l (device layout of the level)
template <typename T>
static void level_apply(Problem& P, int l, const T* x, T* y, hipStream_t s) {
  DevLevel& V = P.lv[l];
  const int64_t n = V.v.n_dofs;
  const LevelOps<T>& op = ops<T>(P);
  T* E = (T*)P.E;
  if (l == 0) {
    op.cell_e(V.v, x, E, mats<T>(P), s);
    hipLaunchKernelGGL(dev::seg_plain<T>, dim3(grid1(n)), dim3(dev::kBlock), 0, s, n, V.v.soff, (const T*)E, y);
  } else {
    dev::Epi<T> ep;
    ep.y = y;
    op.op(V.v, dev::kEpiPlain, x, ep, E, mats<T>(P), s);
    op.sum(V.v, dev::kEpiPlain, E, ep, s);
  }
}

// diagonal of A_l (FP64, device layout)
static void level_diag(Problem& P, int l, double* diag, hipStream_t s) {
  DevLevel& V = P.lv[l];
  if (l == 0) {
    fill_dev(diag, V.v.n_dofs, 0.0, s);
    P.kt->diag0(V.v, diag, P.m64, s);
  } else {
    dev::Epi<double> ep;
    ep.y = diag;
    P.kt->f64.op(V.v, dev::kEpiDiag, nullptr, ep, P.E, P.m64, s);
    P.kt->f64.sum(V.v, dev::kEpiDiag, P.E, ep, s);
  }
}

// ---------------------------------------------------------------- workspace
namespace {
struct Planner {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T) + 1;
    return p;
  }
};
}  // namespace

size_t plan_workspace(Problem& P, char* base) {
  const Maps& M = *P.maps;
  Planner pl{base};
  const size_t esz = P.opt.mg_precision == 32 ? 4 : 8;
  const int L = (int)M.levels.size() - 1;
  P.lv.assign(L + 1, DevLevel{});
  int64_t off = 0;
  int64_t e_max = 0;
  P.max_level_dofs = 0;
  const int nj = M.dim == 3 ? 27 : 9, cpf = 1 << M.dim;
  for (int l = 0; l <= L; ++l) {
    const LevelData& D = M.levels[l];
    DevLevel& V = P.lv[l];
    V.v.n_cells = D.n_cells;
    V.v.n_dofs = D.n_dofs;
    V.v.n_fam = D.n_fam;
    V.off = off;
    off += D.n_dofs;
    V.n_I = (int64_t)D.ilist.size();
    V.n_S = 0;
    for (auto f : D.flags) V.n_S += f == kFlagS;
    P.max_level_dofs = std::max(P.max_level_dofs, D.n_dofs);
    bool uniform = true;
    for (auto c : D.coeff) uniform = uniform && (c == D.coeff[0]);
    const double hd = M.dim == 3 ? std::ldexp(1.0, -l) : 1.0;
    if (uniform) {
      V.v.scale = nullptr;
      V.v.scale0 = (D.coeff.empty() ? 1.0 : D.coeff[0]) * hd;
    } else {
      V.v.scale = pl.take<double>(D.n_cells);
    }
    V.v.flags = pl.take<uint8_t>(D.n_dofs);
    V.ilist = pl.take<int32_t>(D.ilist.size());
    if (l == 0) {
      V.v.cmap = pl.take<int32_t>(size_t(D.n_cells) * M.npc);
      V.v.slot = pl.take<int32_t>(size_t(D.n_cells) * M.npc);
      V.v.soff = pl.take<int32_t>(D.n_dofs + 1);
      V.v.roff = L >= 1 ? pl.take<int32_t>(D.n_dofs + 1) : nullptr;
      e_max = std::max<int64_t>(e_max, D.n_cells * M.npc);
    } else {
      const LevelLayout& Y = M.layouts[l];
      for (int r = 0; r < 5; ++r) {
        V.v.sec[r] = Y.sec[r];
        V.v.shn[r] = Y.shn[r];
        V.v.entoff[r] = Y.entoff[r];
        V.v.eoff[r] = Y.eoff[r];
      }
      V.v.gbase = pl.take<int32_t>(size_t(D.n_fam) * nj);
      V.v.own = pl.take<uint32_t>(D.n_fam);
      V.v.excl = pl.take<uint32_t>(D.n_fam);
      V.v.pmask = pl.take<uint8_t>(Y.n_ent);
      V.v.parent = pl.take<int32_t>(D.n_fam);
      V.v.child = l < L ? pl.take<int32_t>(size_t(D.n_fam) * cpf) : nullptr;
      V.v.rslot = l == 1 ? pl.take<int32_t>(size_t(D.n_fam) * M.npc) : nullptr;
      e_max = std::max<int64_t>(e_max, Y.n_slots);
      if (l == 1) e_max = std::max<int64_t>(e_max, D.n_fam * M.npc);
    }
  }
  P.n_total = off;
  P.lx = pl.take<char>(size_t(off) * esz);
  P.lg = pl.take<char>(size_t(off) * esz);
  P.lt = pl.take<char>(size_t(off) * esz);
  P.ld = pl.take<char>(size_t(off) * esz);
  P.ldinv = pl.take<char>(size_t(off) * esz);
  const int64_t N = M.n_dofs;
  const LeafTiles& LT = M.tiles;
  const bool tiled = LT.n_tiles > 0;
  P.leaf = LeafView{};
  P.leaf.n_cells = M.n_leaves;
  P.leaf.n_dofs = N;
  P.leaf.mask = pl.take<uint16_t>(M.n_leaves);
  P.leaf.scale = pl.take<double>(M.n_leaves);
  P.leaf.mscale = pl.take<double>(M.n_leaves);
  P.leaf.dir = pl.take<uint8_t>(N);
  int64_t e_leaf = 0;
  if (tiled) {
    P.leaf.n_tiles = LT.n_tiles;
    P.leaf.n_slots = LT.n_slots();
    P.leaf.n_p2 = (int64_t)LT.p2_dof.size();
    P.leaf.max_nodes = LT.max_nodes;
    P.leaf.t_own = pl.take<int32_t>(LT.own.size());
    P.leaf.t_loff = pl.take<int64_t>(LT.list_off.size());
    P.leaf.t_list = pl.take<int32_t>(LT.list.size());
    P.leaf.lmap = pl.take<uint16_t>(LT.lmap.size());
    P.leaf.p2_dof = pl.take<int32_t>(LT.p2_dof.size());
    P.leaf.p2_off = pl.take<int32_t>(LT.p2_off.size());
    P.leaf.p2_slot = pl.take<int32_t>(LT.p2_slot.size());
    e_leaf = LT.n_slots();
  } else {
    P.leaf.cmap = pl.take<int32_t>(size_t(M.n_leaves) * M.npc);
    P.leaf.slot = pl.take<int32_t>(size_t(M.n_leaves) * M.npc);
    P.leaf.soff = pl.take<int32_t>(N + 1);
    e_leaf = M.n_leaves * M.npc;
  }
  P.n_dir = 0;
  for (auto d : M.dirichlet) P.n_dir += d;
  P.copy = pl.take<int32_t>(N);
  P.cx = pl.take<double>(N);
  P.cr = pl.take<double>(N);
  P.cz = pl.take<double>(N);
  P.cp = pl.take<double>(N);
  P.cq = pl.take<double>(N);
  P.cb = pl.take<double>(N);
  P.e_levels = e_max;
  e_max = std::max<int64_t>(e_max, e_leaf);
  if (e_max >= INT32_MAX) fail(GMG_E_INVAL, "operator slots exceed 2^31");
  P.E = pl.take<double>(e_max);
  // restricted parent-cell values of the fine families of one level
  int64_t fam_max = 0;
  for (int l = 1; l <= L; ++l) fam_max = std::max<int64_t>(fam_max, M.levels[l].n_fam);
  P.fam_max = fam_max;
  P.rbuf = pl.take<char>(size_t(fam_max) * M.npc * esz);
  P.scal = pl.take<double>(dev::kNumScalars + 8);
  // dot partials: the fixed dot grid, or one per block of the fused kernels
  {
    int64_t np = std::max<int64_t>(dev::kDotBlocks, (N + dev::kBlock - 1) / dev::kBlock);
    if (tiled) np = std::max<int64_t>(np, std::min<int64_t>(LT.n_tiles, dev::kLeafBlocks) + p2_grid(P.leaf.n_p2));
    P.part = pl.take<double>(np);
  }
  int n0 = 0;
  for (auto f : M.levels[0].flags) n0 += f == kFlagS;
  if (n0 > 6000) fail(GMG_E_INVAL, "coarse level too large for the dense coarse solve (> 6000 free nodes)");
  P.n0 = n0;
  P.ainv = pl.take<double>(size_t(n0) * n0);
  P.cidx = pl.take<int32_t>(n0);
  P.eig = pl.take<double>(size_t(P.max_level_dofs) * 6);
  return pl.off + 256;
}

// ---------------------------------------------------------------- setup
namespace {

template <typename T>
void h2d(const T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return;
  HIPCHECK(hipMemcpyAsync((void*)dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

template <typename T>
std::vector<T> soa(const std::vector<T>& a, int64_t rows, int cols) {
  std::vector<T> o(a.size());
  for (int64_t r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) o[size_t(c) * rows + r] = a[size_t(r) * cols + c];
  return o;
}

// Slots of the two-pass operator: every (cell, local node) gets one entry of
// a node-major buffer; the entries of a node are contiguous, in cell order.
void build_slots(const std::vector<int32_t>& cm, int64_t nc, int npc, int64_t nn, std::vector<int32_t>& off,
                 std::vector<int32_t>& slot_soa) {
  off.assign(nn + 1, 0);
  for (size_t i = 0; i < cm.size(); ++i) ++off[cm[i] + 1];
  for (int64_t i = 0; i < nn; ++i) off[i + 1] += off[i];
  std::vector<int32_t> pos(off.begin(), off.end() - 1);
  slot_soa.resize(cm.size());
  for (int64_t c = 0; c < nc; ++c)
    for (int j = 0; j < npc; ++j) slot_soa[size_t(j) * nc + c] = pos[cm[size_t(c) * npc + j]]++;
}

// largest eigenvalue of a symmetric tridiagonal matrix (bisection with
// Sturm counts)
double tridiag_max_eig(const std::vector<double>& d, const std::vector<double>& e) {
  const int m = (int)d.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  auto count_below = [&](double x) {
    int c = 0;
    double q = d[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < m; ++i) {
      if (q == 0.0) q = 1e-300;
      q = d[i] - x - e[i - 1] * e[i - 1] / q;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (count_below(mid) >= m)
      hi = mid;
    else
      lo = mid;
  }
  return hi;
}

double dot_host(Problem& P, const double* a, const double* b, int64_t n, hipStream_t s) {
  unsigned g = dot_grid(n);
  hipLaunchKernelGGL(dev::dot_partial, dim3(g), dim3(dev::kBlock), 0, s, n, a, b, P.part);
  hipLaunchKernelGGL(dev::cg_scalars, dim3(1), dim3(dev::kBlock), 0, s, (int)g, P.part, P.scal + dev::kNumScalars, 3);
  HIPCHECK(hipMemcpyAsync(P.host + 8, P.scal + dev::kNumScalars + dev::kBb, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  return P.host[8];
}

// lambda_max of D^{-1} A^S: Jacobi-PCG from (i mod 12) - 5.5 on S rows,
// largest Ritz value of the Lanczos matrix from the CG coefficients
// (Sec. 4.1 eigenvalue estimate)
double estimate_lambda(Problem& P, int l, hipStream_t s) {
  DevLevel& V = P.lv[l];
  const int64_t n = V.v.n_dofs;
  int iters = (int)std::min<int64_t>(P.opt.eig_iters, V.n_S);
  if (iters <= 0) return 1.0;
  double* dinv = P.eig;
  double* r = P.eig + n;
  double* z = P.eig + 2 * n;
  double* p = P.eig + 3 * n;
  double* q = P.eig + 4 * n;
  double* diag = P.eig + 5 * n;
  level_diag(P, l, diag, s);
  hipLaunchKernelGGL(dev::make_dinv<double>, dim3(grid1(n)), dim3(dev::kBlock), 0, s, n, diag, V.v.flags, dinv);
  {
    // start vector (i mod 12) - 5.5 on the S rows, i the level DoF id
    const LevelData& D = P.maps->levels[l];
    const std::vector<int32_t>& perm = P.maps->layouts[l].perm;
    std::vector<double> r0(n, 0.0);
    for (int64_t i = 0; i < n; ++i)
      if (D.flags[i] == kFlagS) r0[perm[i]] = double(i % 12) - 5.5;
    h2d(r, r0, s);
    HIPCHECK(hipStreamSynchronize(s));
  }
  hipLaunchKernelGGL(dev::eig_init, dim3(grid1(n)), dim3(dev::kBlock), 0, s, n, (const double*)dinv,
                     (const double*)r, z, p);
  double rho = dot_host(P, r, z, n, s);
  std::vector<double> alphas, betas;
  for (int j = 0; j < iters; ++j) {
    if (!(rho > 0.0)) break;
    level_apply<double>(P, l, p, q, s);
    double pq = dot_host(P, p, q, n, s);
    if (!(pq > 0.0)) break;
    double alpha = rho / pq;
    alphas.push_back(alpha);
    if (j == iters - 1) break;
    hipLaunchKernelGGL(dev::axpy_zr, dim3(grid1(n)), dim3(dev::kBlock), 0, s, n, alpha, q, r, dinv, z);
    double rho_new = dot_host(P, r, z, n, s);
    if (!(rho_new > 0.0)) break;
    double beta = rho_new / rho;
    betas.push_back(beta);
    hipLaunchKernelGGL(dev::xpby, dim3(grid1(n)), dim3(dev::kBlock), 0, s, n, z, beta, p);
    rho = rho_new;
  }
  const int m = (int)alphas.size();
  if (m == 0) return 1.0;
  std::vector<double> d(m), e(std::max(0, m - 1));
  for (int j = 0; j < m; ++j) {
    d[j] = 1.0 / alphas[j] + (j > 0 ? betas[j - 1] / alphas[j - 1] : 0.0);
    if (j + 1 < m) e[j] = std::sqrt(betas[j]) / alphas[j];
  }
  return tridiag_max_eig(d, e);
}

// dense FP64 inverse of A_0 restricted to the S nodes of level 0
std::vector<double> coarse_inverse(const Maps& M, std::vector<int32_t>& idx) {
  const LevelData& D = M.levels[0];
  const int n = M.n, npc = M.npc, dim = M.dim;
  std::vector<int32_t> pos(D.n_dofs, -1);
  idx.clear();
  for (int64_t i = 0; i < D.n_dofs; ++i)
    if (D.flags[i] == kFlagS) {
      pos[i] = (int32_t)idx.size();
      idx.push_back((int32_t)i);
    }
  const int n0 = (int)idx.size();
  std::vector<double> A(size_t(n0) * n0, 0.0);
  for (int64_t c = 0; c < D.n_cells; ++c) {
    const double a = D.coeff[c];  // h = 1 on level 0
    for (int i = 0; i < npc; ++i) {
      int pi = pos[D.cellmap[c * npc + i]];
      if (pi < 0) continue;
      int ix = i % n, iy = (i / n) % n, iz = i / (n * n);
      for (int j = 0; j < npc; ++j) {
        int pj = pos[D.cellmap[c * npc + j]];
        if (pj < 0) continue;
        int jx = j % n, jy = (j / n) % n, jz = j / (n * n);
        const double* Mm = M.fe.M;
        const double* Kk = M.fe.K;
        double v;
        if (dim == 3)
          v = Kk[ix * n + jx] * Mm[iy * n + jy] * Mm[iz * n + jz] + Mm[ix * n + jx] * Kk[iy * n + jy] * Mm[iz * n + jz] +
              Mm[ix * n + jx] * Mm[iy * n + jy] * Kk[iz * n + jz];
        else
          v = Kk[ix * n + jx] * Mm[iy * n + jy] + Mm[ix * n + jx] * Kk[iy * n + jy];
        A[size_t(pi) * n0 + pj] += a * v;
      }
    }
  }
  // Cholesky A = L L^T, then the inverse column by column
  std::vector<double> Lm(A);
  for (int j = 0; j < n0; ++j) {
    double s = Lm[size_t(j) * n0 + j];
    for (int k = 0; k < j; ++k) s -= Lm[size_t(j) * n0 + k] * Lm[size_t(j) * n0 + k];
    if (!(s > 0.0)) fail(GMG_E_BREAKDOWN, "coarse matrix not positive definite");
    double d = std::sqrt(s);
    Lm[size_t(j) * n0 + j] = d;
    for (int i = j + 1; i < n0; ++i) {
      double t = Lm[size_t(i) * n0 + j];
      for (int k = 0; k < j; ++k) t -= Lm[size_t(i) * n0 + k] * Lm[size_t(j) * n0 + k];
      Lm[size_t(i) * n0 + j] = t / d;
    }
  }
  std::vector<double> inv(size_t(n0) * n0, 0.0), y(n0);
  for (int c = 0; c < n0; ++c) {
    for (int i = 0; i < n0; ++i) {
      double t = i == c ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= Lm[size_t(i) * n0 + k] * y[k];
      y[i] = t / Lm[size_t(i) * n0 + i];
    }
    for (int i = n0 - 1; i >= 0; --i) {
      double t = y[i];
      for (int k = i + 1; k < n0; ++k) t -= Lm[size_t(k) * n0 + i] * inv[size_t(k) * n0 + c];
      inv[size_t(i) * n0 + c] = t / Lm[size_t(i) * n0 + i];
    }
  }
  return inv;
}

}  // namespace

void bind_problem(Problem& P, void* ws, size_t bytes, hipStream_t s) {
  const Maps& M = *P.maps;
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) fail(GMG_E_INVAL, "workspace must be 256-byte aligned");
  if (bytes < P.ws_need) fail(GMG_E_INVAL, "workspace too small");
  plan_workspace(P, (char*)ws);
  P.ws = (char*)ws;
  P.ws_bytes = bytes;
  HIPCHECK(hipGetDevice(&P.device));
  if (!P.host) HIPCHECK(hipHostMalloc((void**)&P.host, 64 * sizeof(double), hipHostMallocDefault));
  if (P.ev.empty()) {
    P.ev.resize(5);
    for (auto& e : P.ev) HIPCHECK(hipEventCreate(&e));
  }
  const int L = (int)M.levels.size() - 1;
  const bool f32 = P.opt.mg_precision == 32;
  const int nj = M.dim == 3 ? 27 : 9, cpf = 1 << M.dim;
  for (int l = 0; l <= L; ++l) {
    const LevelData& D = M.levels[l];
    DevLevel& V = P.lv[l];
    if (V.v.scale) {
      std::vector<double> sc(D.n_cells);
      double hd = M.dim == 3 ? std::ldexp(1.0, -l) : 1.0;
      for (int64_t c = 0; c < D.n_cells; ++c) sc[c] = D.coeff[c] * hd;
      h2d(V.v.scale, sc, s);
    }
    if (l == 0) {
      h2d(V.v.cmap, soa(D.cellmap, D.n_cells, M.npc), s);
      std::vector<int32_t> off, sl;
      build_slots(D.cellmap, D.n_cells, M.npc, D.n_dofs, off, sl);
      h2d(V.v.slot, sl, s);
      h2d(V.v.soff, off, s);
      h2d(V.v.flags, D.flags, s);
      h2d(V.ilist, D.ilist, s);
      HIPCHECK(hipStreamSynchronize(s));
      continue;
    }
    // entity layout: flags and I-node list in device numbering
    const LevelLayout& Y = M.layouts[l];
    {
      std::vector<uint8_t> fl(D.n_dofs);
      for (int64_t i = 0; i < D.n_dofs; ++i) fl[Y.perm[i]] = D.flags[i];
      std::vector<int32_t> il(D.ilist.size());
      for (size_t i = 0; i < il.size(); ++i) il[i] = Y.perm[D.ilist[i]];
      h2d(V.v.flags, fl, s);
      h2d(V.ilist, il, s);
      h2d(V.v.gbase, soa(Y.gbase, D.n_fam, nj), s);
      h2d(V.v.own, Y.own, s);
      h2d(V.v.excl, Y.excl, s);
      h2d(V.v.pmask, Y.pmask, s);
      h2d(V.v.parent, D.parent, s);
      if (V.v.child) h2d(V.v.child, soa(Y.child, D.n_fam, cpf), s);
      HIPCHECK(hipStreamSynchronize(s));
    }
    if (l == 1) {
      // restriction into level 0: (family, parent node) -> level-0 node-major slots
      const LevelData& Pl = M.levels[0];
      std::vector<int32_t> pm(size_t(D.n_fam) * M.npc);
      for (int64_t f = 0; f < D.n_fam; ++f)
        for (int j = 0; j < M.npc; ++j) pm[size_t(f) * M.npc + j] = Pl.cellmap[size_t(D.parent[f]) * M.npc + j];
      std::vector<int32_t> off, sl;
      build_slots(pm, D.n_fam, M.npc, Pl.n_dofs, off, sl);
      h2d(V.v.rslot, sl, s);
      h2d(P.lv[0].v.roff, off, s);
      HIPCHECK(hipStreamSynchronize(s));
    }
  }
  {
    // 3D at degree >= 3: leaf cells with in-cell constraints first, each
    // group in leaf order, so that the cells without constraints go to the
    // cooperative kernel, which has no constraint step.  Otherwise leaf
    // order throughout (measured faster at degree 2: the constrained cells
    // spread over the whole mesh, and a wave of them gathers from far apart)
    // and n_con = n_cells.
    const bool split = M.dim == 3 && M.k >= 3;
    std::vector<int64_t> ord;
    ord.reserve(M.n_leaves);
    for (int64_t c = 0; c < M.n_leaves; ++c)
      if (!split || (M.leaf_mask[c] >> 3)) ord.push_back(c);
    P.leaf.n_con = (int64_t)ord.size();
    for (int64_t c = 0; c < M.n_leaves; ++c)
      if (split && !(M.leaf_mask[c] >> 3)) ord.push_back(c);
    // the tiled operator keeps leaf order (its tiles are runs of it) and
    // needs no cell map
    std::vector<int32_t> cm(P.leaf.n_tiles ? 0 : M.leaf_cellmap_parent.size());
    std::vector<uint16_t> mk(M.n_leaves);
    for (int64_t c = 0; c < M.n_leaves; ++c) {
      mk[c] = M.leaf_mask[ord[c]];
      if (!P.leaf.n_tiles)
        for (int j = 0; j < M.npc; ++j)
          cm[size_t(c) * M.npc + j] = M.leaf_cellmap_parent[size_t(ord[c]) * M.npc + j];
    }
    h2d(P.leaf.mask, mk, s);
    h2d(P.leaf.dir, M.dirichlet, s);
    if (P.leaf.n_tiles) {
      const LeafTiles& LT = M.tiles;
      h2d(P.leaf.t_own, LT.own, s);
      h2d(P.leaf.t_loff, LT.list_off, s);
      h2d(P.leaf.t_list, LT.list, s);
      h2d(P.leaf.lmap, soa(LT.lmap, M.n_leaves, M.npc), s);
      h2d(P.leaf.p2_dof, LT.p2_dof, s);
      h2d(P.leaf.p2_off, LT.p2_off, s);
      h2d(P.leaf.p2_slot, LT.p2_slot, s);
      HIPCHECK(hipStreamSynchronize(s));
    } else {
      h2d(P.leaf.cmap, soa(cm, M.n_leaves, M.npc), s);
      std::vector<int32_t> off, sl;
      build_slots(cm, M.n_leaves, M.npc, M.n_dofs, off, sl);
      h2d(P.leaf.slot, sl, s);
      h2d(P.leaf.soff, off, s);
      HIPCHECK(hipStreamSynchronize(s));
    }
    std::vector<double> sc(M.n_leaves), ms(M.n_leaves);
    for (int64_t c = 0; c < M.n_leaves; ++c) {
      double h = std::ldexp(1.0, -M.leaf_level[ord[c]]);
      sc[c] = M.leaf_coeff[ord[c]] * (M.dim == 3 ? h : 1.0);
      ms[c] = M.dim == 3 ? h * h * h : h * h;
    }
    h2d(P.leaf.scale, sc, s);
    h2d(P.leaf.mscale, ms, s);
    std::vector<int32_t> cp(M.n_dofs);
    for (int64_t i = 0; i < M.n_dofs; ++i) {
      const int l = M.copy_level[i];
      const int32_t li = l >= 1 ? M.layouts[l].perm[M.copy_index[i]] : M.copy_index[i];
      int64_t g = P.lv[l].off + li;
      if (g > INT32_MAX) fail(GMG_E_INVAL, "level vectors exceed 2^31 entries");
      cp[i] = (int32_t)g;
    }
    h2d(P.copy, cp, s);
    HIPCHECK(hipStreamSynchronize(s));
  }
  std::vector<int32_t> cidx;
  std::vector<double> inv = coarse_inverse(M, cidx);
  h2d(P.ainv, inv, s);
  h2d(P.cidx, cidx, s);
  // level vectors start at zero: t is kept zero between operator uses
  const size_t esz = f32 ? 4 : 8;
  HIPCHECK(hipMemsetAsync(P.lx, 0, P.n_total * esz, s));
  HIPCHECK(hipMemsetAsync(P.lt, 0, P.n_total * esz, s));
  HIPCHECK(hipMemsetAsync(P.ld, 0, P.n_total * esz, s));
  HIPCHECK(hipMemsetAsync(P.lg, 0, P.n_total * esz, s));
  // Jacobi diagonals and eigenvalue estimates
  for (int l = 0; l <= L; ++l) {
    DevLevel& V = P.lv[l];
    const int64_t n = V.v.n_dofs;
    double* diag = P.eig + 5 * n;
    level_diag(P, l, diag, s);
    if (f32)
      hipLaunchKernelGGL(dev::make_dinv<float>, dim3(grid1(n)), dim3(dev::kBlock), 0, s, n, diag, V.v.flags,
                         (float*)P.ldinv + V.off);
    else
      hipLaunchKernelGGL(dev::make_dinv<double>, dim3(grid1(n)), dim3(dev::kBlock), 0, s, n, diag, V.v.flags,
                         (double*)P.ldinv + V.off);
    V.lam = l >= 1 && P.opt.smoother == GMG_SMOOTHER_CHEBYSHEV ? estimate_lambda(P, l, s) : 1.0;
  }
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(s));
  if (P.graph) {
    (void)hipGraphExecDestroy(P.graph);
    P.graph = nullptr;
  }
  P.bound = true;
}

// ---------------------------------------------------------------- operators
// leaf operator q = C^T A C p with Dirichlet rows zero (or the mass matrix):
// hanging-node constraints applied inside the cells (pass 1), per-DoF sums
// (pass 2)
// leaf operator with the partial sums of x.y (part non-null, not with mass):
// returns the number of partials written to part
static int leaf_op(Problem& P, const double* x, double* y, bool mass, double* part, hipStream_t s, double* E) {
  const int64_t N = P.maps->n_dofs;
  if (!E) E = P.E;
  if (P.leaf.n_tiles) {
    const unsigned g1 = P.kt->leaf_t(P.leaf, x, y, E, part, mass, P.m64, s);
    const int64_t n2 = P.leaf.n_p2;
    if (n2 == 0 && part) {
      fill_dev(part + g1, 1, 0.0, s);
      return (int)g1 + 1;
    }
    if (n2 == 0) return (int)g1;
    const unsigned g2 = p2_grid(n2);
    if (part)
      hipLaunchKernelGGL(dev::leaf_pass2<true>, dim3(g2), dim3(dev::kBlock), 0, s, P.leaf, (const double*)E, x, y,
                         part + g1);
    else
      hipLaunchKernelGGL(dev::leaf_pass2<false>, dim3(g2), dim3(dev::kBlock), 0, s, P.leaf, (const double*)E, x, y,
                         (double*)nullptr);
    return (int)(g1 + g2);
  }
  P.kt->leaf_e(P.leaf, x, E, mass, P.m64, s);
  if (part) {
    hipLaunchKernelGGL(dev::seg_dir_dot, dim3(fuse_grid(N)), dim3(dev::kBlock), 0, s, N, P.leaf.soff,
                       (const double*)E, P.leaf.dir, y, x, part);
    return (int)fuse_grid(N);
  }
  hipLaunchKernelGGL(dev::seg_dir, dim3(grid1(N)), dim3(dev::kBlock), 0, s, N, P.leaf.soff, (const double*)E,
                     P.leaf.dir, y);
  return 0;
}

void apply_leaf(Problem& P, const double* x, double* y, bool mass, hipStream_t s, double* E) {
  leaf_op(P, x, y, mass, nullptr, s, E);
}

int64_t leaf_slots(const Problem& P) {
  return P.leaf.n_tiles ? P.maps->tiles.n_slots() : P.maps->n_leaves * P.maps->npc;
}


struct Cheb {
  double theta, delta, sigma;
};
static Cheb cheb_of(const Problem& P, int l) {
  const double a = P.opt.cheb_lo * P.lv[l].lam, b = P.opt.cheb_hi * P.lv[l].lam;
  Cheb c;
  c.theta = 0.5 * (b + a);
  c.delta = 0.5 * (b - a);
  c.sigma = c.theta / c.delta;
  return c;
}

// Coefficients of smoothing step j (1-based) on level l, a step being
// d = c1 d + c2 D^{-1} (g - A x), x += d.  Chebyshev (Sec. 4.1): the
// three-term semi-iteration on D^{-1} A^S over [lo, hi] lambda_max; Jacobi
// (Sec. 4.3): c1 = 0, c2 = relax.
struct StepCoef {
  double c1, c2;
};
static StepCoef step_coef(const Problem& P, int l, int j) {
  if (P.opt.smoother == GMG_SMOOTHER_JACOBI) return {0.0, P.opt.relax};
  const Cheb c = cheb_of(P, l);
  double rho_old = 1.0 / c.sigma, c1 = 0.0, c2 = 1.0 / c.theta;
  for (int i = 2; i <= j; ++i) {
    const double rho = 1.0 / (2.0 * c.sigma - rho_old);
    c1 = rho * rho_old;
    c2 = 2.0 * rho / c.delta;
    rho_old = rho;
  }
  return {c1, c2};
}

// Smoothing steps first..m on level l >= 1 (Sec. 4.1 / 4.3 smoother on
// D^{-1} A^S), each an operator application whose two passes perform the
// vector update as their epilogue.  Pre-smoothing enters with step 1
// already done (from x = 0, no operator needed); post-smoothing starts at
// step 1 from the prolongated x, whose interface values stay fixed
// (D^{-1} = 0 there) so that every residual includes A^{SI} x^I.
template <typename T>
static void smooth_steps(Problem& P, const VWork& W, int l, int first, hipStream_t s) {
  DevLevel& V = P.lv[l];
  const int64_t o = V.off;
  T* E = (T*)W.E;
  dev::Epi<T> ep;
  ep.x = (T*)W.lx + o;
  ep.d = (T*)W.ld + o;
  ep.g = (T*)W.lg + o;
  ep.dinv = (const T*)P.ldinv + o;
  ep.flags = V.v.flags;
  const LevelOps<T>& op = ops<T>(P);
  for (int j = first; j <= P.opt.cheb_degree; ++j) {
    const StepCoef c = step_coef(P, l, j);
    ep.c1 = T(c.c1);
    ep.c2 = T(c.c2);
    op.op(V.v, dev::kEpiCheb, ep.x, ep, E, mats<T>(P), s);
    op.sum(V.v, dev::kEpiCheb, E, ep, s);
  }
}

// One V-cycle with local smoothing (Alg. 2 in the storage-efficient form of
// Sec. 2.3): leaf residual entries enter the hierarchy on the coarsest level
// holding them as S nodes; smoothing acts on V^S only; the residual on S and
// I rows is restricted; after prolongation the interface values enter the
// post-smoothing residuals through A^{SI}.
template <typename T>
static void vcycle_t(Problem& P, const VWork& Wk, const double* r, double* z, hipStream_t s, bool dot_rz) {
  const Maps& M = *P.maps;
  const int L = (int)P.lv.size() - 1;
  const int64_t N = M.n_dofs;
  T *X = (T*)Wk.lx, *G = (T*)Wk.lg, *R = (T*)Wk.lt, *Dd = (T*)Wk.ld, *Di = (T*)P.ldinv;
  T* E = (T*)Wk.E;
  const LevelOps<T>& op = ops<T>(P);
  fill_dev(G, P.n_total, T(0), s);
  hipLaunchKernelGGL(dev::copy_to_levels<T>, dim3(grid1(N)), dim3(dev::kBlock), 0, s, N, P.copy, r, G);
  if (L >= 1) {
    // first pre-smoothing step on the finest level: x = D^{-1} g / theta
    DevLevel& V = P.lv[L];
    hipLaunchKernelGGL(dev::cheb_step<T>, dim3(grid1(V.v.n_dofs)), dim3(dev::kBlock), 0, s, V.v.n_dofs, X + V.off,
                       Dd + V.off, G + V.off, R + V.off, Di + V.off, T(0), T(step_coef(P, L, 1).c2), 1);
  }
  for (int l = L; l >= 1; --l) {
    DevLevel& V = P.lv[l];
    const int64_t n = V.v.n_dofs;
    // residual r = g - A x on S and I rows (0 on D rows)
    if (V.n_S > 0) {
      smooth_steps<T>(P, Wk, l, 2, s);
      dev::Epi<T> ep;
      ep.y = R + V.off;
      ep.g = G + V.off;
      ep.flags = V.v.flags;
      op.op(V.v, dev::kEpiResid, X + V.off, ep, E, mats<T>(P), s);
      op.sum(V.v, dev::kEpiResid, E, ep, s);
    } else {
      hipLaunchKernelGGL(dev::seg_residual<T>, dim3(grid1(n)), dim3(dev::kBlock), 0, s, n, (const int32_t*)nullptr,
                         (const T*)E, G + V.off, V.v.flags, R + V.off, 0);
    }
    // restriction into level l-1 and its first smoothing step from x = 0
    DevLevel& W = P.lv[l - 1];
    if (l - 1 >= 1) {
      dev::Epi<T> ep;
      ep.x = X + W.off;
      ep.d = Dd + W.off;
      ep.g = G + W.off;
      ep.dinv = Di + W.off;
      ep.flags = W.v.flags;
      ep.c2 = T(step_coef(P, l - 1, 1).c2);
      ep.smooth = 1;
      op.restrict_fc(V.v, W.v, R + V.off, ep, (T*)Wk.rbuf, E, mats<T>(P), s);
      op.sum(W.v, dev::kEpiRStart, E, ep, s);
    } else {
      op.restrict0(V.v, R + V.off, E, mats<T>(P), s);
      hipLaunchKernelGGL(dev::seg_restrict_start<T>, dim3(grid1(W.v.n_dofs)), dim3(dev::kBlock), 0, s, W.v.n_dofs,
                         W.v.roff, (const T*)E, G + W.off, X + W.off, Dd + W.off, Di + W.off, T(0), 0);
    }
  }
  hipLaunchKernelGGL(dev::coarse_solve<T>, dim3(1), dim3(dev::kBlock), P.n0 * sizeof(double), s,
                     (int)P.lv[0].v.n_dofs, P.n0, P.ainv, P.cidx, G + P.lv[0].off, X + P.lv[0].off);
  for (int l = 1; l <= L; ++l) {
    DevLevel& V = P.lv[l];
    op.prolong(V.v, P.lv[l - 1].v, X + P.lv[l - 1].off, X + V.off, mats<T>(P), s);
    if (V.n_S > 0) smooth_steps<T>(P, Wk, l, 1, s);
  }
  if (dot_rz)  // partial sums of r.z for the CG (the dot's grid)
    hipLaunchKernelGGL(dev::copy_from_levels_dot<T>, dim3(fuse_grid(N)), dim3(dev::kBlock), 0, s, N, P.copy,
                       (const T*)X, z, r, P.part);
  else
    hipLaunchKernelGGL(dev::copy_from_levels<T>, dim3(grid1(N)), dim3(dev::kBlock), 0, s, N, P.copy, X, z);
}

// the V-cycle work memory inside the problem's workspace
static VWork own_work(const Problem& P) {
  VWork W;
  W.lx = P.lx;
  W.lg = P.lg;
  W.lt = P.lt;
  W.ld = P.ld;
  W.E = P.E;
  W.rbuf = P.rbuf;
  return W;
}

static void vcycle_any(Problem& P, const VWork& W, const double* r, double* z, hipStream_t s,
                       bool dot_rz = false) {
  if (P.opt.mg_precision == 32)
    vcycle_t<float>(P, W, r, z, s, dot_rz);
  else
    vcycle_t<double>(P, W, r, z, s, dot_rz);
}

void vcycle(Problem& P, const double* r, double* z, hipStream_t s) {
  if (!P.bound) fail(GMG_E_STATE, "problem not bound");
  vcycle_any(P, own_work(P), r, z, s);
  HIPCHECK(hipGetLastError());
}

// ---------------------------------------------------------------- fixed scratch
// Work memory of gmg_vcycle_noalloc, for callers that cannot allocate device
// memory: one array per GPU, created when the library's code is loaded on
// that GPU and held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device
// address): the device address comes from hipGetSymbolAddress, looked up once
// per device with that device current.
static __device__ __align__(256) char scratch[GMG_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};
}  // namespace

// device address of the scratch array on the current device
static char* scratch_on(int device) {
  if (device < 0 || device >= kMaxDevices) fail(GMG_E_INVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      fail(GMG_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[device] = (char*)ptr;
  }
  return g_scratch[device];
}

// the V-cycle work memory carved from base (256-byte aligned pieces); with
// base == nullptr only the size is computed
static size_t carve_work(const Problem& P, char* base, VWork* W) {
  const size_t esz = P.opt.mg_precision == 32 ? 4 : 8;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return p;
  };
  VWork w;
  w.lx = take(size_t(P.n_total) * esz);
  w.lg = take(size_t(P.n_total) * esz);
  w.lt = take(size_t(P.n_total) * esz);
  w.ld = take(size_t(P.n_total) * esz);
  w.E = (double*)take(size_t(P.e_levels) * sizeof(double));
  w.rbuf = take(size_t(P.fam_max) * P.maps->npc * esz);
  if (W) *W = w;
  return off;
}

void vcycle_noalloc(Problem& P, const double* r, double* z, hipStream_t s) {
  if (!P.bound) fail(GMG_E_STATE, "problem not bound");
  int device = -1;
  HIPCHECK(hipGetDevice(&device));
  if (device != P.device) fail(GMG_E_STATE, "the current device is not the one the problem is bound on");
  const size_t need = carve_work(P, nullptr, nullptr);
  if (need > GMG_NOALLOC_SCRATCH_BYTES)
    fail(GMG_E_INVAL, "V-cycle work memory of this problem (" + std::to_string(need) +
                          " bytes) exceeds the fixed scratch (" + std::to_string((size_t)GMG_NOALLOC_SCRATCH_BYTES) +
                          " bytes)");
  char* base = scratch_on(device);
  VWork W;
  carve_work(P, base, &W);
  // the array keeps the previous call's contents: start from zero level
  // vectors as a freshly bound problem does (a fill kernel, no memset node)
  fill_dev((double*)base, int64_t(need / sizeof(double)), 0.0, s);
  vcycle_any(P, W, r, z, s);
  HIPCHECK(hipGetLastError());
}

// ---------------------------------------------------------------- batched V-cycle
// One V-cycle for each of several bound problems of the same dimension,
// degree, precision and smoother, with the level sweeps of all of them in
// one launch each: the levels are aligned from the coarse end (level l of
// every problem that has one, finest levels first on the way down), every
// smoothing step and residual pass (pass 1 and pass 2 of the level
// operator, with their epilogues) and the second pass of every restriction
// is one batched launch over the problems' levels, and the per-problem
// steps (leaf <-> level copies, transfers, coarse solve) run between them on
// the same stream.  Every problem sees exactly the operations of its own
// V-cycle in the same order, and the batched kernels give every family the
// logical block it gets alone, so each result equals the solo V-cycle's bit
// for bit.
namespace {
// A batched V-cycle (or CG iteration) as a host image of its launch tables
// and the launches that read them, in order (argument: the device address
// of the tables).
struct BatchPlan {
  std::vector<char> blob;
  std::vector<std::function<void(const char*)>> q;
  template <typename Item>
  size_t put(const std::vector<Item>& items) {
    const size_t off = (blob.size() + 255) & ~size_t(255);
    blob.resize(off + items.size() * sizeof(Item));
    std::memcpy(blob.data() + off, items.data(), items.size() * sizeof(Item));
    return off;
  }
};

// the items of one batched launch of a kernel body (a device function
// object called with its block index and grid size)
template <class F>
struct Launch {
  std::vector<dev::LaunchItem<F>> items;
  int64_t blocks = 0;
  size_t shmem = 0;
  void add(const F& f, int64_t nb) {
    if (nb <= 0) return;
    items.push_back(dev::LaunchItem<F>{f, blocks, nb});
    blocks += nb;
  }
  template <int TH = dev::kBlock>
  void emit(BatchPlan& B, hipStream_t s) const {
    if (items.empty()) return;
    const size_t off = B.put(items);
    const int n = (int)items.size();
    const int64_t nb = blocks;
    const size_t sh = shmem;
    B.q.push_back([=](const char* t) {
      hipLaunchKernelGGL((dev::run_items<F, TH>), dim3((unsigned)nb), dim3(TH), sh, s,
                         (const dev::LaunchItem<F>*)(t + off), n);
    });
  }
};

// batched transfers of one kind
template <typename T>
struct Xfer {
  std::vector<dev::XferItem<T>> items;
  int64_t blocks = 0;
  void add(dev::XferItem<T> it, int64_t nb) {
    if (nb <= 0) return;
    it.b0 = blocks;
    it.nb = nb;
    items.push_back(it);
    blocks += nb;
  }
  void emit(BatchPlan& B, const LevelOps<T>& op, int kind, const MatsH<T>& mt, hipStream_t s) const {
    if (items.empty()) return;
    const size_t off = B.put(items);
    const int n = (int)items.size();
    const int64_t nb = blocks;
    const LevelOps<T>* o = &op;
    B.q.push_back([=](const char* t) { o->xfer_batch(kind, (const dev::XferItem<T>*)(t + off), n, nb, mt, s); });
  }
};

// kernel bodies of the batched launches (device function objects)
template <typename T>
auto fill_body(int64_t n, T* p, T v) {
  return [=] __device__(int64_t b, int64_t nb) { dev::fill_at(n, p, v, b, nb); };
}
template <typename T>
auto copy_to_body(int64_t n, const int32_t* copy, const double* r, T* g) {
  return [=] __device__(int64_t b, int64_t) { dev::copy_to_levels_at(n, copy, r, g, b); };
}
template <typename T>
auto cheb_body(int64_t n, T* x, T* d, const T* g, T* t, const T* dinv, T c1, T c2, int zero_start) {
  return [=] __device__(int64_t b, int64_t) { dev::cheb_step_at(n, x, d, g, t, dinv, c1, c2, zero_start, b); };
}
template <typename T>
auto residual_body(int64_t n, const T* E, const T* g, const uint8_t* flags, T* r) {
  return [=] __device__(int64_t b, int64_t) {
    dev::seg_residual_at(n, (const int32_t*)nullptr, E, g, flags, r, 0, b);
  };
}
template <typename T>
auto rstart0_body(int64_t n, const int32_t* off, const T* E, T* g, T* x, T* d, const T* dinv) {
  return [=] __device__(int64_t b, int64_t) { dev::seg_restrict_start_at(n, off, E, g, x, d, dinv, T(0), 0, b); };
}
template <typename T>
auto coarse_body(int n_nodes, int n0, const double* ainv, const int32_t* idx, const T* d0, T* x0) {
  return [=] __device__(int64_t, int64_t) { dev::coarse_solve_at(n_nodes, n0, ainv, idx, d0, x0); };
}
template <typename T>
auto copy_from_body(int64_t n, const int32_t* copy, const T* lx, double* z) {
  return [=] __device__(int64_t b, int64_t) { dev::copy_from_levels_at(n, copy, lx, z, b); };
}
template <typename T>
auto copy_from_dot_body(int64_t n, const int32_t* copy, const T* lx, double* z, const double* r, double* part) {
  return [=] __device__(int64_t b, int64_t) { dev::copy_from_levels_dot_at(n, copy, lx, z, r, part, b); };
}
auto scalars_body(int nparts, const double* part, double* sc, int op) {
  return [=] __device__(int64_t, int64_t) { dev::cg_scalars_at(nparts, part, sc, op); };
}
auto update_p_body(int64_t n, double* p, const double* z, const double* sc) {
  return [=] __device__(int64_t b, int64_t) { dev::update_p_at(n, p, z, sc, b); };
}
auto update_xr_body(int64_t n, double* x, double* r, const double* p, const double* q, const double* sc,
                    double* part) {
  return [=] __device__(int64_t b, int64_t nb) { dev::update_xr_at(n, x, r, p, q, sc, part, b, nb); };
}
auto pass2_body(LeafView v, const double* E, const double* x, double* y, double* part) {
  return [=] __device__(int64_t b, int64_t) { dev::leaf_pass2_at<true>(v, E, x, y, part, b); };
}
}  // namespace

template <typename T>
static void plan_vcycle_batch(const std::vector<Problem*>& ps, const double* const* r, double* const* z,
                              hipStream_t s, bool dot_rz, BatchPlan& B) {
  const int np = (int)ps.size();
  const LevelOps<T>& op = ops<T>(*ps[0]);
  const MatsH<T> mt = mats<T>(*ps[0]);
  const int dim = ps[0]->maps->dim;
  const int m = ps[0]->opt.cheb_degree;
  const bool xb = op.xfer_batch != nullptr;
  int Lmax = 0;
  for (Problem* P : ps) Lmax = std::max(Lmax, (int)P->lv.size() - 1);
  auto level_of = [](Problem* P) { return (int)P->lv.size() - 1; };
  auto cheb_ep = [](Problem& P, int l, int j) {
    DevLevel& V = P.lv[l];
    dev::Epi<T> ep;
    ep.x = (T*)P.lx + V.off;
    ep.d = (T*)P.ld + V.off;
    ep.g = (T*)P.lg + V.off;
    ep.dinv = (const T*)P.ldinv + V.off;
    ep.flags = V.v.flags;
    const StepCoef c = step_coef(P, l, j);
    ep.c1 = T(c.c1);
    ep.c2 = T(c.c2);
    return ep;
  };
  // one batched level sweep (pass 1 + pass 2) with epilogue epi on level l of
  // the problems `who`; input of pass 1: their x on that level
  auto sweep = [&](int l, int epi, int step, const std::vector<int>& who) {
    if (who.empty()) return;
    std::vector<dev::OpItem<T>> oi;
    std::vector<dev::SumItem<T>> si;
    int64_t ob = 0, sb = 0;
    for (int i : who) {
      Problem& P = *ps[i];
      DevLevel& V = P.lv[l];
      dev::Epi<T> ep;
      if (epi == dev::kEpiCheb) {
        ep = cheb_ep(P, l, step);
      } else {
        ep.y = (T*)P.lt + V.off;
        ep.g = (T*)P.lg + V.off;
        ep.flags = V.v.flags;
      }
      oi.push_back(dev::OpItem<T>{V.v, ep, (const T*)P.lx + V.off, (T*)P.E, ob});
      si.push_back(dev::SumItem<T>{V.v, ep, (const T*)P.E, sb});
      ob += op.op_blocks(V.v);
      sb += (V.v.shn[dim + 1] + dev::kBlock - 1) / dev::kBlock;
    }
    const int n = (int)who.size();
    if (op.op_batch) {
      const size_t oo = B.put(oi);
      B.q.push_back([=, &op](const char* t) { op.op_batch((const dev::OpItem<T>*)(t + oo), n, ob, epi, mt, s); });
    } else {
      for (const auto& it : oi)
        B.q.push_back([=, &op](const char*) { op.op(it.v, epi, it.x, it.ep, it.E, mt, s); });
    }
    const size_t so = B.put(si);
    B.q.push_back([=, &op](const char* t) { op.sum_batch((const dev::SumItem<T>*)(t + so), n, sb, epi, s); });
  };
  // residual into the levels, first pre-smoothing step on each finest level
  {
    Launch<decltype(fill_body<T>(0, nullptr, T(0)))> lf;
    Launch<decltype(copy_to_body<T>(0, nullptr, nullptr, nullptr))> lc;
    Launch<decltype(cheb_body<T>(0, nullptr, nullptr, nullptr, nullptr, nullptr, T(0), T(0), 0))> lh;
    for (int i = 0; i < np; ++i) {
      Problem* P = ps[i];
      const int L = level_of(P);
      const int64_t N = P->maps->n_dofs;
      T *X = (T*)P->lx, *G = (T*)P->lg, *R = (T*)P->lt, *Dd = (T*)P->ld, *Di = (T*)P->ldinv;
      lf.add(fill_body<T>(P->n_total, G, T(0)), std::min<int64_t>(4096, grid1(P->n_total)));
      lc.add(copy_to_body<T>(N, P->copy, r ? r[i] : nullptr, G), grid1(N));
      if (L >= 1) {
        DevLevel& V = P->lv[L];
        lh.add(cheb_body<T>(V.v.n_dofs, X + V.off, Dd + V.off, G + V.off, R + V.off, Di + V.off, T(0),
                            T(step_coef(*P, L, 1).c2), 1),
               grid1(V.v.n_dofs));
      }
    }
    lf.emit(B, s);
    lc.emit(B, s);
    lh.emit(B, s);
  }
  for (int l = Lmax; l >= 1; --l) {
    std::vector<int> act, sm;
    for (int i = 0; i < np; ++i)
      if (level_of(ps[i]) >= l) {
        act.push_back(i);
        if (ps[i]->lv[l].n_S > 0) sm.push_back(i);
      }
    for (int j = 2; j <= m; ++j) sweep(l, dev::kEpiCheb, j, sm);
    sweep(l, dev::kEpiResid, 0, sm);
    Launch<decltype(residual_body<T>(0, nullptr, nullptr, nullptr, nullptr))> lres;
    Launch<decltype(rstart0_body<T>(0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr))> lrs0;
    Xfer<T> xf, xc, x0;
    std::vector<dev::SumItem<T>> rs;
    int64_t rb = 0;
    for (int i : act) {
      Problem* P = ps[i];
      DevLevel& V = P->lv[l];
      DevLevel& W = P->lv[l - 1];
      T *X = (T*)P->lx, *G = (T*)P->lg, *R = (T*)P->lt, *Dd = (T*)P->ld, *Di = (T*)P->ldinv;
      T* E = (T*)P->E;
      if (V.n_S == 0) lres.add(residual_body<T>(V.v.n_dofs, E, G + V.off, V.v.flags, R + V.off), grid1(V.v.n_dofs));
      if (l - 1 >= 1) {
        dev::Epi<T> ep;
        ep.x = X + W.off;
        ep.d = Dd + W.off;
        ep.g = G + W.off;
        ep.dinv = Di + W.off;
        ep.flags = W.v.flags;
        ep.c2 = T(step_coef(*P, l - 1, 1).c2);
        ep.smooth = 1;
        const LevelView fv = V.v, cv = W.v;
        T* rbuf = (T*)P->rbuf;
        const T* rin = R + V.off;
        if (xb) {
          dev::XferItem<T> a{};
          a.f = fv;
          a.in = rin;
          a.out = rbuf;
          xf.add(a, fv.n_fam ? op.xfer_blocks(kXRFine, fv) : 0);
          dev::XferItem<T> c{};
          c.c = cv;
          c.in = rbuf;
          c.ep = ep;
          c.E = E;
          xc.add(c, cv.n_fam ? op.xfer_blocks(kXRestrict, cv) : 0);
        } else {
          B.q.push_back([=, &op](const char*) { op.restrict_fc(fv, cv, rin, ep, rbuf, E, mt, s); });
        }
        rs.push_back(dev::SumItem<T>{W.v, ep, (const T*)E, rb});
        rb += (W.v.shn[dim + 1] + dev::kBlock - 1) / dev::kBlock;
      } else {
        const LevelView fv = V.v, cv = W.v;
        const T* rin = R + V.off;
        if (xb) {
          dev::XferItem<T> a{};
          a.f = fv;
          a.in = rin;
          a.E = E;
          x0.add(a, fv.n_fam ? op.xfer_blocks(kXRestrict0, fv) : 0);
        } else {
          B.q.push_back([=, &op](const char*) { op.restrict0(fv, rin, E, mt, s); });
        }
        lrs0.add(rstart0_body<T>(cv.n_dofs, cv.roff, E, G + W.off, X + W.off, Dd + W.off, Di + W.off),
                 grid1(cv.n_dofs));
      }
    }
    lres.emit(B, s);
    // the restriction launches after every residual of the level (the
    // non-batched ones were queued per problem above, in order)
    xf.emit(B, op, kXRFine, mt, s);
    xc.emit(B, op, kXRestrict, mt, s);
    x0.emit(B, op, kXRestrict0, mt, s);
    lrs0.emit(B, s);
    if (!rs.empty()) {
      const size_t so = B.put(rs);
      const int n = (int)rs.size();
      B.q.push_back([=, &op](const char* t) {
        op.sum_batch((const dev::SumItem<T>*)(t + so), n, rb, dev::kEpiRStart, s);
      });
    }
  }
  {
    Launch<decltype(coarse_body<T>(0, 0, nullptr, nullptr, nullptr, nullptr))> lco;
    for (int i = 0; i < np; ++i) {
      Problem* P = ps[i];
      lco.add(coarse_body<T>((int)P->lv[0].v.n_dofs, P->n0, P->ainv, P->cidx, (T*)P->lg + P->lv[0].off,
                             (T*)P->lx + P->lv[0].off),
              1);
      lco.shmem = std::max(lco.shmem, size_t(P->n0) * sizeof(double));
    }
    lco.emit(B, s);
  }
  for (int l = 1; l <= Lmax; ++l) {
    std::vector<int> sm;
    Xfer<T> xp;
    for (int i = 0; i < np; ++i) {
      Problem* P = ps[i];
      if (level_of(P) < l) continue;
      const LevelView fv = P->lv[l].v, cv = P->lv[l - 1].v;
      T* X = (T*)P->lx;
      const int64_t fo = P->lv[l].off, co = P->lv[l - 1].off;
      if (xb) {
        dev::XferItem<T> a{};
        a.f = fv;
        a.c = cv;
        a.in = X + co;
        a.out = X + fo;
        xp.add(a, fv.n_fam ? op.xfer_blocks(kXProlong, fv) : 0);
      } else {
        B.q.push_back([=, &op](const char*) { op.prolong(fv, cv, X + co, X + fo, mt, s); });
      }
      if (P->lv[l].n_S > 0) sm.push_back(i);
    }
    xp.emit(B, op, kXProlong, mt, s);
    for (int j = 1; j <= m; ++j) sweep(l, dev::kEpiCheb, j, sm);
  }
  if (dot_rz) {
    Launch<decltype(copy_from_dot_body<T>(0, nullptr, nullptr, nullptr, nullptr, nullptr))> lz;
    for (int i = 0; i < np; ++i) {
      Problem* P = ps[i];
      const int64_t N = P->maps->n_dofs;
      lz.add(copy_from_dot_body<T>(N, P->copy, (const T*)P->lx, z ? z[i] : nullptr, r ? r[i] : nullptr, P->part),
             fuse_grid(N));
    }
    lz.emit(B, s);
  } else {
    Launch<decltype(copy_from_body<T>(0, nullptr, nullptr, nullptr))> lz;
    for (int i = 0; i < np; ++i) {
      Problem* P = ps[i];
      const int64_t N = P->maps->n_dofs;
      lz.add(copy_from_body<T>(N, P->copy, (const T*)P->lx, z ? z[i] : nullptr), grid1(N));
    }
    lz.emit(B, s);
  }
}

// The CG iteration after the preconditioner (as cg_enqueue_tail) for every
// problem, each step one launch over all of them: beta and p = z + beta p;
// q = A p (tiled leaf operator, pass 2) with the partials of p.q; alpha;
// x += alpha p, r -= alpha q with the partials of r.r; the scalars to the
// host, the iteration's event recorded per problem.
static void plan_cg_tail_batch(const std::vector<Problem*>& ps, hipStream_t s, BatchPlan& B) {
  const int np = (int)ps.size();
  const KernelTable* kt = ps[0]->kt;
  Launch<decltype(scalars_body(0, nullptr, nullptr, 0))> s0, s1, s2;
  Launch<decltype(update_p_body(0, nullptr, nullptr, nullptr))> lp;
  Launch<decltype(fill_body<double>(0, nullptr, 0.0))> lz;
  Launch<decltype(pass2_body(LeafView{}, nullptr, nullptr, nullptr, nullptr))> l2;
  Launch<decltype(update_xr_body(0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr))> lx;
  std::vector<dev::LeafItem> li;
  int64_t lb = 0;
  size_t lds = 0;
  std::vector<int> per;  // problems whose leaf operator runs on its own (not tiled)
  for (int i = 0; i < np; ++i) {
    Problem* P = ps[i];
    const int64_t N = P->maps->n_dofs;
    s0.add(scalars_body((int)fuse_grid(N), P->part, P->scal, 0), 1);
    lp.add(update_p_body(N, P->cp, P->cz, P->scal), grid1(N));
    int nq;
    if (P->leaf.n_tiles && kt->leaf_t_batch) {
      const int64_t g1 = std::min<int64_t>(P->leaf.n_tiles, dev::kLeafBlocks);
      li.push_back(dev::LeafItem{P->leaf, P->cp, P->cq, P->E, P->part, lb, g1});
      lb += g1;
      lds = std::max(lds, size_t(P->leaf.max_nodes) * sizeof(double));
      if (P->leaf.n_p2 == 0) {
        lz.add(fill_body<double>(1, P->part + g1, 0.0), 1);
        nq = (int)g1 + 1;
      } else {
        const unsigned g2 = p2_grid(P->leaf.n_p2);
        l2.add(pass2_body(P->leaf, P->E, P->cp, P->cq, P->part + g1), g2);
        nq = (int)(g1 + g2);
      }
    } else {
      per.push_back(i);
      nq = P->leaf.n_tiles ? -1 : (int)fuse_grid(N);
      if (nq < 0) fail(GMG_E_STATE, "batched leaf operator unavailable");
    }
    s1.add(scalars_body(nq, P->part, P->scal, 1), 1);
    lx.add(update_xr_body(N, P->cg.u, P->cr, P->cp, P->cq, P->scal, P->part), dot_grid(N));
    s2.add(scalars_body((int)dot_grid(N), P->part, P->scal, 2), 1);
  }
  s0.emit(B, s);
  lp.emit(B, s);
  if (!li.empty()) {
    const size_t off = B.put(li);
    const int n = (int)li.size();
    const MatsH<double> m64 = ps[0]->m64;
    B.q.push_back([=](const char* t) { kt->leaf_t_batch((const dev::LeafItem*)(t + off), n, lb, lds, m64, s); });
  }
  for (int i : per) {
    Problem* P = ps[i];
    B.q.push_back([=](const char*) {
      const int64_t N = P->maps->n_dofs;
      P->kt->leaf_e(P->leaf, P->cp, P->E, false, P->m64, s);
      hipLaunchKernelGGL(dev::seg_dir_dot, dim3(fuse_grid(N)), dim3(dev::kBlock), 0, s, N, P->leaf.soff,
                         (const double*)P->E, P->leaf.dir, P->cq, P->cp, P->part);
    });
  }
  lz.emit(B, s);
  l2.emit(B, s);
  s1.emit(B, s);
  lx.emit(B, s);
  s2.emit(B, s);
  for (int i = 0; i < np; ++i) {
    Problem* P = ps[i];
    B.q.push_back([=](const char*) {
      HIPCHECK(hipMemcpyAsync(P->host, P->scal, dev::kNumScalars * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHECK(hipEventRecord(P->ev[4], s));
      P->cg.pending = true;
    });
  }
}

static void check_batch(const std::vector<Problem*>& ps) {
  if (ps.empty()) fail(GMG_E_INVAL, "empty batch");
  {
    std::vector<Problem*> u(ps);
    std::sort(u.begin(), u.end());
    if (std::adjacent_find(u.begin(), u.end()) != u.end()) fail(GMG_E_INVAL, "a problem twice in one batch");
  }
  for (Problem* P : ps) {
    if (!P->bound) fail(GMG_E_STATE, "problem not bound");
    if (P->kt != ps[0]->kt || P->opt.mg_precision != ps[0]->opt.mg_precision ||
        P->opt.cheb_degree != ps[0]->opt.cheb_degree || P->opt.smoother != ps[0]->opt.smoother ||
        P->device != ps[0]->device)
      fail(GMG_E_INVAL, "a batch needs one dimension, degree, precision, smoother and device");
  }
}

// uploads the plan's tables (through h_stage when given) and enqueues its
// launches; *need: bytes of the tables
static void run_plan(BatchPlan& B, char* d_table, size_t table_bytes, size_t* need, char* h_stage, hipStream_t s,
                     hipEvent_t staged) {
  const size_t bytes = std::max<size_t>(256, (B.blob.size() + 255) & ~size_t(255));
  if (need) *need = bytes;
  if (!d_table) return;
  if ((reinterpret_cast<uintptr_t>(d_table) & 255) != 0) fail(GMG_E_INVAL, "batch table must be 256-byte aligned");
  if (table_bytes < bytes) fail(GMG_E_INVAL, "batch table too small");
  if (!B.blob.empty()) {
    const char* src = B.blob.data();
    if (h_stage) {
      std::memcpy(h_stage, B.blob.data(), B.blob.size());
      src = h_stage;
    }
    HIPCHECK(hipMemcpyAsync(d_table, src, B.blob.size(), hipMemcpyHostToDevice, s));
  }
  if (staged) HIPCHECK(hipEventRecord(staged, s));
  for (auto& f : B.q) f(d_table);
  HIPCHECK(hipGetLastError());
}

void cg_iteration_batch(const std::vector<Problem*>& ps, char* d_table, size_t table_bytes, size_t* need,
                        char* h_stage, hipStream_t s, hipEvent_t staged) {
  check_batch(ps);
  std::vector<const double*> rs;
  std::vector<double*> zs;
  for (Problem* P : ps) {
    if (!P->cg.running) fail(GMG_E_STATE, "no solve in progress");
    rs.push_back(P->cr);
    zs.push_back(P->cz);
  }
  BatchPlan B;
  if (ps[0]->opt.mg_precision == 32)
    plan_vcycle_batch<float>(ps, rs.data(), zs.data(), s, true, B);
  else
    plan_vcycle_batch<double>(ps, rs.data(), zs.data(), s, true, B);
  plan_cg_tail_batch(ps, s, B);
  run_plan(B, d_table, table_bytes, need, h_stage, s, staged);
}

// Plans the batched V-cycle; with d_table, uploads the item tables (through
// h_stage, pinned host memory of at least table_bytes, when given; the event
// `staged`, when given, is recorded once the upload has read it) and
// enqueues it.  *need: bytes of the item tables.
void vcycle_batch(const std::vector<Problem*>& ps, const double* const* r, double* const* z, char* d_table,
                  size_t table_bytes, size_t* need, char* h_stage, hipStream_t s, bool dot_rz, hipEvent_t staged) {
  check_batch(ps);
  BatchPlan B;
  if (ps[0]->opt.mg_precision == 32)
    plan_vcycle_batch<float>(ps, r, z, s, dot_rz, B);
  else
    plan_vcycle_batch<double>(ps, r, z, s, dot_rz, B);
  run_plan(B, d_table, table_bytes, need, h_stage, s, staged);
}

// the CG preconditioner: replay of a captured graph of one V-cycle on the
// fixed CG buffers r -> z when enabled
static void precondition(Problem& P, hipStream_t s) {
  if (!P.opt.use_graph) {
    vcycle_any(P, own_work(P), P.cr, P.cz, s, true);
    return;
  }
  if (!P.graph) {
    hipStream_t cs;
    HIPCHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g;
    HIPCHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    vcycle_any(P, own_work(P), P.cr, P.cz, cs, true);
    HIPCHECK(hipStreamEndCapture(cs, &g));
    HIPCHECK(hipGraphInstantiate(&P.graph, g, nullptr, nullptr, 0));
    HIPCHECK(hipGraphDestroy(g));
    HIPCHECK(hipStreamDestroy(cs));
  }
  HIPCHECK(hipGraphLaunch(P.graph, s));
}

// level operator test hook in the device layout of the level: variant 0
// y = A_l x; variant 1 y = A^{SI} x^I on S rows, 0 elsewhere (the input
// restricted to I rows through the level's temporary vector)
template <typename T>
static void level_hook(Problem& P, int l, int variant, const T* x, T* y, hipStream_t s) {
  DevLevel& V = P.lv[l];
  const int64_t n = V.v.n_dofs;
  if (variant == 2) {
    // one Chebyshev step (the second of the semi-iteration) on the level's
    // V-cycle work vectors; x and y are not used
    if (l < 1) fail(GMG_E_INVAL, "smoothing step needs a level >= 1");
    const int keep = P.opt.cheb_degree;
    P.opt.cheb_degree = 2;
    smooth_steps<T>(P, own_work(P), l, 2, s);
    P.opt.cheb_degree = keep;
    return;
  }
  if (variant == 0) {
    level_apply<T>(P, l, x, y, s);
    return;
  }
  T* t = (T*)P.lt + V.off;
  hipLaunchKernelGGL(dev::mask_rows<T>, dim3(grid1(n)), dim3(dev::kBlock), 0, s, n, V.v.flags, 1, x, t);
  level_apply<T>(P, l, (const T*)t, y, s);
  hipLaunchKernelGGL(dev::mask_rows<T>, dim3(grid1(n)), dim3(dev::kBlock), 0, s, n, V.v.flags, 0, (const T*)y, y);
  fill_dev(t, n, T(0), s);
}

void apply_level_hook(Problem& P, int l, int variant, const void* x, void* y, hipStream_t s) {
  if (!P.bound) fail(GMG_E_STATE, "problem not bound");
  if (l < 0 || l >= (int)P.lv.size()) fail(GMG_E_INVAL, "level out of range");
  if (variant < 0 || variant > 2) fail(GMG_E_INVAL, "variant must be 0, 1 or 2");
  if (P.opt.mg_precision == 32)
    level_hook<float>(P, l, variant, (const float*)x, (float*)y, s);
  else
    level_hook<double>(P, l, variant, (const double*)x, (double*)y, s);
  HIPCHECK(hipGetLastError());
}

// ---------------------------------------------------------------- CG
// Preconditioned CG (x0 = 0, stop at ||r|| <= rtol ||b||) as a state machine:
// cg_start enqueues the set-up and the read-back of ||b||^2; every
// cg_poll that finds the last read-back complete checks it and enqueues the
// next iteration (V-cycle, r.z, p update, leaf operator, p.Ap, x/r update,
// r.r, read-back).  The scalars alpha, beta, rho stay on the device.
void cg_start(Problem& P, const double* b, double* u, hipStream_t s, bool timed) {
  if (!P.bound) fail(GMG_E_STATE, "problem not bound");
  const int64_t N = P.maps->n_dofs;
  const unsigned dg = dot_grid(N);
  double* sc = P.scal;
  CgState& C = P.cg;
  C = CgState{};
  C.u = u;
  C.stream = s;
  C.timed = timed;
  C.hist.assign(P.opt.max_iter + 1, 0.0);
  if (timed) HIPCHECK(hipEventRecord(P.ev[0], s));
  fill_dev(u, N, 0.0, s);
  fill_dev(P.cp, N, 0.0, s);
  hipLaunchKernelGGL(dev::copy_vec, dim3(dot_grid(N)), dim3(dev::kBlock), 0, s, N, b, P.cr);
  hipLaunchKernelGGL(dev::dot_partial, dim3(dg), dim3(dev::kBlock), 0, s, N, b, b, P.part);
  hipLaunchKernelGGL(dev::cg_scalars, dim3(1), dim3(dev::kBlock), 0, s, (int)dg, P.part, sc, 3);
  fill_dev(sc + dev::kFirst, 1, 1.0, s);
  HIPCHECK(hipMemcpyAsync(P.host, sc, dev::kNumScalars * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipEventRecord(P.ev[4], s));
  C.pending = true;
  C.running = true;
  P.timing[1] = 0.0;
  P.timing[2] = 0.0;
}

// the CG iteration after the preconditioner (z = B r with the partial sums
// of r.z already enqueued on s)
void cg_enqueue_tail(Problem& P, hipStream_t s) {
  CgState& C = P.cg;
  const int64_t N = P.maps->n_dofs;
  const unsigned dg = dot_grid(N);
  double* sc = P.scal;
  hipLaunchKernelGGL(dev::cg_scalars, dim3(1), dim3(dev::kBlock), 0, s, (int)fuse_grid(N), P.part, sc, 0);
  hipLaunchKernelGGL(dev::update_p, dim3(grid1(N)), dim3(dev::kBlock), 0, s, N, P.cp, P.cz, sc);
  // q = A p, with the partial sums of p.q
  const int nq = leaf_op(P, P.cp, P.cq, false, P.part, s, nullptr);
  hipLaunchKernelGGL(dev::cg_scalars, dim3(1), dim3(dev::kBlock), 0, s, nq, P.part, sc, 1);
  hipLaunchKernelGGL(dev::update_xr, dim3(dg), dim3(dev::kBlock), 0, s, N, C.u, P.cr, P.cp, P.cq, sc, P.part);
  hipLaunchKernelGGL(dev::cg_scalars, dim3(1), dim3(dev::kBlock), 0, s, (int)dg, P.part, sc, 2);
  HIPCHECK(hipMemcpyAsync(P.host, sc, dev::kNumScalars * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipEventRecord(P.ev[4], s));
  C.pending = true;
}

void cg_enqueue_iteration(Problem& P) {
  CgState& C = P.cg;
  hipStream_t s = C.stream;
  if (C.timed) HIPCHECK(hipEventRecord(P.ev[2], s));
  precondition(P, s);  // z = B r, with the partial sums of r.z
  if (C.timed) HIPCHECK(hipEventRecord(P.ev[3], s));
  cg_enqueue_tail(P, s);
}

static void cg_finish(Problem& P, int status) {
  CgState& C = P.cg;
  C.status = status;
  C.running = false;
  if (C.timed) {
    HIPCHECK(hipEventRecord(P.ev[1], C.stream));
    HIPCHECK(hipEventSynchronize(P.ev[1]));
    float ms = 0;
    (void)hipEventElapsedTime(&ms, P.ev[0], P.ev[1]);
    P.timing[0] = ms * 1e-3;
  }
}

// 0: the last enqueued work is still running; 1: the solve has finished
// (status in P.cg.status); 2: the next iteration is due (iteration count
// advanced, nothing enqueued yet)
int cg_check(Problem& P, bool block) {
  CgState& C = P.cg;
  if (!C.running) return 1;
  if (C.pending) {
    if (block) {
      HIPCHECK(hipEventSynchronize(P.ev[4]));
    } else {
      hipError_t e = hipEventQuery(P.ev[4]);
      if (e == hipErrorNotReady) return 0;
      if (e != hipSuccess) fail(GMG_E_HIP, std::string("hipEventQuery: ") + hipGetErrorString(e));
    }
    C.pending = false;
  }
  if (C.it == 0) {
    const double bb = P.host[dev::kBb];
    C.hist[0] = bb > 0 ? 1.0 : 0.0;
    if (!std::isfinite(bb)) {
      cg_finish(P, GMG_E_NAN);
      return 1;
    }
    if (bb == 0.0) {
      cg_finish(P, GMG_OK);
      return 1;
    }
    C.nb = std::sqrt(bb);
  } else {
    if (C.timed) {
      float ms = 0;
      (void)hipEventElapsedTime(&ms, P.ev[2], P.ev[3]);
      P.timing[1] += ms * 1e-3;
      P.timing[2] += 1;
    }
    const double rr = P.host[dev::kRr], rho = P.host[dev::kRho], pq = P.host[dev::kPq];
    const double res = std::sqrt(rr);
    C.hist[C.it] = res / C.nb;
    if (!std::isfinite(rr) || !std::isfinite(rho) || !std::isfinite(pq)) {
      cg_finish(P, GMG_E_NAN);
      return 1;
    }
    if (!(rho > 0.0) || !(pq > 0.0)) {
      cg_finish(P, GMG_E_BREAKDOWN);
      return 1;
    }
    if (res <= P.opt.rtol * C.nb) {
      cg_finish(P, GMG_OK);
      return 1;
    }
    if (C.it >= P.opt.max_iter) {
      cg_finish(P, GMG_NOT_CONVERGED);
      return 1;
    }
  }
  ++C.it;
  return 2;
}

// returns true when the solve has finished (status in P.cg.status); else
// enqueues the next iteration when it is due
bool cg_poll(Problem& P, bool block) {
  const int r = cg_check(P, block);
  if (r == 2) cg_enqueue_iteration(P);
  return r == 1;
}

int solve(Problem& P, const double* b, double* u, int32_t* iters, double* hist, hipStream_t s) {
  cg_start(P, b, u, s, true);
  while (!cg_poll(P, true)) {
  }
  *iters = P.cg.it;
  if (hist)
    for (int i = 0; i <= P.cg.it; ++i) hist[i] = P.cg.hist[i];
  HIPCHECK(hipGetLastError());
  return P.cg.status;
}

}  // namespace gmg
