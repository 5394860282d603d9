// Residual error estimator and marking of the adaptive loop (Sec. 4.3): the
// device work memory, the upload of the face tables, the launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>

#include "estkernels.hpp"
#include "host/common.hpp"
#include "problem.hpp"

namespace gmg {

namespace {

#define EHIPCHECK(x)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (x);                                                                      \
    if (e_ != hipSuccess) fail(GMG_E_HIP, std::string(#x ": ") + hipGetErrorString(e_));      \
  } while (0)

// layout of the estimator workspace (256-byte aligned parts)
struct EstLayout {
  size_t cmap, con_off, con_mas, con_w, level, eps, kind, off, nb, keys, idx_in, idx_out, temp, temp_bytes, total;
};

EstLayout est_layout(const Maps& M, const EstTables& T) {
  EstLayout L{};
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t o = at;
    at += (bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t nl = (size_t)M.n_leaves;
  L.cmap = take(nl * M.npc * sizeof(int32_t));
  L.con_off = take(T.con_off.size() * sizeof(int64_t));
  L.con_mas = take(std::max<size_t>(1, M.con_mas.size()) * sizeof(int32_t));
  L.con_w = take(std::max<size_t>(1, M.con_w.size()) * sizeof(double));
  L.level = take(nl);
  L.eps = take(nl * sizeof(double));
  L.kind = take(T.kind.size());
  L.off = take(T.off.size());
  L.nb = take(T.nb.size() * sizeof(int32_t));
  L.keys = take(nl * sizeof(double));
  L.idx_in = take(nl * sizeof(int32_t));
  L.idx_out = take(nl * sizeof(int32_t));
  L.temp_bytes = mark_temp_bytes((int64_t)nl);
  L.temp = take(L.temp_bytes);
  L.total = at;
  return L;
}

const EstTables& tables(Problem& P) {
  if (!P.est) P.est = std::make_shared<const EstTables>(build_est_tables(*P.maps));
  return *P.est;
}

// true when ws last received the tables of this problem; else records that
// it does now (the caller uploads them)
bool uploaded_by(const char* ws, const Problem& P) {
  static std::mutex mu;
  static std::unordered_map<const char*, const Maps*> owner;
  std::lock_guard<std::mutex> lk(mu);
  const Maps* m = P.maps.get();
  auto it = owner.find(ws);
  if (it != owner.end() && it->second == m && P.est_uploaded == ws) return true;
  owner[ws] = m;
  P.est_uploaded = ws;
  return false;
}

void check_ws(char* ws, size_t bytes, const EstLayout& L) {
  if (!ws) fail(GMG_E_INVAL, "null estimator workspace");
  if (reinterpret_cast<uintptr_t>(ws) & 255) fail(GMG_E_INVAL, "estimator workspace must be 256-byte aligned");
  if (bytes < L.total) fail(GMG_E_INVAL, "estimator workspace too small");
}

}  // namespace

size_t est_workspace_bytes(Problem& P) { return est_layout(*P.maps, tables(P)).total; }

void estimate(Problem& P, const double* u, const double* f, char* ws, size_t bytes, double* eta, hipStream_t s) {
  const Maps& M = *P.maps;
  const EstTables& T = tables(P);
  const EstLayout L = est_layout(M, T);
  check_ws(ws, bytes, L);
  if (!uploaded_by(ws, P)) {
    // the tables of this mesh into the workspace (once per workspace)
    EHIPCHECK(hipMemcpyAsync(ws + L.cmap, M.leaf_cellmap.data(), M.leaf_cellmap.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, s));
    EHIPCHECK(hipMemcpyAsync(ws + L.con_off, T.con_off.data(), T.con_off.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, s));
    if (!M.con_mas.empty()) {
      EHIPCHECK(hipMemcpyAsync(ws + L.con_mas, M.con_mas.data(), M.con_mas.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, s));
      EHIPCHECK(hipMemcpyAsync(ws + L.con_w, M.con_w.data(), M.con_w.size() * sizeof(double), hipMemcpyHostToDevice,
                               s));
    }
    EHIPCHECK(hipMemcpyAsync(ws + L.level, M.leaf_level.data(), M.leaf_level.size(), hipMemcpyHostToDevice, s));
    EHIPCHECK(hipMemcpyAsync(ws + L.eps, M.leaf_coeff.data(), M.leaf_coeff.size() * sizeof(double),
                             hipMemcpyHostToDevice, s));
    EHIPCHECK(hipMemcpyAsync(ws + L.kind, T.kind.data(), T.kind.size(), hipMemcpyHostToDevice, s));
    EHIPCHECK(hipMemcpyAsync(ws + L.off, T.off.data(), T.off.size(), hipMemcpyHostToDevice, s));
    EHIPCHECK(hipMemcpyAsync(ws + L.nb, T.nb.data(), T.nb.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    // the sources are host vectors of the problem, which outlive the copies
  }
  dev::EstView v;
  v.n_cells = M.n_leaves;
  v.cmap = reinterpret_cast<const int32_t*>(ws + L.cmap);
  v.con_off = reinterpret_cast<const int64_t*>(ws + L.con_off);
  v.con_mas = reinterpret_cast<const int32_t*>(ws + L.con_mas);
  v.con_w = reinterpret_cast<const double*>(ws + L.con_w);
  v.level = reinterpret_cast<const int8_t*>(ws + L.level);
  v.eps = reinterpret_cast<const double*>(ws + L.eps);
  v.kind = reinterpret_cast<const uint8_t*>(ws + L.kind);
  v.off = reinterpret_cast<const uint8_t*>(ws + L.off);
  v.nb = reinterpret_cast<const int32_t*>(ws + L.nb);
  const EstMats hm = est_mats(M);
  dev::EstMatsD m;
  static_assert(sizeof(EstMats) == sizeof(dev::EstMatsD), "estimator matrices layout");
  std::memcpy(&m, &hm, sizeof(m));
  P.kt->est(v, u, f, eta, m, s);
  EHIPCHECK(hipGetLastError());
}

void mark(Problem& P, const double* eta, double fraction, uint8_t* flags, char* ws, size_t bytes, hipStream_t s) {
  const Maps& M = *P.maps;
  const EstLayout L = est_layout(M, tables(P));
  check_ws(ws, bytes, L);
  if (!(fraction >= 0.0 && fraction <= 1.0)) fail(GMG_E_INVAL, "marking fraction must be in [0, 1]");
  const int64_t n = M.n_leaves;
  const int64_t m = (int64_t)std::floor(fraction * (double)n + 0.5);
  mark_top(eta, n, m, reinterpret_cast<double*>(ws + L.keys), reinterpret_cast<int32_t*>(ws + L.idx_in),
           reinterpret_cast<int32_t*>(ws + L.idx_out), ws + L.temp, L.temp_bytes, flags, s);
}

}  // namespace gmg
