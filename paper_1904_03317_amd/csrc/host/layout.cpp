#include "layout.hpp"

#include <exception>
#include <string>
#include <thread>

#include "common.hpp"
#include "maps.hpp"

namespace gmg {

namespace {

struct EntityInfo {
  int r = 0;     // axes on the patch boundary
  int size = 1;  // nodes of the entity
  int q0 = 0;    // patch position of its first node
  int pos = 0;   // the family's position around the entity
};

// entity j = c_x + 3 c_y (+ 9 c_z) with c = 0 (low face), 1 (inside), 2 (high face)
EntityInfo entity_info(int dim, int k, int j) {
  const int m2 = 2 * k + 1, s1 = 2 * k - 1;
  EntityInfo e;
  int q[3] = {0, 0, 0};
  for (int a = 0, t = j; a < dim; ++a, t /= 3) {
    const int c = t % 3;
    if (c == 1) {
      q[a] = 1;
      e.size *= s1;
    } else {
      q[a] = c == 0 ? 0 : 2 * k;
      e.pos |= (c == 2 ? 1 : 0) << e.r;
      ++e.r;
    }
  }
  e.q0 = q[0] + m2 * (q[1] + m2 * q[2]);
  return e;
}

// entity and offset inside it of patch position q
void classify(int dim, int k, int q, int& j, int& loc) {
  const int m2 = 2 * k + 1, s1 = 2 * k - 1;
  j = 0;
  loc = 0;
  int mul = 1, st = 1;
  for (int a = 0; a < dim; ++a, q /= m2, mul *= 3) {
    const int qa = q % m2;
    const int c = qa == 0 ? 0 : qa == 2 * k ? 2 : 1;
    j += c * mul;
    if (c == 1) {
      loc += (qa - 1) * st;
      st *= s1;
    }
  }
}

void build_level(const Maps& M, const LevelData& D, LevelLayout& Y) {
  const int dim = M.dim, k = M.k, mf = M.mf;
  const int nj = dim == 3 ? 27 : 9;
  const int64_t nfam = D.n_fam;
  Y.n_fam = nfam;
  Y.n_dofs = D.n_dofs;
  std::vector<EntityInfo> ji(nj);
  for (int j = 0; j < nj; ++j) ji[j] = entity_info(dim, k, j);
  int size_r[4] = {1, 1, 1, 1};
  for (int j = 0; j < nj; ++j) size_r[ji[j].r] = ji[j].size;
  // entities in order of first appearance per section; the first family to
  // touch an entity owns it
  std::vector<int32_t> ent_of(D.n_dofs, -1);
  int64_t n_sec[4] = {nfam, 0, 0, 0};
  std::vector<int32_t> ent(size_t(nfam) * nj);
  std::vector<uint8_t> cnt_pm[4];  // per entity: presence mask
  Y.own.assign(nfam, 0u);
  for (int64_t f = 0; f < nfam; ++f)
    for (int j = 0; j < nj; ++j) {
      const EntityInfo& e = ji[j];
      if (e.r == 0) {
        ent[size_t(f) * nj + j] = (int32_t)f;
        Y.own[f] |= 1u << j;
        continue;
      }
      const int32_t old = D.famap[size_t(f) * mf + e.q0];
      if (ent_of[old] < 0) {
        ent_of[old] = (int32_t)n_sec[e.r]++;
        cnt_pm[e.r].push_back(0);
        Y.own[f] |= 1u << j;
      }
      const int32_t id = ent_of[old];
      ent[size_t(f) * nj + j] = id;
      uint8_t& pm = cnt_pm[e.r][id];
      if (pm & (1u << e.pos)) fail(-8, "two families at the same position of an entity");
      pm |= (uint8_t)(1u << e.pos);
    }
  // renumber inside each section: shared entities first (order kept)
  std::vector<int32_t> ren[4];
  for (int r = 1; r <= dim; ++r) {
    ren[r].assign(n_sec[r], -1);
    int32_t nxt = 0;
    for (int64_t i = 0; i < n_sec[r]; ++i)
      if (__builtin_popcount(cnt_pm[r][i]) >= 2) ren[r][i] = nxt++;
    Y.nsh[r] = nxt;
    for (int64_t i = 0; i < n_sec[r]; ++i)
      if (ren[r][i] < 0) ren[r][i] = nxt++;
  }
  for (int r = 0; r <= dim; ++r) {
    Y.sec[r + 1] = Y.sec[r] + n_sec[r] * size_r[r];
    if (r >= 1) {
      Y.shn[r + 1] = Y.shn[r] + Y.nsh[r] * size_r[r];
      Y.entoff[r + 1] = Y.entoff[r] + Y.nsh[r];
      Y.eoff[r + 1] = Y.eoff[r] + (int64_t(1) << r) * Y.nsh[r] * size_r[r];
    }
  }
  for (int r = dim + 2; r < 5; ++r) {
    Y.sec[r] = Y.sec[dim + 1];
    Y.shn[r] = Y.shn[dim + 1];
    Y.entoff[r] = Y.entoff[dim + 1];
    Y.eoff[r] = Y.eoff[dim + 1];
  }
  if (Y.sec[dim + 1] != D.n_dofs) fail(-8, "entity layout does not cover the level");
  Y.n_ent = Y.entoff[dim + 1];
  Y.n_slots = Y.eoff[dim + 1];
  if (Y.n_slots >= INT32_MAX || D.n_dofs >= INT32_MAX) fail(-1, "level exceeds 2^31 entries");
  Y.gbase.resize(size_t(nfam) * nj);
  Y.excl.assign(nfam, 0u);
  Y.pmask.assign(Y.n_ent, 0);
  for (int64_t f = 0; f < nfam; ++f)
    for (int j = 0; j < nj; ++j) {
      const EntityInfo& e = ji[j];
      if (e.r == 0) {
        Y.gbase[size_t(f) * nj + j] = (int32_t)(f * size_r[0]);
        Y.excl[f] |= 1u << j;
        continue;
      }
      const int32_t id0 = ent[size_t(f) * nj + j];
      const int32_t id = ren[e.r][id0];
      Y.gbase[size_t(f) * nj + j] = (int32_t)(Y.sec[e.r] + int64_t(id) * e.size);
      if (id < Y.nsh[e.r])
        Y.pmask[Y.entoff[e.r] + id] = cnt_pm[e.r][id0];
      else
        Y.excl[f] |= 1u << j;
    }
  // permutation, checked to be a bijection consistent over all families
  Y.perm.assign(D.n_dofs, -1);
  for (int64_t f = 0; f < nfam; ++f)
    for (int q = 0; q < mf; ++q) {
      int j, loc;
      classify(dim, k, q, j, loc);
      const int32_t nw = Y.gbase[size_t(f) * nj + j] + loc;
      int32_t& p = Y.perm[D.famap[size_t(f) * mf + q]];
      if (p >= 0 && p != nw) fail(-8, "entity layout inconsistent between families");
      p = nw;
    }
  std::vector<uint8_t> hit(D.n_dofs, 0);
  for (int64_t i = 0; i < D.n_dofs; ++i) {
    const int32_t p = Y.perm[i];
    if (p < 0 || p >= D.n_dofs || hit[p]) fail(-8, "entity layout is not a permutation");
    hit[p] = 1;
  }
}

}  // namespace

void build_layouts(Maps& M) {
  const int L = (int)M.levels.size() - 1;
  M.layouts.assign(L + 1, LevelLayout{});
  // level 0 keeps its numbering
  M.layouts[0].n_dofs = M.levels[0].n_dofs;
  M.layouts[0].perm.resize(M.levels[0].n_dofs);
  for (int64_t i = 0; i < M.levels[0].n_dofs; ++i) M.layouts[0].perm[i] = (int32_t)i;
  // levels are independent: one thread each (first exception rethrown)
  std::vector<std::thread> th;
  std::vector<std::exception_ptr> err(L + 1);
  for (int l = 1; l <= L; ++l)
    th.emplace_back([&M, &err, l] {
      try {
        build_level(M, M.levels[l], M.layouts[l]);
      } catch (...) {
        err[l] = std::current_exception();
      }
    });
  for (auto& t : th) t.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
  const int nf = 1 << M.dim;
  for (int l = 1; l < L; ++l) {
    LevelLayout& Y = M.layouts[l];
    const LevelData& F = M.levels[l + 1];
    Y.child.assign(size_t(Y.n_fam) * nf, -1);
    for (int64_t f = 0; f < F.n_fam; ++f) Y.child[F.parent[f]] = (int32_t)f;
  }
}

}  // namespace gmg
