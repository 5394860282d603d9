// Tiles of the leaf operator (see leaftiles.hpp).
#include "leaftiles.hpp"

#include <algorithm>
#include <atomic>
#include <exception>
#include <mutex>
#include <thread>

#include "common.hpp"
#include "maps.hpp"

namespace gmg {

namespace {

// fn(chunk) for chunk in [0, nch) on up to nt threads (this one included);
// the first exception is rethrown after all chunks finished
template <class F>
void for_chunks(int nch, int nt, F&& fn) {
  std::atomic<int> next{0};
  std::exception_ptr err;
  std::mutex mu;
  auto work = [&] {
    for (int c = next++; c < nch; c = next++) {
      try {
        fn(c);
      } catch (...) {
        std::lock_guard<std::mutex> lk(mu);
        if (!err) err = std::current_exception();
      }
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < std::min(nt, nch); ++t) th.emplace_back(work);
  work();
  for (auto& x : th) x.join();
  if (err) std::rethrow_exception(err);
}

// DoF -> local index of one tile (open addressing, cleared per tile)
class TileMap {
 public:
  TileMap() : keys_(kCap, -1), vals_(kCap, 0) {}
  // index of d, inserting it with index `next` if absent
  int32_t get_or_insert(int32_t d, int32_t next) {
    uint32_t i = (uint32_t)(mix64((uint64_t)(uint32_t)d) & (kCap - 1));
    while (true) {
      if (keys_[i] < 0) {
        keys_[i] = d;
        vals_[i] = next;
        used_.push_back(i);
        return next;
      }
      if (keys_[i] == d) return vals_[i];
      i = (i + 1) & (kCap - 1);
    }
  }
  void clear() {
    for (uint32_t i : used_) keys_[i] = -1;
    used_.clear();
  }

 private:
  // more than twice the largest node count of a tile (64 cells x 27)
  static constexpr uint32_t kCap = 4096;
  std::vector<int32_t> keys_, vals_;
  std::vector<uint32_t> used_;
};

struct ChunkOut {
  std::vector<int32_t> node;
  std::vector<int32_t> na, nb, ntot;
};

}  // namespace

LeafTiles build_leaf_tiles(const Maps& M, int threads) {
  constexpr int TC = LeafTiles::kCells;
  const int nt = threads > 0 ? threads : (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
  const int npc = M.npc;
  if (npc * TC > 0x8000) fail(-1, "leaf tiles need at most 512 nodes per cell");
  const int64_t nl = M.n_leaves, N = M.n_dofs;
  const std::vector<int32_t>& cm = M.leaf_cellmap_parent;
  LeafTiles T;
  T.n_tiles = (nl + TC - 1) / TC;
  const int64_t ntl = T.n_tiles;

  // contributions per DoF: the (cell, position) entries targeting it
  std::vector<uint16_t> total(N, 0);
  const int nch = (int)std::max<int64_t>(1, std::min<int64_t>(4 * nt, (nl + 4095) / 4096));
  for_chunks(nch, nt, [&](int ch) {
    const int64_t c0 = nl * ch / nch, c1 = nl * (ch + 1) / nch;
    for (int64_t c = c0; c < c1; ++c) {
      for (int j = 0; j < npc; ++j) {
        const int32_t d = cm[size_t(c) * npc + j];
        if (d < 0 || d >= N) fail(-8, "leaf cell map out of range");
        __atomic_fetch_add(&total[d], (uint16_t)1, __ATOMIC_RELAXED);
      }
    }
  });

  // per tile: first-touch node list; complete nodes (every contribution in
  // this tile) first
  T.lmap.assign(size_t(nl) * npc, 0);
  std::vector<uint8_t> complete(N, 0);
  const int tch = (int)std::max<int64_t>(1, std::min<int64_t>(8 * nt, (ntl + 63) / 64));
  std::vector<ChunkOut> outs(tch);
  for_chunks(tch, nt, [&](int ch) {
    const int64_t t0 = ntl * ch / tch, t1 = ntl * (ch + 1) / tch;
    ChunkOut& O = outs[ch];
    TileMap tm;
    std::vector<int32_t> ft, acc, rank;
    std::vector<int32_t> idx(size_t(TC) * npc);
    for (int64_t t = t0; t < t1; ++t) {
      const int64_t c0 = t * TC, c1 = std::min<int64_t>(nl, c0 + TC);
      tm.clear();
      ft.clear();
      acc.clear();
      for (int64_t c = c0; c < c1; ++c)
        for (int j = 0; j < npc; ++j) {
          const int32_t d = cm[size_t(c) * npc + j];
          const int32_t i = tm.get_or_insert(d, (int32_t)ft.size());
          if (i == (int32_t)ft.size()) {
            ft.push_back(d);
            acc.push_back(0);
          }
          ++acc[i];
          idx[size_t(c - c0) * npc + j] = i;
        }
      const int32_t n = (int32_t)ft.size();
      if (n >= 0x8000) fail(-8, "leaf tile with too many nodes");
      rank.assign(n, 0);
      int32_t na = 0;
      for (int32_t i = 0; i < n; ++i) na += acc[i] == total[ft[i]];
      int32_t pa = 0, pb = na;
      const size_t base = O.node.size();
      O.node.resize(base + n);
      for (int32_t i = 0; i < n; ++i) {
        const int32_t d = ft[i];
        int32_t r;
        if (acc[i] == total[d]) {
          r = pa++;
          complete[d] = 1;  // this tile is the only one touching d
          O.node[base + r] = M.dirichlet[d] ? ~d : d;
        } else {
          r = pb++;
          O.node[base + r] = d;
        }
        rank[i] = r;
      }
      for (int64_t c = c0; c < c1; ++c)
        for (int j = 0; j < npc; ++j) T.lmap[size_t(c) * npc + j] = (uint16_t)rank[idx[size_t(c - c0) * npc + j]];
      O.na.push_back(na);
      O.nb.push_back(n - na);
      O.ntot.push_back(n);
    }
  });
  T.node_off.assign(ntl + 1, 0);
  T.n_complete.resize(ntl);
  T.n_partial.resize(ntl);
  T.pbase.resize(ntl);
  {
    int64_t t = 0, off = 0, pb = 0;
    for (int ch = 0; ch < tch; ++ch)
      for (size_t i = 0; i < outs[ch].na.size(); ++i, ++t) {
        T.node_off[t] = off;
        T.n_complete[t] = outs[ch].na[i];
        T.n_partial[t] = outs[ch].nb[i];
        T.pbase[t] = (int32_t)pb;
        off += outs[ch].ntot[i];
        pb += outs[ch].nb[i];
        T.max_nodes = std::max(T.max_nodes, outs[ch].ntot[i]);
      }
    T.node_off[ntl] = off;
    T.n_part = pb;
    if (off >= INT32_MAX || pb >= INT32_MAX) fail(-1, "leaf tiles exceed 2^31 entries");
    T.node.resize(off);
    int64_t o = 0;
    for (int ch = 0; ch < tch; ++ch) {
      std::copy(outs[ch].node.begin(), outs[ch].node.end(), T.node.begin() + o);
      o += (int64_t)outs[ch].node.size();
      std::vector<int32_t>().swap(outs[ch].node);
    }
  }

  // second pass: every DoF not complete in a tile, with the partial slots
  // of the tiles touching it, in tile order
  std::vector<int32_t> pos(N, -1);
  for (int64_t d = 0; d < N; ++d)
    if (!complete[d]) {
      pos[d] = (int32_t)T.p2_dof.size();
      T.p2_dof.push_back((int32_t)d);
    }
  const int64_t n2 = (int64_t)T.p2_dof.size();
  std::vector<int64_t> cnt(n2 + 1, 0);
  for (int64_t t = 0; t < ntl; ++t) {
    const int64_t i0 = T.node_off[t] + T.n_complete[t];
    for (int32_t i = 0; i < T.n_partial[t]; ++i) ++cnt[pos[T.node[i0 + i]] + 1];
  }
  for (int64_t i = 0; i < n2; ++i) cnt[i + 1] += cnt[i];
  if (cnt[n2] >= INT32_MAX) fail(-1, "leaf slots exceed 2^31");
  T.p2_off.assign(cnt.begin(), cnt.end());
  T.p2_slot.assign(cnt[n2], 0);
  std::vector<int64_t> cur(cnt.begin(), cnt.end() - 1);
  for (int64_t t = 0; t < ntl; ++t) {
    const int64_t i0 = T.node_off[t] + T.n_complete[t];
    for (int32_t i = 0; i < T.n_partial[t]; ++i) T.p2_slot[cur[pos[T.node[i0 + i]]]++] = T.pbase[t] + i;
  }
  return T;
}

}  // namespace gmg
