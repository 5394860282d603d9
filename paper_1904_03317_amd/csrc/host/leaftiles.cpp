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
  std::vector<int32_t> list;
  std::vector<int64_t> nlist;
  int32_t max_nodes = 0;
};

}  // namespace

LeafTiles build_leaf_tiles(const Maps& M, int threads) {
  constexpr int TC = LeafTiles::kCells;
  const int nt = threads > 0 ? threads : (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
  const int npc = M.npc;
  if (npc * TC > 0x8000) fail(-1, "leaf tiles need at most 512 nodes per cell");
  const int64_t nl = M.n_leaves, N = M.n_dofs;
  if (N >= INT32_MAX) fail(-1, "leaf tiles need fewer than 2^31 DoFs");
  const std::vector<int32_t>& cm = M.leaf_cellmap;          // DoF or -(h+1) (hanging)
  const std::vector<int32_t>& cp = M.leaf_cellmap_parent;   // DoFs only
  LeafTiles T;
  T.n_tiles = (nl + TC - 1) / TC;
  const int64_t ntl = T.n_tiles;

  // own ranges: with first-touch numbering in leaf order, the DoFs numbered
  // before tile t are 0 .. (largest DoF of a node of the tiles before t);
  // the ranges partition [0, N) in any case, which is all that correctness
  // needs (a DoF outside its tile's range is listed by the tiles touching it)
  std::vector<int32_t> tmax(ntl, -1);
  const int tch = (int)std::max<int64_t>(1, std::min<int64_t>(8 * nt, (ntl + 63) / 64));
  for_chunks(tch, nt, [&](int ch) {
    const int64_t t0 = ntl * ch / tch, t1 = ntl * (ch + 1) / tch;
    for (int64_t t = t0; t < t1; ++t) {
      int32_t mx = -1;
      for (int64_t i = t * TC * npc, e = std::min<int64_t>(nl, (t + 1) * TC) * npc; i < e; ++i) {
        const int32_t d = cm[size_t(i)];
        if (d >= N) fail(-8, "leaf cell map out of range");
        mx = std::max(mx, d);
      }
      tmax[t] = mx;
    }
  });
  T.own.assign(ntl + 1, 0);
  for (int64_t t = 0; t < ntl; ++t) T.own[t + 1] = std::max(T.own[t], tmax[t] + 1);
  T.own[ntl] = (int32_t)N;

  // per tile: local index of every (cell, position), listed nodes in order of
  // first reference
  T.lmap.assign(size_t(nl) * npc, 0);
  std::vector<ChunkOut> outs(tch);
  for_chunks(tch, nt, [&](int ch) {
    const int64_t t0 = ntl * ch / tch, t1 = ntl * (ch + 1) / tch;
    ChunkOut& O = outs[ch];
    TileMap tm;
    for (int64_t t = t0; t < t1; ++t) {
      const int64_t c0 = t * TC, c1 = std::min<int64_t>(nl, c0 + TC);
      const int32_t lo = T.own[t], R = T.own[t + 1] - lo;
      const size_t base = O.list.size();
      tm.clear();
      for (int64_t c = c0; c < c1; ++c)
        for (int j = 0; j < npc; ++j) {
          const int32_t d = cp[size_t(c) * npc + j];
          if (d < 0 || d >= N) fail(-8, "leaf cell map out of range");
          int32_t i = d - lo;
          if (i < 0 || i >= R) {
            const int32_t n = (int32_t)(O.list.size() - base);
            const int32_t li = tm.get_or_insert(d, n);
            if (li == n) O.list.push_back(d);
            i = R + li;
          }
          if (i >= 0x8000) fail(-8, "leaf tile with too many nodes");
          T.lmap[size_t(c) * npc + j] = (uint16_t)i;
        }
      const int64_t L = (int64_t)(O.list.size() - base);
      O.nlist.push_back(L);
      O.max_nodes = std::max<int32_t>(O.max_nodes, R + (int32_t)L);
    }
  });
  T.list_off.assign(ntl + 1, 0);
  {
    int64_t t = 0, off = 0;
    for (int ch = 0; ch < tch; ++ch) {
      for (int64_t L : outs[ch].nlist) {
        T.list_off[t++] = off;
        off += L;
      }
      T.max_nodes = std::max(T.max_nodes, outs[ch].max_nodes);
    }
    T.list_off[ntl] = off;
    if (off >= INT32_MAX) fail(-1, "leaf tiles exceed 2^31 listed entries");
    T.list.assign(off + 1, 0);  // one padding entry, read by lanes without a listed node
    int64_t o = 0;
    for (int ch = 0; ch < tch; ++ch) {
      std::copy(outs[ch].list.begin(), outs[ch].list.end(), T.list.begin() + o);
      o += (int64_t)outs[ch].list.size();
      std::vector<int32_t>().swap(outs[ch].list);
    }
  }

  // second pass: every DoF with listed entries, its slots in ascending order
  const int64_t ns = T.n_slots();
  std::vector<int32_t> cnt(N, 0);
  for (int64_t i = 0; i < ns; ++i) ++cnt[T.list[i]];
  std::vector<int32_t> pos(N, -1);
  T.p2_off.push_back(0);
  for (int64_t d = 0; d < N; ++d)
    if (cnt[d]) {
      pos[d] = (int32_t)T.p2_dof.size();
      T.p2_dof.push_back((int32_t)d);
      T.p2_off.push_back(T.p2_off.back() + cnt[d]);
    }
  T.p2_slot.assign(ns, 0);
  std::vector<int32_t> cur(T.p2_off.begin(), T.p2_off.end() - 1);
  for (int64_t i = 0; i < ns; ++i) T.p2_slot[cur[pos[T.list[i]]]++] = (int32_t)i;
  return T;
}

}  // namespace gmg
