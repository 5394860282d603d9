#include "maps.hpp"

#include <algorithm>
#include <atomic>
#include <exception>
#include <mutex>
#include <thread>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>

namespace gmg {

namespace {

// Per-axis node code.  Nodes at the cell ends and (even k) at the midpoint
// are identified by their exact dyadic coordinate (units 2^-21, relative to
// the lower corner of the coarse bounding box).  Interior Gauss-Lobatto
// points (k >= 3) never coincide with a node of another cell level or
// position; they are identified by (level, cell index, j), tagged by bit 31.
struct AxisCoder {
  int k;
  int64_t lo;  // box lower corner along the axis, units 2^-20
  uint32_t code(int level, int64_t a, int j) const {
    int64_t s = side_of(level);
    int64_t X;
    if (j == 0)
      X = 2 * a;
    else if (j == k)
      X = 2 * (a + s);
    else if ((k % 2 == 0) && 2 * j == k)
      X = 2 * a + s;
    else {
      uint64_t c = uint64_t((a - lo) / s);
      return 0x80000000u | (uint32_t(level) << 26) | (uint32_t(j) << 23) | uint32_t(c);
    }
    return uint32_t(X - 2 * lo);
  }
};

inline u128 make_key(const uint32_t* c, int dim) {
  u128 k = c[0];
  k |= u128(c[1]) << 32;
  if (dim == 3) k |= u128(c[2]) << 64;
  return k;
}

struct Ctx {
  const Forest& f;
  int dim, k, n, npc;
  AxisCoder ax[3];
  FE1D fe;
  Ctx(const Forest& f_, int k_) : f(f_), dim(f_.dim()), k(k_), n(k_ + 1) {
    npc = 1;
    for (int i = 0; i < dim; ++i) npc *= n;
    for (int i = 0; i < 3; ++i) ax[i] = AxisCoder{k, int64_t(f.box_lo()[i]) << kDepth};
    fe = make_fe1d(k);
  }
  // codes[i][j] of a cell
  void cell_codes(const Cell& c, uint32_t codes[3][5]) const {
    for (int i = 0; i < dim; ++i)
      for (int j = 0; j < n; ++j) codes[i][j] = ax[i].code(c.level, c.a[i], j);
  }
  u128 node_key(const uint32_t codes[3][5], int lidx) const {
    uint32_t c[3] = {0, 0, 0};
    for (int i = 0; i < dim; ++i) {
      c[i] = codes[i][lidx % n];
      lidx /= n;
    }
    return make_key(c, dim);
  }
  // node on the boundary of the domain (a union of unit cells): some unit
  // cell around it is not a coarse cell
  bool on_boundary(u128 key) const {
    int64_t cand[3][2];
    int nc[3] = {1, 1, 1};
    cand[2][0] = 0;
    bool any_int = false;
    for (int i = 0; i < dim; ++i) {
      uint32_t c = uint32_t(key >> (32 * i));
      int64_t lo = ax[i].lo;
      if (c & 0x80000000u) {
        int level = (c >> 26) & 31;
        int64_t ci = c & ((1u << 23) - 1);
        int64_t a = lo + ci * side_of(level);
        cand[i][0] = floor_to(a, int64_t(1) << kDepth) >> kDepth;
      } else {
        int64_t X = int64_t(c) + 2 * lo;   // units 2^-21
        int64_t unit = int64_t(1) << (kDepth + 1);
        int64_t q = floor_to(X, unit) / unit;
        if (X % unit == 0) {
          cand[i][0] = q - 1;
          cand[i][1] = q;
          nc[i] = 2;
          any_int = true;
        } else {
          cand[i][0] = q;
        }
      }
    }
    if (!any_int) return false;
    for (int z = 0; z < nc[2]; ++z)
      for (int y = 0; y < nc[1]; ++y)
        for (int x = 0; x < nc[0]; ++x) {
          int64_t u[3] = {cand[0][x], cand[1][y], cand[2][z]};
          if (f.tree_of_unit(u) < 0) return true;
        }
    return false;
  }
  Cell parent_of(const Cell& c) const {
    Cell p = c;
    p.level = c.level - 1;
    int64_t S = side_of(p.level);
    for (int i = 0; i < dim; ++i) p.a[i] = (int32_t)floor_to(c.a[i], S);
    return p;
  }
  // leaf neighbours of the parent of a level-l cell (level l-1, across faces,
  // edges and corners); returns offsets whose neighbour is a leaf
  int leaf_neighbours(const Cell& p, std::array<int, 3>* out) const {
    int m = 0;
    int64_t S = side_of(p.level);
    for (auto& off : f.offsets()) {
      int64_t na[3] = {p.a[0] + off[0] * S, p.a[1] + off[1] * S, dim == 3 ? p.a[2] + off[2] * S : 0};
      if (f.status(p.level, na) == 1) out[m++] = off;
    }
    return m;
  }
  // per-axis K-local indices in the closure of the parent's neighbour at
  // offset `off`; false if K does not touch it
  bool touch(const Cell& K, const Cell& P, const std::array<int, 3>& off, int lists[3][5],
             int cnt[3]) const {
    int64_t S = side_of(P.level), s = side_of(K.level);
    for (int i = 0; i < dim; ++i) {
      if (off[i] == 1) {
        if (K.a[i] + s != P.a[i] + S) return false;
        lists[i][0] = k;
        cnt[i] = 1;
      } else if (off[i] == -1) {
        if (K.a[i] != P.a[i]) return false;
        lists[i][0] = 0;
        cnt[i] = 1;
      } else {
        for (int j = 0; j < n; ++j) lists[i][j] = j;
        cnt[i] = n;
      }
    }
    if (dim == 2) {
      lists[2][0] = 0;
      cnt[2] = 1;
    }
    return true;
  }
};

struct HangRec {
  int64_t start = 0;   // masters in the pools of chunk `part`
  int32_t nm = 0;
  int32_t id = -1;     // hanging id (first touch), -1 until numbered
  int32_t part = 0;
};

// fn(chunk, begin, end) over [0, n) cut into nch contiguous chunks, on nt
// threads (this one included); the first exception is rethrown after all
// chunks finished.
template <class F>
void chunked(int64_t n, int nch, int nt, F&& fn) {
  std::atomic<int> next{0};
  std::exception_ptr err;
  std::mutex mu;
  auto work = [&] {
    for (int c = next++; c < nch; c = next++) {
      try {
        fn(c, n * c / nch, n * (c + 1) / nch);
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

// Global first-touch ids of keys listed per chunk (chunks in order; inside
// a chunk in its first-touch order, without repeats): remap[c][i] is the id
// of key ck[c][i], keys lists the keys by id and M maps key -> id.  The id
// of a key is the rank of its first occurrence in chunk order, as a
// sequential pass would number it.  Parallel over the parts of M: every
// occurrence of a key falls in the same part.
void merge_first_touch(const std::vector<std::vector<u128>>& ck, int nt, PKeyMap& M, std::vector<u128>& keys,
                       std::vector<std::vector<int32_t>>& remap) {
  const int nch = (int)ck.size();
  constexpr int P = PKeyMap::P;
  size_t total = 0;
  for (const auto& c : ck) total += c.size();
  if (total < 100000) nt = 1;  // small meshes: no threads (their start-up costs more than the work)
  std::vector<std::vector<int32_t>> bk(size_t(nch) * P);
  chunked(nch, nch, nt, [&](int c, int64_t, int64_t) {
    for (size_t i = 0; i < ck[c].size(); ++i) bk[size_t(c) * P + PKeyMap::part_of(ck[c][i])].push_back((int32_t)i);
  });
  // per part, in chunk order: the first occurrence of each key, and for
  // every later one a reference (c0 << 32 | i0) to it
  std::vector<std::vector<int64_t>> ref(nch);
  for (int c = 0; c < nch; ++c) ref[c].assign(ck[c].size(), -1);
  std::vector<std::vector<int64_t>> firsts(P);
  chunked(P, P, nt, [&](int p, int64_t, int64_t) {
    size_t n = 0;
    for (int c = 0; c < nch; ++c) n += bk[size_t(c) * P + p].size();
    KeyMap& m = M.part(p);
    m = KeyMap(n + 64);
    std::vector<int64_t>& fs = firsts[p];
    for (int c = 0; c < nch; ++c)
      for (int32_t i : bk[size_t(c) * P + p]) {
        const int32_t nxt = (int32_t)fs.size();
        const int32_t v = m.get_or_insert(ck[c][i], nxt);
        if (v == nxt)
          fs.push_back((int64_t(c) << 32) | uint32_t(i));
        else
          ref[c][i] = fs[v];
      }
  });
  bk = std::vector<std::vector<int32_t>>();
  // ids in chunk order: first occurrences counted per chunk, numbered
  // from the chunk's prefix
  std::vector<int64_t> base(nch + 1, 0);
  chunked(nch, nch, nt, [&](int c, int64_t, int64_t) {
    int64_t n = 0;
    for (size_t i = 0; i < ck[c].size(); ++i) n += ref[c][i] < 0;
    base[c + 1] = n;
  });
  for (int c = 0; c < nch; ++c) base[c + 1] += base[c];
  keys.assign(base[nch], u128(0));
  remap.assign(nch, std::vector<int32_t>());
  chunked(nch, nch, nt, [&](int c, int64_t, int64_t) {
    remap[c].assign(ck[c].size(), -1);
    int64_t id = base[c];
    for (size_t i = 0; i < ck[c].size(); ++i)
      if (ref[c][i] < 0) {
        remap[c][i] = (int32_t)id;
        keys[id++] = ck[c][i];
      }
  });
  chunked(nch, nch, nt, [&](int c, int64_t, int64_t) {
    for (size_t i = 0; i < ck[c].size(); ++i)
      if (ref[c][i] >= 0) remap[c][i] = remap[ref[c][i] >> 32][uint32_t(ref[c][i])];
  });
  chunked(P, P, nt, [&](int p, int64_t, int64_t) {
    KeyMap& m = M.part(p);
    for (int64_t f : firsts[p]) m.set(ck[f >> 32][uint32_t(f)], remap[f >> 32][uint32_t(f)]);
  });
}


}  // namespace

namespace {
struct PhaseTimer {
  bool on = std::getenv("GMG_TRACE") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void mark(const char* what) {
    if (!on) return;
    auto n = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[gmg maps] %-18s %8.3f s\n", what, std::chrono::duration<double>(n - t).count());
    t = n;
  }
};
}  // namespace

Maps build_maps(const Forest& f, int k, const double* coeff, int threads) {
  PhaseTimer T;
  const int nthreads =
      threads > 0 ? threads : (int)std::min(16u, std::max(1u, std::thread::hardware_concurrency()));
  Ctx C(f, k);
  const int dim = C.dim, n = C.n, npc = C.npc;
  Maps M;
  M.dim = dim;
  M.k = k;
  M.n = n;
  M.npc = npc;
  M.mf = 1;
  for (int i = 0; i < dim; ++i) M.mf *= (2 * k + 1);
  M.own_words = (M.mf + 31) / 32;
  M.fe = C.fe;
  const auto& leaves = f.leaves();
  const int64_t nl = (int64_t)leaves.size();
  M.n_leaves = nl;
  M.leaf_level.resize(nl);
  M.leaf_anchor.resize(size_t(nl) * 3);
  M.leaf_coeff.resize(nl);
  for (int64_t i = 0; i < nl; ++i) {
    M.leaf_level[i] = leaves[i].c.level;
    for (int a = 0; a < 3; ++a) M.leaf_anchor[size_t(i) * 3 + a] = leaves[i].c.a[a];
    M.leaf_coeff[i] = coeff ? coeff[i] : 1.0;
    if (!(M.leaf_coeff[i] > 0.0) || !std::isfinite(M.leaf_coeff[i]))
      fail(-1, "cell coefficients must be positive and finite");
  }

  // ---------------------------------------------------------- levels (cores)
  // Level meshes depend only on the forest: number them on worker threads
  // while this thread numbers the leaf mesh.
  const int L = f.max_level();
  M.levels.resize(L + 1);
  std::vector<PKeyMap> lmaps(L + 1);
  std::exception_ptr level_error;
  std::mutex level_mu;
  auto parallel_levels = [&](auto&& fn) {
    std::atomic<int> next_level{0};
    const int nthreads = std::max(1, std::min<int>(L + 1, std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t)
      th.emplace_back([&] {
        for (int l = next_level++; l <= L; l = next_level++) {
          try {
            fn(l);
          } catch (...) {
            std::lock_guard<std::mutex> lk(level_mu);
            if (!level_error) level_error = std::current_exception();
          }
        }
      });
    for (auto& x : th) x.join();
    if (level_error) std::rethrow_exception(level_error);
  };
  std::vector<std::thread> level_threads;
  level_threads.emplace_back([&] {
    try {
      parallel_levels([&](int l) {
        PKeyMap& lmap = lmaps[l];
    LevelData& D = M.levels[l];
    D.level = l;
    const auto t_level = std::chrono::steady_clock::now();
    {
      int64_t s = side_of(l);
      uint64_t last = ~0ull;
      for (int64_t li = 0; li < nl; ++li) {
        const Cell& c = leaves[li].c;
        if (c.level < l) continue;
        Cell a = c;
        a.level = (int8_t)l;
        for (int i = 0; i < dim; ++i) a.a[i] = (int32_t)floor_to(c.a[i], s);
        uint64_t kk = f.key(a);
        if (kk == last) continue;
        last = kk;
        D.cells.push_back(a);
        D.keys.push_back(kk);
        D.leaf_index.push_back(c.level == l ? (int32_t)li : -1);
      }
    }
    D.n_cells = (int64_t)D.cells.size();
    D.cellmap.resize(size_t(D.n_cells) * npc);
    // first touch over the level cells, in chunks merged in cell order (as
    // the leaf numbering)
    const int lch = D.n_cells < 4096 ? 1 : 4 * nthreads;
    std::vector<std::vector<u128>> ckeys(lch);
    std::vector<std::vector<int32_t>> cremap(lch);
    chunked(D.n_cells, lch, nthreads, [&](int ch, int64_t cb, int64_t ce) {
      KeyMap lm(size_t(ce - cb) * (dim == 3 ? k * k * k : k * k) + 64);
      std::vector<u128>& ck = ckeys[ch];
      for (int64_t ci = cb; ci < ce; ++ci) {
        uint32_t kc[3][5];
        C.cell_codes(D.cells[ci], kc);
        for (int li = 0; li < npc; ++li) {
          u128 key = C.node_key(kc, li);
          const int32_t nxt = (int32_t)ck.size();
          int32_t id = lm.get_or_insert(key, nxt);
          if (id == nxt) ck.push_back(key);
          D.cellmap[size_t(ci) * npc + li] = id;
        }
      }
    });
    std::vector<u128> lkeys;
    merge_first_touch(ckeys, nthreads, lmap, lkeys, cremap);
    ckeys = std::vector<std::vector<u128>>();
    const int32_t next = (int32_t)lkeys.size();
    chunked(D.n_cells, lch, nthreads, [&](int ch, int64_t cb, int64_t ce) {
      for (size_t i = size_t(cb) * npc; i < size_t(ce) * npc; ++i) D.cellmap[i] = cremap[ch][D.cellmap[i]];
    });
    D.n_dofs = next;
    D.flags.assign(D.n_dofs, kFlagS);
    if (l >= 1) {
      // interface nodes: chunks collect them, the marking is sequential
      std::vector<std::vector<int32_t>> inode(lch);
      chunked(D.n_cells, lch, nthreads, [&](int ch, int64_t cb, int64_t ce) {
        std::array<int, 3> offs[26];
        uint64_t last_parent = ~0ull;
        int nn = 0;
        for (int64_t ci = cb; ci < ce; ++ci) {
          const Cell& K = D.cells[ci];
          Cell P = C.parent_of(K);
          uint64_t pk = f.key(P);
          if (pk != last_parent) {
            nn = C.leaf_neighbours(P, offs);
            last_parent = pk;
          }
          for (int q = 0; q < nn; ++q) {
            int lists[3][5], cnt[3];
            if (!C.touch(K, P, offs[q], lists, cnt)) continue;
            for (int jz = 0; jz < cnt[2]; ++jz)
              for (int jy = 0; jy < cnt[1]; ++jy)
                for (int jx = 0; jx < cnt[0]; ++jx) {
                  int li = lists[0][jx] + n * (lists[1][jy] + n * lists[2][jz]);
                  inode[ch].push_back(D.cellmap[size_t(ci) * npc + li]);
                }
          }
        }
      });
      for (const auto& v : inode)
        for (int32_t i : v) D.flags[i] = kFlagI;
    }
    chunked(D.n_dofs, lch, nthreads, [&](int, int64_t b0, int64_t e0) {
      for (int64_t i = b0; i < e0; ++i)
        if (C.on_boundary(lkeys[i])) D.flags[i] = kFlagD;
    });
    for (int64_t i = 0; i < D.n_dofs; ++i)
      if (D.flags[i] == kFlagI) D.ilist.push_back((int32_t)i);
    for (int64_t ci = 0; ci < D.n_cells; ++ci) {
      for (int li = 0; li < npc; ++li)
        if (D.flags[D.cellmap[size_t(ci) * npc + li]] == kFlagI) {
          D.edge_cells.push_back((int32_t)ci);
          break;
        }
    }
    if (T.on)
      std::fprintf(stderr, "[gmg maps] level %d: %lld cells, %lld nodes, %.3f s\n", l, (long long)D.n_cells,
                   (long long)D.n_dofs,
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t_level).count());
      });
    } catch (...) {
      std::lock_guard<std::mutex> lk(level_mu);
      if (!level_error) level_error = std::current_exception();
    }
  });
  struct JoinGuard {
    std::vector<std::thread>& t;
    ~JoinGuard() {
      for (auto& x : t)
        if (x.joinable()) x.join();
    }
  } join_guard{level_threads};

  // ---------------------------------------------------------- hanging nodes
  // a node of leaf K (level l) is hanging iff it lies in the closure of a
  // level-(l-1) leaf N (a neighbour of K's parent) and is not a node of N;
  // masters: N's nodes on the smallest entity holding it with nonzero
  // weight, z-major order; weights: N's tensor Lagrange basis at the node.
  // Leaves are split into contiguous chunks worked on in parallel; each
  // chunk records the hanging nodes it touches first, and the merge in leaf
  // order keeps the record of the first leaf touching each node (the record
  // a sequential pass over the leaves would make).
  const int nch = nl < 4096 ? 1 : 4 * nthreads;
  std::vector<uint8_t> maybe_hang(nl, 0);   // leaf touches a coarser leaf
  struct HangPart {
    std::vector<u128> key;
    std::vector<HangRec> rec;
    std::vector<u128> pm;
    std::vector<double> pw;
  };
  std::vector<HangPart> hparts(nch);
  chunked(nl, nch, nthreads, [&](int ch, int64_t cb, int64_t ce) {
    HangPart& H = hparts[ch];
    KeyMap lh(1024);
    std::array<int, 3> offs[26];
    uint64_t last_parent = ~0ull;
    int nn = 0;
    for (int64_t ci = cb; ci < ce; ++ci) {
      const Cell& K = leaves[ci].c;
      if (K.level == 0) continue;
      Cell P = C.parent_of(K);
      uint64_t pk = f.key(P);
      if (pk != last_parent) {
        nn = C.leaf_neighbours(P, offs);
        last_parent = pk;
      }
      if (nn == 0) continue;
      uint32_t kc[3][5];
      C.cell_codes(K, kc);
      for (int q = 0; q < nn; ++q) {
        const auto& off = offs[q];
        int lists[3][5], cnt[3];
        if (!C.touch(K, P, off, lists, cnt)) continue;
        maybe_hang[ci] = 1;
        Cell N = P;
        int64_t S = side_of(P.level), s = side_of(K.level);
        for (int i = 0; i < dim; ++i) N.a[i] = (int32_t)(P.a[i] + off[i] * S);
        uint32_t nc[3][5];
        C.cell_codes(N, nc);
        for (int jz = 0; jz < cnt[2]; ++jz)
          for (int jy = 0; jy < cnt[1]; ++jy)
            for (int jx = 0; jx < cnt[0]; ++jx) {
              int jl[3] = {lists[0][jx], lists[1][jy], lists[2][jz]};
              uint32_t hc[3] = {kc[0][jl[0]], kc[1][jl[1]], dim == 3 ? kc[2][jl[2]] : 0};
              const u128 key = make_key(hc, dim);
              if (lh.get(key) >= 0) continue;
              // per axis: fixed N index, or varying with the N basis weights
              int fixedJ[3] = {0, 0, 0};
              double w[3][5];
              bool all_fixed = true;
              for (int i = 0; i < dim; ++i) {
                if (off[i] == 1) {
                  fixedJ[i] = 0;
                } else if (off[i] == -1) {
                  fixedJ[i] = k;
                } else {
                  const uint32_t kcode = kc[i][jl[i]];
                  fixedJ[i] = -1;
                  for (int J = 0; J < n; ++J)
                    if (nc[i][J] == kcode) fixedJ[i] = J;
                  if (fixedJ[i] < 0) {
                    all_fixed = false;
                    int b = (int)((K.a[i] - P.a[i]) / s);
                    double xi = 0.5 * b + 0.5 * C.fe.x[jl[i]];
                    lagrange_values(C.fe, xi, w[i]);
                  }
                }
              }
              if (all_fixed) continue;
              int rc[3];
              for (int i = 0; i < 3; ++i) rc[i] = (i < dim && fixedJ[i] < 0) ? n : 1;
              HangRec r;
              r.start = (int64_t)H.pm.size();
              for (int a2 = 0; a2 < rc[2]; ++a2)
                for (int a1 = 0; a1 < rc[1]; ++a1)
                  for (int a0 = 0; a0 < rc[0]; ++a0) {
                    const int av[3] = {a0, a1, a2};
                    int J[3];
                    double ww = 1.0;
                    for (int i = 0; i < 3; ++i) {
                      if (i < dim && fixedJ[i] < 0) {
                        J[i] = av[i];
                        ww *= w[i][J[i]];
                      } else {
                        J[i] = i < dim ? fixedJ[i] : 0;
                      }
                    }
                    uint32_t mc[3] = {nc[0][J[0]], nc[1][J[1]], dim == 3 ? nc[2][J[2]] : 0};
                    H.pm.push_back(make_key(mc, dim));
                    H.pw.push_back(ww);
                  }
              r.nm = (int)((int64_t)H.pm.size() - r.start);
              lh.get_or_insert(key, (int32_t)H.rec.size());
              H.rec.push_back(r);
              H.key.push_back(key);
            }
      }
    }
  });
  T.mark("hanging (chunks)");
  size_t n_rec = 0;
  for (const HangPart& H : hparts) n_rec += H.rec.size();
  KeyMap hang(n_rec + 64);
  std::vector<HangRec> hrec;
  hrec.reserve(n_rec);
  for (int ch = 0; ch < nch; ++ch) {
    HangPart& H = hparts[ch];
    for (size_t i = 0; i < H.rec.size(); ++i) {
      const int32_t nxt = (int32_t)hrec.size();
      if (hang.get_or_insert(H.key[i], nxt) != nxt) continue;
      HangRec r = H.rec[i];
      r.part = ch;
      hrec.push_back(r);
    }
    H.key = std::vector<u128>();
    H.rec = std::vector<HangRec>();
  }

  T.mark("hanging");
  // ---------------------------------------------------------- leaf numbering
  // First touch over the leaves in order.  Each chunk numbers the nodes it
  // touches in its own first-touch order; merging the chunks in leaf order
  // then gives every node the id of the sequential pass (a node new to
  // chunk c is numbered in the order of its first touch inside c, which is
  // its first touch overall).  Hanging-node ids follow the same rule.
  PKeyMap dofs;
  std::vector<u128> dof_keys;
  std::vector<int8_t> dof_minlevel;
  std::vector<int32_t> hang_order;
  M.leaf_cellmap.resize(size_t(nl) * npc);
  {
    struct NumPart {
      std::vector<u128> key;
      std::vector<int8_t> minlev;
      std::vector<int32_t> hfirst;
      std::vector<int32_t> remap;
    };
    std::vector<NumPart> parts(nch);
    // cell map entries: local node id (>= 0) or -(hanging record + 1)
    chunked(nl, nch, nthreads, [&](int ch, int64_t cb, int64_t ce) {
      NumPart& Q = parts[ch];
      KeyMap lm(size_t(ce - cb) * (dim == 3 ? k * k * k : k * k) + 64);
      KeyMap lhs(64);
      for (int64_t ci = cb; ci < ce; ++ci) {
        const Cell& K = leaves[ci].c;
        uint32_t kc[3][5];
        C.cell_codes(K, kc);
        for (int li = 0; li < npc; ++li) {
          u128 key = C.node_key(kc, li);
          int32_t h = (hrec.empty() || !maybe_hang[ci]) ? -1 : hang.get(key);
          if (h >= 0) {
            if (lhs.get(u128(h)) < 0) {
              lhs.get_or_insert(u128(h), 0);
              Q.hfirst.push_back(h);
            }
            M.leaf_cellmap[size_t(ci) * npc + li] = -(h + 1);
            continue;
          }
          const int32_t nxt = (int32_t)Q.key.size();
          int32_t id = lm.get_or_insert(key, nxt);
          if (id == nxt) {
            Q.key.push_back(key);
            Q.minlev.push_back(K.level);
          } else if (K.level < Q.minlev[id]) {
            Q.minlev[id] = K.level;
          }
          M.leaf_cellmap[size_t(ci) * npc + li] = id;
        }
      }
    });
    T.mark("numbering (chunks)");
    {
      std::vector<std::vector<u128>> ck(nch);
      std::vector<std::vector<int32_t>> rm;
      for (int ch = 0; ch < nch; ++ch) ck[ch].swap(parts[ch].key);
      merge_first_touch(ck, nthreads, dofs, dof_keys, rm);
      ck = std::vector<std::vector<u128>>();
      // smallest level of the leaves containing each node
      dof_minlevel.assign(dof_keys.size(), INT8_MAX);
      for (int ch = 0; ch < nch; ++ch) {
        NumPart& Q = parts[ch];
        for (size_t i = 0; i < rm[ch].size(); ++i)
          if (Q.minlev[i] < dof_minlevel[rm[ch][i]]) dof_minlevel[rm[ch][i]] = Q.minlev[i];
        Q.remap.swap(rm[ch]);
        Q.minlev = std::vector<int8_t>();
        for (int32_t h : Q.hfirst)
          if (hrec[h].id < 0) {
            hrec[h].id = (int32_t)hang_order.size();
            hang_order.push_back(h);
          }
      }
    }
    const int32_t next = (int32_t)dof_keys.size();
    T.mark("numbering (merge)");
    chunked(nl, nch, nthreads, [&](int ch, int64_t cb, int64_t ce) {
      const std::vector<int32_t>& rm = parts[ch].remap;
      for (size_t i = size_t(cb) * npc; i < size_t(ce) * npc; ++i) {
        const int32_t v = M.leaf_cellmap[i];
        M.leaf_cellmap[i] = v >= 0 ? rm[v] : -(hrec[-v - 1].id + 1);
      }
    });
    M.n_dofs = next;
  }
  T.mark("leaf numbering");
  M.n_hanging = (int64_t)hang_order.size();
  M.dirichlet.resize(M.n_dofs);
  chunked(M.n_dofs, nch, nthreads, [&](int, int64_t b, int64_t e) {
    for (int64_t i = b; i < e; ++i) M.dirichlet[i] = C.on_boundary(dof_keys[i]) ? 1 : 0;
  });
  {
    const int64_t H = M.n_hanging;
    M.con_off.assign(H + 1, 0);
    for (int64_t i = 0; i < H; ++i) M.con_off[i + 1] = M.con_off[i] + hrec[hang_order[i]].nm;
    M.con_mas.resize(M.con_off[H]);
    M.con_w.resize(M.con_off[H]);
    chunked(H, nch, nthreads, [&](int, int64_t b, int64_t e) {
      for (int64_t i = b; i < e; ++i) {
        const HangRec& r = hrec[hang_order[i]];
        double sw = 0.0;
        const HangPart& H = hparts[r.part];
        for (int q = 0; q < r.nm; ++q) {
          int32_t id = dofs.get(H.pm[r.start + q]);
          if (id < 0) fail(-8, "constraint master is not a DoF (constraint chain)");
          M.con_mas[M.con_off[i] + q] = id;
          M.con_w[M.con_off[i] + q] = H.pw[r.start + q];
          sw += H.pw[r.start + q];
        }
        if (std::fabs(sw - 1.0) > 1e-12) fail(-8, "constraint weights do not sum to one");
      }
    });
  }
  // in-cell constraints: masks and parent-arranged DoF ids
  M.leaf_mask.assign(nl, 0);
  M.leaf_cellmap_parent = M.leaf_cellmap;
  chunked(nl, nch, nthreads, [&](int, int64_t cb, int64_t ce) {
    std::array<int, 3> offs[26];
    for (int64_t ci = cb; ci < ce; ++ci) {
      if (!maybe_hang[ci]) continue;
      const Cell& K = leaves[ci].c;
      const Cell P = C.parent_of(K);
      const int nn = C.leaf_neighbours(P, offs);
      int bit[3] = {0, 0, 0};
      for (int i = 0; i < dim; ++i) bit[i] = (int)((K.a[i] - P.a[i]) / side_of(K.level));
      bool face[3] = {false, false, false}, edge[3] = {false, false, false};
      for (int q = 0; q < nn; ++q) {
        const auto& o = offs[q];
        int nz = 0, touches = 1;
        for (int i = 0; i < dim; ++i)
          if (o[i]) {
            ++nz;
            if ((o[i] > 0 ? 1 : 0) != bit[i]) touches = 0;
          }
        if (!touches) continue;
        if (nz == 1) {
          for (int i = 0; i < dim; ++i)
            if (o[i]) face[i] = true;
        } else if (nz == 2 && dim == 3) {
          for (int i = 0; i < 3; ++i)
            if (!o[i]) edge[i] = true;
        }
      }
      // an edge of two hanging faces is part of them
      for (int a = 0; a < dim; ++a)
        if (edge[a])
          for (int b = 0; b < dim; ++b)
            if (b != a && face[b]) edge[a] = false;
      uint16_t mk = 0;
      for (int i = 0; i < dim; ++i) {
        mk |= (uint16_t)(bit[i] << i);
        if (face[i]) mk |= (uint16_t)(1u << (3 + i));
        if (edge[i]) mk |= (uint16_t)(1u << (6 + i));
      }
      if (!(mk >> 3)) continue;
      M.leaf_mask[ci] = mk;
      uint32_t pc[3][5];
      C.cell_codes(P, pc);
      for (int li = 0; li < npc; ++li) {
        int j[3] = {li % n, (li / n) % n, dim == 3 ? li / (n * n) : 0};
        bool hang_pos = false;
        for (int a = 0; a < dim; ++a) {
          if (face[a] && j[a] == bit[a] * k) hang_pos = true;
          if (edge[a]) {
            bool on = true;
            for (int b = 0; b < dim; ++b)
              if (b != a && j[b] != bit[b] * k) on = false;
            if (on) hang_pos = true;
          }
        }
        if (!hang_pos) continue;
        // parent node at the same local position
        uint32_t c3[3] = {pc[0][j[0]], pc[1][j[1]], dim == 3 ? pc[2][j[2]] : 0};
        int32_t id = dofs.get(make_key(c3, dim));
        if (id < 0) fail(-8, "parent node on a refinement edge is not a DoF");
        M.leaf_cellmap_parent[size_t(ci) * npc + li] = id;
      }
    }
  });
  for (auto v : M.leaf_cellmap_parent)
    if (v < 0) fail(-8, "hanging node outside an in-cell constraint");
  dofs.clear();
  T.mark("dirichlet+constraints");

  // ---------------------------------------------------------- levels (rest)
  for (auto& t : level_threads) t.join();
  if (level_error) std::rethrow_exception(level_error);
  T.mark("level numbering");
  // bucket leaf DoFs by the level that owns them in the hierarchy
  std::vector<int64_t> bstart(L + 2, 0);
  for (int64_t i = 0; i < M.n_dofs; ++i) ++bstart[dof_minlevel[i] + 1];
  for (int l = 0; l <= L; ++l) bstart[l + 1] += bstart[l];
  std::vector<int64_t> bucket(M.n_dofs);
  {
    std::vector<int64_t> pos(bstart.begin(), bstart.end() - 1);
    for (int64_t i = 0; i < M.n_dofs; ++i) bucket[pos[dof_minlevel[i]]++] = i;
  }
  M.copy_level.resize(M.n_dofs);
  M.copy_index.resize(M.n_dofs);
  parallel_levels([&](int l) {
    LevelData& D = M.levels[l];
    PKeyMap& lmap = lmaps[l];
    // copy map for the leaf DoFs owned by this level
    const int fch = bstart[l + 1] - bstart[l] < 65536 ? 1 : 4 * nthreads;
    chunked(bstart[l + 1] - bstart[l], fch, nthreads, [&](int, int64_t b0, int64_t e0) {
      for (int64_t b = bstart[l] + b0; b < bstart[l] + e0; ++b) {
        int64_t i = bucket[b];
        int32_t id = lmap.get(dof_keys[i]);
        if (id < 0 || D.flags[id] == kFlagI) fail(-8, "copy map: leaf DoF not an S/D node of its level");
        M.copy_level[i] = (int8_t)l;
        M.copy_index[i] = id;
      }
    });
    lmap.clear();
    // families and transfer maps
    if (l >= 1) {
      const LevelData& Pl = M.levels[l - 1];
      const int nf = 1 << dim;
      if (D.n_cells % nf) fail(-8, "level cells do not come in sibling families");
      D.n_fam = D.n_cells / nf;
      const int m2 = 2 * k + 1;
      D.parent.resize(D.n_fam);
      D.famap.assign(size_t(D.n_fam) * M.mf, -1);
      D.own.assign(size_t(D.n_fam) * M.own_words, 0u);
      // parents, family maps and the complete-layer check per family (in
      // chunks), then ownership by the first family touching each node
      const int pch = D.n_fam < 1024 ? 1 : 4 * nthreads;
      chunked(D.n_fam, pch, nthreads, [&](int, int64_t f0, int64_t f1) {
        for (int64_t fi = f0; fi < f1; ++fi) {
          Cell P = C.parent_of(D.cells[fi * nf]);
          uint64_t pk = f.key(P);
          auto it = std::lower_bound(Pl.keys.begin(), Pl.keys.end(), pk);
          if (it == Pl.keys.end() || *it != pk) fail(-8, "family parent not found");
          D.parent[fi] = (int32_t)(it - Pl.keys.begin());
          for (int cid = 0; cid < nf; ++cid) {
            const Cell& ch = D.cells[fi * nf + cid];
            for (int i = 0; i < dim; ++i)
              if (ch.a[i] != P.a[i] + ((cid >> i) & 1) * side_of(l))
                fail(-8, "family children out of order");
            for (int li = 0; li < npc; ++li) {
              int jx = li % n, jy = (li / n) % n, jz = li / (n * n);
              int fx = (cid & 1) * k + jx, fy = ((cid >> 1) & 1) * k + jy;
              int fz = dim == 3 ? ((cid >> 2) & 1) * k + jz : 0;
              int fidx = fx + m2 * (fy + m2 * fz);
              int32_t v = D.cellmap[size_t(fi * nf + cid) * npc + li];
              int32_t& slot = D.famap[size_t(fi) * M.mf + fidx];
              if (slot >= 0 && slot != v) fail(-8, "inconsistent family map");
              slot = v;
            }
          }
          // complete-layer rule: parent nodes touched by the transfer are S or D
          for (int li = 0; li < npc; ++li)
            if (Pl.flags[Pl.cellmap[size_t(D.parent[fi]) * npc + li]] == kFlagI)
              fail(-8, "complete-layer rule violated");
        }
      });
      std::vector<uint8_t> seen(D.n_dofs, 0);
      for (int64_t fi = 0; fi < D.n_fam; ++fi)
        for (int q = 0; q < M.mf; ++q) {
          int32_t v = D.famap[size_t(fi) * M.mf + q];
          if (!seen[v]) {
            seen[v] = 1;
            D.own[size_t(fi) * M.own_words + q / 32] |= 1u << (q % 32);
          }
        }
    }
    });
  T.mark("levels done");
  // cell coefficients: leaves from the input, other cells the mean of their
  // children (Sec. 4.3 coefficient, applied on every level)
  for (int l = L; l >= 0; --l) {
    LevelData& D = M.levels[l];
    D.coeff.assign(D.n_cells, 0.0);
    for (int64_t c = 0; c < D.n_cells; ++c)
      if (D.leaf_index[c] >= 0) D.coeff[c] = M.leaf_coeff[D.leaf_index[c]];
    if (l < L) {
      const LevelData& F = M.levels[l + 1];
      const int nf = 1 << dim;
      for (int64_t fi = 0; fi < F.n_fam; ++fi) {
        double s = 0.0;
        for (int c = 0; c < nf; ++c) s += F.coeff[fi * nf + c];
        D.coeff[F.parent[fi]] = s / nf;
      }
    }
  }
  build_layouts(M);
  T.mark("layouts");
  if (!(dim == 3 && k >= 3)) {
    M.tiles = build_leaf_tiles(M, nthreads);
    T.mark("leaf tiles");
    if (T.on)
      std::fprintf(stderr, "[gmg maps] leaf tiles: %lld tiles, %lld listed nodes, %zu second-pass DoFs, largest "
                   "tile %d nodes\n",
                   (long long)M.tiles.n_tiles, (long long)M.tiles.n_slots(), M.tiles.p2_dof.size(),
                   M.tiles.max_nodes);
  }
  return M;
}

}  // namespace gmg
