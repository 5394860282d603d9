#include "forest.hpp"

#include <algorithm>

namespace gmg {

namespace {
constexpr uint8_t kLeaf = 1, kRefined = 2;

uint64_t interleave(const uint64_t* v, int dim) {
  // bits of the three coordinates (16 each at the finest level) interleaved
  // with x in the lowest position: child id = x + 2y + 4z
  uint64_t m = 0;
  for (int b = kMaxLevel - 1; b >= 0; --b)
    for (int i = dim - 1; i >= 0; --i) m = (m << 1) | ((v[i] >> b) & 1u);
  return m;
}
}  // namespace

Forest::Forest(int dim, int n, const int32_t* origins) : dim_(dim) {
  if (dim != 2 && dim != 3) fail(-1, "dim must be 2 or 3");
  if (n < 1 || n > kMaxCoarse) fail(-1, "1 <= n_coarse <= 128 required");
  for (int i = 0; i < 3; ++i) {
    lo_[i] = 0;
    ext_[i] = 1;
  }
  std::array<int32_t, 3> hi{};
  for (int t = 0; t < n; ++t) {
    std::array<int32_t, 3> o{0, 0, 0};
    for (int i = 0; i < dim; ++i) o[i] = origins[t * dim + i];
    for (int i = 0; i < dim; ++i) {
      if (o[i] < -255 || o[i] > 255) fail(-1, "coarse origins must lie in [-255, 255]");
      lo_[i] = t == 0 ? o[i] : std::min(lo_[i], o[i]);
      hi[i] = t == 0 ? o[i] : std::max(hi[i], o[i]);
    }
    origins_.push_back(o);
  }
  for (int i = 0; i < dim; ++i) {
    ext_[i] = hi[i] - lo_[i] + 1;
    if (ext_[i] > kMaxExtent) fail(-1, "coarse mesh extent must be <= 16 cells per axis");
  }
  unit_tree_.assign(size_t(ext_[0]) * ext_[1] * ext_[2], -1);
  for (int t = 0; t < n; ++t) {
    auto& o = origins_[t];
    size_t idx = size_t(o[0] - lo_[0]) + size_t(ext_[0]) * (size_t(o[1] - lo_[1]) +
                                                            size_t(ext_[1]) * size_t(o[2] - lo_[2]));
    if (unit_tree_[idx] >= 0) fail(-1, "coarse cells must be distinct");
    unit_tree_[idx] = (int16_t)t;
  }
  for (int oz = (dim == 3 ? -1 : 0); oz <= (dim == 3 ? 1 : 0); ++oz)
    for (int oy = -1; oy <= 1; ++oy)
      for (int ox = -1; ox <= 1; ++ox)
        if (ox || oy || oz) offsets_.push_back({ox, oy, oz});
  for (int t = 0; t < n; ++t) {
    Cell c;
    c.level = 0;
    c.tree = (int16_t)t;
    for (int i = 0; i < 3; ++i) c.a[i] = origins_[t][i] * (int32_t)(1 << kDepth);
    if (dim == 2) c.a[2] = 0;
    cells_.set(key(c), kLeaf);
    leaves_.push_back({key(c), c});
  }
  std::sort(leaves_.begin(), leaves_.end(),
            [](const Leaf& x, const Leaf& y) { return x.key < y.key; });
}

int Forest::tree_of_unit(const int64_t* u) const {
  size_t idx = 0, mul = 1;
  for (int i = 0; i < dim_; ++i) {
    int64_t r = u[i] - lo_[i];
    if (r < 0 || r >= ext_[i]) return -1;
    idx += size_t(r) * mul;
    mul *= ext_[i];
  }
  return unit_tree_[idx];
}

int Forest::tree_of_anchor(const int64_t* a) const {
  int64_t u[3] = {0, 0, 0};
  for (int i = 0; i < dim_; ++i) u[i] = floor_to(a[i], int64_t(1) << kDepth) >> kDepth;
  return tree_of_unit(u);
}

uint64_t Forest::key(int level, const int64_t* a, int tree) const {
  uint64_t v[3] = {0, 0, 0};
  for (int i = 0; i < dim_; ++i)
    v[i] = uint64_t(a[i] - int64_t(origins_[tree][i]) * (int64_t(1) << kDepth)) >>
           (kDepth - kMaxLevel);
  return (uint64_t(tree) << 57) | (interleave(v, dim_) << 5) | uint64_t(level);
}

uint64_t Forest::key(const Cell& c) const {
  int64_t a[3] = {c.a[0], c.a[1], c.a[2]};
  return key(c.level, a, c.tree);
}

uint8_t Forest::status(int level, const int64_t* a) const {
  int t = tree_of_anchor(a);
  if (t < 0) return 0;
  return cells_.get(key(level, a, t));
}

int Forest::max_level() const {
  int m = 0;
  for (auto& l : leaves_) m = std::max(m, (int)l.c.level);
  return m;
}

void Forest::set_children(const Cell& c) {
  cells_.set(key(c), kRefined);
  int64_t s = side_of(c.level + 1);
  for (int cid = 0; cid < (1 << dim_); ++cid) {
    Cell ch = c;
    ch.level = c.level + 1;
    for (int i = 0; i < dim_; ++i) ch.a[i] = c.a[i] + (int32_t)(((cid >> i) & 1) * s);
    cells_.set(key(ch), kLeaf);
  }
}

void Forest::emit(const Cell& c, std::vector<Leaf>& out) const {
  uint64_t k = key(c);
  if (cells_.get(k) == kLeaf) {
    out.push_back({k, c});
    return;
  }
  int64_t s = side_of(c.level + 1);
  for (int cid = 0; cid < (1 << dim_); ++cid) {
    Cell ch = c;
    ch.level = c.level + 1;
    for (int i = 0; i < dim_; ++i) ch.a[i] = c.a[i] + (int32_t)(((cid >> i) & 1) * s);
    emit(ch, out);
  }
}

int64_t Forest::refine(const uint8_t* flags) {
  // cells refined in this round; the 2:1 requirement of their new children
  // is that every level-l neighbour of the refined level-l cell exists.
  std::vector<Cell> work;
  for (size_t i = 0; i < leaves_.size(); ++i)
    if (flags[i]) {
      if (leaves_[i].c.level >= kMaxLevel) fail(-1, "maximum level exceeded");
      work.push_back(leaves_[i].c);
    }
  while (!work.empty()) {
    for (auto& c : work)
      if (cells_.get(key(c)) == kLeaf) set_children(c);
    std::vector<Leaf> next;
    for (auto& c : work) {
      int l = c.level;
      if (l < 1) continue;
      int64_t s = side_of(l);
      for (auto& off : offsets_) {
        int64_t na[3] = {c.a[0] + off[0] * s, c.a[1] + off[1] * s, c.a[2] + off[2] * s};
        if (dim_ == 2) na[2] = 0;
        int t = tree_of_anchor(na);
        if (t < 0) continue;
        if (cells_.get(key(l, na, t))) continue;
        for (int m = l - 1; m >= 0; --m) {
          int64_t sm = side_of(m);
          int64_t aa[3] = {floor_to(na[0], sm), floor_to(na[1], sm), dim_ == 3 ? floor_to(na[2], sm) : 0};
          uint64_t k = key(m, aa, t);
          if (cells_.get(k) == kLeaf) {
            if (m >= kMaxLevel) fail(-1, "maximum level exceeded");
            Cell cc;
            cc.level = (int8_t)m;
            cc.tree = (int16_t)t;
            for (int i = 0; i < 3; ++i) cc.a[i] = (int32_t)aa[i];
            next.push_back({k, cc});
            break;
          }
        }
      }
    }
    std::sort(next.begin(), next.end(), [](const Leaf& x, const Leaf& y) { return x.key < y.key; });
    next.erase(std::unique(next.begin(), next.end(),
                           [](const Leaf& x, const Leaf& y) { return x.key == y.key; }),
               next.end());
    work.clear();
    for (auto& l : next) work.push_back(l.c);
  }
  std::vector<Leaf> out;
  out.reserve(leaves_.size() * 2);
  for (auto& l : leaves_) emit(l.c, out);
  leaves_.swap(out);
  return (int64_t)leaves_.size();
}

}  // namespace gmg
