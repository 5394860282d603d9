// Shared host utilities: error type, thread-local last error, open-addressing
// hash tables keyed by 64- and 128-bit integers.
#pragma once
#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

namespace gmg {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }
void set_last_error(const std::string& msg);

using u128 = unsigned __int128;

inline uint64_t mix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  return x ^ (x >> 31);
}
inline uint64_t hash128(u128 k) {
  return mix64((uint64_t)k ^ mix64((uint64_t)(k >> 64)));
}

// u128 -> int32 map, values >= 0; linear probing; grows at 50% load.
class KeyMap {
 public:
  explicit KeyMap(size_t expect = 1024) { reset(expect); }
  void reset(size_t expect) {
    size_t cap = 16;
    while (cap < 2 * expect + 16) cap <<= 1;
    keys_.assign(cap, 0);
    vals_.assign(cap, -1);
    mask_ = cap - 1;
    size_ = 0;
  }
  size_t size() const { return size_; }
  // value for key, or -1
  int32_t get(u128 k) const {
    size_t i = hash128(k) & mask_;
    while (true) {
      int32_t v = vals_[i];
      if (v < 0) return -1;
      if (keys_[i] == k) return v;
      i = (i + 1) & mask_;
    }
  }
  // replace the value of a present key
  void set(u128 k, int32_t v) {
    size_t i = hash128(k) & mask_;
    while (vals_[i] >= 0 && keys_[i] != k) i = (i + 1) & mask_;
    if (vals_[i] < 0) fail(-8, "key map: key absent");
    vals_[i] = v;
  }
  // insert (k, v) if absent; returns the stored value
  int32_t get_or_insert(u128 k, int32_t v) {
    if (2 * (size_ + 1) > keys_.size()) grow();
    size_t i = hash128(k) & mask_;
    while (true) {
      int32_t cur = vals_[i];
      if (cur < 0) {
        keys_[i] = k;
        vals_[i] = v;
        ++size_;
        return v;
      }
      if (keys_[i] == k) return cur;
      i = (i + 1) & mask_;
    }
  }

 private:
  void grow() {
    std::vector<u128> ok;
    std::vector<int32_t> ov;
    ok.swap(keys_);
    ov.swap(vals_);
    size_t cap = ok.size() * 2;
    keys_.assign(cap, 0);
    vals_.assign(cap, -1);
    mask_ = cap - 1;
    size_ = 0;
    for (size_t i = 0; i < ok.size(); ++i)
      if (ov[i] >= 0) get_or_insert(ok[i], ov[i]);
  }
  std::vector<u128> keys_;
  std::vector<int32_t> vals_;
  size_t mask_ = 0, size_ = 0;
};

// KeyMap in 16 parts chosen by the top bits of the hash (the slot index uses
// the low bits), so that threads can fill the parts in parallel.
class PKeyMap {
 public:
  static constexpr int P = 16;
  static int part_of(u128 k) { return (int)(hash128(k) >> 60); }
  int32_t get(u128 k) const { return m_[part_of(k)].get(k); }
  KeyMap& part(int p) { return m_[p]; }
  void clear() {
    for (auto& m : m_) m = KeyMap(16);
  }

 private:
  std::vector<KeyMap> m_ = std::vector<KeyMap>(P, KeyMap(16));
};

// uint64 -> uint8 map (0 = absent), linear probing, grows at 50% load.
class CellMap {
 public:
  CellMap() { keys_.assign(1024, 0); vals_.assign(1024, 0); mask_ = 1023; }
  uint8_t get(uint64_t k) const {
    size_t i = mix64(k) & mask_;
    while (true) {
      uint8_t v = vals_[i];
      if (!v) return 0;
      if (keys_[i] == k) return v;
      i = (i + 1) & mask_;
    }
  }
  void set(uint64_t k, uint8_t v) {
    if (2 * (size_ + 1) > keys_.size()) grow();
    size_t i = mix64(k) & mask_;
    while (true) {
      if (!vals_[i]) {
        keys_[i] = k;
        vals_[i] = v;
        ++size_;
        return;
      }
      if (keys_[i] == k) {
        vals_[i] = v;
        return;
      }
      i = (i + 1) & mask_;
    }
  }
  size_t size() const { return size_; }

 private:
  void grow() {
    std::vector<uint64_t> ok;
    std::vector<uint8_t> ov;
    ok.swap(keys_);
    ov.swap(vals_);
    size_t cap = ok.size() * 2;
    keys_.assign(cap, 0);
    vals_.assign(cap, 0);
    mask_ = cap - 1;
    size_ = 0;
    for (size_t i = 0; i < ok.size(); ++i)
      if (ov[i]) set(ok[i], ov[i]);
  }
  std::vector<uint64_t> keys_;
  std::vector<uint8_t> vals_;
  size_t mask_, size_ = 0;
};

}  // namespace gmg
