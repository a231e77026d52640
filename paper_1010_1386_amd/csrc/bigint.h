// Minimal unsigned big integers for host-side planning: Hadamard bounds,
// prime products and CRT constants.  Little-endian 32-bit limbs, no leading
// zero limbs (zero is the empty vector).  Schoolbook arithmetic: operands
// here are at most a few tens of thousands of bits.
#pragma once
#include <cstdint>
#include <vector>
#include <algorithm>

namespace rsl {

struct BigU {
  std::vector<uint32_t> d;

  BigU() = default;
  explicit BigU(uint64_t v) {
    while (v) { d.push_back(static_cast<uint32_t>(v)); v >>= 32; }
  }
  bool is_zero() const { return d.empty(); }
  void trim() { while (!d.empty() && d.back() == 0) d.pop_back(); }

  int bitlen() const {
    if (d.empty()) return 0;
    return static_cast<int>(32 * (d.size() - 1)) + (32 - __builtin_clz(d.back()));
  }

  static int cmp(const BigU& a, const BigU& b) {
    if (a.d.size() != b.d.size()) return a.d.size() < b.d.size() ? -1 : 1;
    for (size_t i = a.d.size(); i-- > 0;)
      if (a.d[i] != b.d[i]) return a.d[i] < b.d[i] ? -1 : 1;
    return 0;
  }

  static BigU add(const BigU& a, const BigU& b) {
    BigU r;
    size_t n = std::max(a.d.size(), b.d.size());
    r.d.resize(n + 1);
    uint64_t c = 0;
    for (size_t i = 0; i < n; ++i) {
      c += (i < a.d.size() ? a.d[i] : 0u);
      c += (i < b.d.size() ? b.d[i] : 0u);
      r.d[i] = static_cast<uint32_t>(c);
      c >>= 32;
    }
    r.d[n] = static_cast<uint32_t>(c);
    r.trim();
    return r;
  }

  // a - b, requires a >= b
  static BigU sub(const BigU& a, const BigU& b) {
    BigU r;
    r.d.resize(a.d.size());
    int64_t br = 0;
    for (size_t i = 0; i < a.d.size(); ++i) {
      int64_t v = static_cast<int64_t>(a.d[i]) - (i < b.d.size() ? b.d[i] : 0u) - br;
      br = v < 0;
      r.d[i] = static_cast<uint32_t>(v + (br << 32));
    }
    r.trim();
    return r;
  }

  static BigU mul(const BigU& a, const BigU& b) {
    if (a.is_zero() || b.is_zero()) return BigU();
    BigU r;
    r.d.assign(a.d.size() + b.d.size(), 0);
    for (size_t i = 0; i < a.d.size(); ++i) {
      uint64_t c = 0, ai = a.d[i];
      for (size_t j = 0; j < b.d.size(); ++j) {
        c += ai * b.d[j] + r.d[i + j];
        r.d[i + j] = static_cast<uint32_t>(c);
        c >>= 32;
      }
      r.d[i + b.d.size()] = static_cast<uint32_t>(c);
    }
    r.trim();
    return r;
  }

  static BigU mul_small(const BigU& a, uint32_t m) {
    BigU r;
    r.d.resize(a.d.size() + 1);
    uint64_t c = 0;
    for (size_t i = 0; i < a.d.size(); ++i) {
      c += static_cast<uint64_t>(a.d[i]) * m;
      r.d[i] = static_cast<uint32_t>(c);
      c >>= 32;
    }
    r.d[a.d.size()] = static_cast<uint32_t>(c);
    r.trim();
    return r;
  }

  static BigU pow(BigU base, uint64_t e) {
    BigU r(1);
    while (e) {
      if (e & 1) r = mul(r, base);
      e >>= 1;
      if (e) base = mul(base, base);
    }
    return r;
  }

  // floor(a / m)
  BigU div_small(uint32_t m) const {
    BigU r;
    r.d.assign(d.size(), 0u);
    uint64_t rem = 0;
    for (size_t i = d.size(); i-- > 0;) {
      const uint64_t cur = (rem << 32) | d[i];
      r.d[i] = static_cast<uint32_t>(cur / m);
      rem = cur % m;
    }
    r.trim();
    return r;
  }

  uint32_t mod_small(uint32_t m) const {
    uint64_t r = 0;
    for (size_t i = d.size(); i-- > 0;) r = ((r << 32) | d[i]) % m;
    return static_cast<uint32_t>(r);
  }

  // floor(a / 2)
  BigU half() const {
    BigU r;
    r.d.resize(d.size());
    for (size_t i = 0; i < d.size(); ++i) {
      uint32_t hi = (i + 1 < d.size()) ? d[i + 1] : 0u;
      r.d[i] = (d[i] >> 1) | (hi << 31);
    }
    r.trim();
    return r;
  }

  // 2^(32 L) - a as exactly L limbs (requires a < 2^(32 L)); a = 0 gives 0.
  std::vector<uint32_t> neg_limbs(int L) const {
    std::vector<uint32_t> out(L, 0);
    uint64_t c = 1;
    for (int i = 0; i < L; ++i) {
      uint32_t v = (static_cast<size_t>(i) < d.size()) ? d[i] : 0u;
      c += static_cast<uint32_t>(~v);
      out[i] = static_cast<uint32_t>(c);
      c >>= 32;
    }
    return out;
  }

  // a >> k bits
  BigU shr(int k) const {
    BigU r;
    const int w = k / 32, b = k % 32;
    if (static_cast<size_t>(w) >= d.size()) return r;
    r.d.resize(d.size() - w);
    for (size_t i = 0; i < r.d.size(); ++i) {
      const uint64_t lo = d[i + w], hi = (i + w + 1 < d.size()) ? d[i + w + 1] : 0u;
      r.d[i] = static_cast<uint32_t>(((hi << 32) | lo) >> b);
    }
    while (!r.d.empty() && r.d.back() == 0u) r.d.pop_back();
    return r;
  }
  int ctz() const {  // trailing zero bits (0 for zero)
    for (size_t i = 0; i < d.size(); ++i)
      if (d[i]) return static_cast<int>(32 * i) + __builtin_ctz(d[i]);
    return 0;
  }
  // a << k bits
  BigU shl(int k) const {
    if (d.empty()) return BigU();
    BigU r;
    const int w = k / 32, b = k % 32;
    r.d.assign(d.size() + w + 1, 0u);
    for (size_t i = 0; i < d.size(); ++i) {
      const uint64_t v = static_cast<uint64_t>(d[i]) << b;
      r.d[i + w] |= static_cast<uint32_t>(v);
      r.d[i + w + 1] |= static_cast<uint32_t>(v >> 32);
    }
    while (!r.d.empty() && r.d.back() == 0u) r.d.pop_back();
    return r;
  }
  // greatest common divisor (binary algorithm; gcd(0, b) = b)
  static BigU gcd(BigU a, BigU b) {
    if (a.is_zero()) return b;
    if (b.is_zero()) return a;
    const int za = a.ctz(), zb = b.ctz(), z = za < zb ? za : zb;
    a = a.shr(za);
    b = b.shr(zb);
    while (!b.is_zero()) {  // both odd here
      if (cmp(a, b) > 0) { BigU t = a; a = b; b = t; }
      b = sub(b, a);
      if (!b.is_zero()) b = b.shr(b.ctz());
    }
    return a.shl(z);
  }

  std::vector<uint32_t> limbs(int L) const {
    std::vector<uint32_t> out(L, 0);
    for (int i = 0; i < L && static_cast<size_t>(i) < d.size(); ++i) out[i] = d[i];
    return out;
  }
};

// |v| of an L-limb two's complement integer, and its sign.
inline BigU abs_limbs(const uint32_t* w, int L, bool* neg) {
  bool n = (w[L - 1] >> 31) & 1u;
  BigU r;
  r.d.resize(L);
  if (!n) {
    for (int i = 0; i < L; ++i) r.d[i] = w[i];
  } else {
    uint64_t c = 1;
    for (int i = 0; i < L; ++i) {
      c += static_cast<uint32_t>(~w[i]);
      r.d[i] = static_cast<uint32_t>(c);
      c >>= 32;
    }
  }
  r.trim();
  if (neg) *neg = n && !r.is_zero();
  return r;
}

}  // namespace rsl
