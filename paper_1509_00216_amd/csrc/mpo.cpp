// MPO construction for H = sum h a+a + 1/2 sum (ij|kl) a+a+aa + sum u n_up n_dn + e_const
// (MPO equation of the Implementation section; bond dimension O(k^2) for two-body terms).
//
// Every operator string is sorted by site (fermionic sign of the permutation) and written
// as a product of site-local 4x4 matrices with Jordan-Wigner parity strings:
//   factor at site t = (string's operators at t, in order) * F^(#operators right of t),
//   F = diag(1,-1,-1,1).
// At MPO bond b (left of site b) a string with nL operators left of b and nR right of it
// travels in one channel:
//   nL = 0 -> "I"            nR = 0 -> "H"
//   nL < nR -> labelled by its left operators (coefficient not yet applied)
//   nL > nR -> labelled by its right operators (coefficient already applied)
//   nL = nR = 1 -> left label; nL = nR = 2 -> left label for b < switch, right label after.
// So channels hold at most two operators, which keeps D at about 2 + 4k + (2k)^2/2 at the
// centre instead of growing with the number of terms.  The coefficient is applied on the
// single transition from a left-labelled (or I) channel into a right-labelled (or H) one;
// all other transitions depend on the labels only.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "internal.h"

namespace lcc {
namespace {

// operator code: site * 4 + spin * 2 + dagger
inline int op_site(uint16_t c) { return c >> 2; }
inline int op_spin(uint16_t c) { return (c >> 1) & 1; }
inline int op_dag(uint16_t c) { return c & 1; }
inline uint16_t make_op(int site, int spin, int dag) { return (uint16_t)(site * 4 + spin * 2 + dag); }

struct Mat4 {
  double a[16];
};
inline Mat4 identity4() {
  Mat4 m{};
  for (int i = 0; i < 4; ++i) m.a[i * 4 + i] = 1.0;
  return m;
}
inline Mat4 mul4(const Mat4& x, const Mat4& y) {
  Mat4 r{};
  for (int i = 0; i < 4; ++i)
    for (int k = 0; k < 4; ++k) {
      const double v = x.a[i * 4 + k];
      if (v == 0.0) continue;
      for (int j = 0; j < 4; ++j) r.a[i * 4 + j] += v * y.a[k * 4 + j];
    }
  return r;
}
// local basis |0>, |up>, |dn>, |updn> with |updn> = c+_up c+_dn |0>
inline Mat4 local_matrix(int spin, int dag) {
  Mat4 m{};
  if (spin == 0) {  // c+_up: |0> -> |up>, |dn> -> |updn>
    m.a[1 * 4 + 0] = 1.0;
    m.a[3 * 4 + 2] = 1.0;
  } else {          // c+_dn: |0> -> |dn>, |up> -> -|updn>
    m.a[2 * 4 + 0] = 1.0;
    m.a[3 * 4 + 1] = -1.0;
  }
  if (!dag) {
    Mat4 t{};
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) t.a[i * 4 + j] = m.a[j * 4 + i];
    return t;
  }
  return m;
}
inline Mat4 parity4() {
  Mat4 m{};
  m.a[0] = 1.0;
  m.a[5] = -1.0;
  m.a[10] = -1.0;
  m.a[15] = 1.0;
  return m;
}
inline bool is_zero(const Mat4& m) {
  for (double v : m.a)
    if (v != 0.0) return false;
  return true;
}

struct Term {
  double coef;
  int n;                         // 2 or 4 operators (0 for the constant)
  std::array<uint16_t, 4> ops;   // sorted by site (stable)
};

// Label: kind (0 I, 1 H, 2 left, 3 right) | count | three 16-bit operator codes
inline uint64_t label_key(int kind, int count, const uint16_t* ops) {
  uint64_t k = (uint64_t)kind << 62 | (uint64_t)count << 60;
  for (int i = 0; i < count; ++i) k |= (uint64_t)(ops[i] + 1) << (16 * i);
  return k;
}
constexpr uint64_t kLabelI = 0;
constexpr uint64_t kLabelH = (uint64_t)1 << 62;
inline int label_kind(uint64_t k) { return (int)(k >> 62); }

struct Labeller {
  int sw;
  // number of operators strictly left of bond b
  static int n_left(const Term& t, int b) {
    int c = 0;
    for (int i = 0; i < t.n; ++i) c += op_site(t.ops[i]) < b;
    return c;
  }
  uint64_t at(const Term& t, int b) const {
    const int nl = n_left(t, b), nr = t.n - nl;
    if (nl == 0) return kLabelI;
    if (nr == 0) return kLabelH;
    bool left;
    if (nl < nr) left = true;
    else if (nl > nr) left = false;
    else if (nl == 1) left = true;
    else left = b < sw;
    if (left) return label_key(2, nl, t.ops.data());
    return label_key(3, nr, t.ops.data() + nl);
  }
};

QN label_dq(uint64_t key) {
  const int kind = label_kind(key);
  if (kind < 2) return QN(0, 0);
  const int count = (int)((key >> 60) & 3);
  int dn = 0, dz = 0;
  for (int i = 0; i < count; ++i) {
    const uint16_t c = (uint16_t)(((key >> (16 * i)) & 0xffff) - 1);
    const int s = op_dag(c) ? 1 : -1;
    dn += s;
    dz += s * (op_spin(c) == 0 ? 1 : -1);
  }
  // a right label carries the operators right of the bond; the left part carries the rest
  if (kind == 3) return QN(-dn, -dz);
  return QN(dn, dz);
}

// order of channels within a bond: I, H, left labels, right labels (each by key)
bool channel_less(uint64_t a, uint64_t b) {
  const int ka = label_kind(a), kb = label_kind(b);
  if (ka != kb) return ka < kb;
  return a < b;
}

}  // namespace

std::string build_mpo(const HamDesc& d, Mpo& out) {
  const int K = d.K;
  if (K < 2 || K > 64) return "n_orb must be in [2, 64]";
  // ---- operator strings, site-sorted with permutation sign
  std::vector<Term> terms;
  // Partition (Theory section, partitioned Hamiltonian): H0 keeps the terms that move no
  // electron between the orbital classes (every class has as many creators as annihilators),
  // U the others.
  auto in_part = [&](std::initializer_list<uint16_t> ops) {
    if (d.part == 0) return true;
    int bal[3] = {0, 0, 0};
    for (uint16_t o : ops) bal[d.orb_class[op_site(o)]] += op_dag(o) ? 1 : -1;
    const bool keeps = bal[0] == 0 && bal[1] == 0 && bal[2] == 0;
    return d.part == 1 ? keeps : !keeps;
  };
  auto push = [&](double coef, std::initializer_list<uint16_t> ops) {
    if (coef == 0.0 || !in_part(ops)) return;
    Term t;
    t.coef = coef;
    t.n = (int)ops.size();
    int i = 0;
    for (uint16_t o : ops) t.ops[i++] = o;
    // stable insertion sort by site, counting transpositions
    int swaps = 0;
    for (int a = 1; a < t.n; ++a)
      for (int b = a; b > 0 && op_site(t.ops[b - 1]) > op_site(t.ops[b]); --b) {
        std::swap(t.ops[b - 1], t.ops[b]);
        ++swaps;
      }
    if (swaps & 1) t.coef = -t.coef;
    // drop strings that vanish on a site (e.g. a+_p a+_p)
    for (int a = 0; a < t.n;) {
      int b = a;
      Mat4 m = identity4();
      while (b < t.n && op_site(t.ops[b]) == op_site(t.ops[a])) {
        m = mul4(m, local_matrix(op_spin(t.ops[b]), op_dag(t.ops[b])));
        ++b;
      }
      if (is_zero(m)) return;
      a = b;
    }
    terms.push_back(t);
  };
  for (int i = 0; i < K; ++i)
    for (int j = 0; j < K; ++j) {
      const double v = d.h[(size_t)i * K + j];
      for (int s = 0; s < 2; ++s) push(v, {make_op(i, s, 1), make_op(j, s, 0)});
    }
  if (!d.u.empty())
    for (int i = 0; i < K; ++i)
      push(d.u[i], {make_op(i, 0, 1), make_op(i, 0, 0), make_op(i, 1, 1), make_op(i, 1, 0)});
  if (!d.eri.empty()) {
    const size_t K2 = (size_t)K * K, K3 = K2 * K;
    for (int i = 0; i < K; ++i)
      for (int j = 0; j < K; ++j)
        for (int k = 0; k < K; ++k)
          for (int l = 0; l < K; ++l) {
            const double v = d.eri[i * K3 + j * K2 + k * (size_t)K + l];
            if (v == 0.0) continue;
            for (int s = 0; s < 2; ++s)
              for (int t = 0; t < 2; ++t) {
                if (i == k && s == t) continue;
                if (l == j && t == s) continue;
                push(0.5 * v, {make_op(i, s, 1), make_op(k, t, 1), make_op(l, t, 0), make_op(j, s, 0)});
              }
          }
  }
  const int sw = d.switch_bond >= 0 ? d.switch_bond : K / 2 + 1;
  Labeller lab{sw};

  // ---- pass 1: channel ranges (a channel lives on a contiguous range of bonds)
  std::unordered_map<uint64_t, std::pair<int, int>> range;
  range.reserve(1 << 16);
  auto touch = [&](uint64_t key, int b0, int b1) {
    auto it = range.find(key);
    if (it == range.end()) range.emplace(key, std::make_pair(b0, b1));
    else {
      it->second.first = std::min(it->second.first, b0);
      it->second.second = std::max(it->second.second, b1);
    }
  };
  // break points of a term: bonds where its label may change
  auto breakpoints = [&](const Term& t, int* bp) {
    int n = 0;
    bp[n++] = 0;
    for (int i = 0; i < t.n; ++i) bp[n++] = op_site(t.ops[i]) + 1;
    bp[n++] = sw;
    bp[n++] = K + 1;
    std::sort(bp, bp + n);
    int m = 0;
    for (int i = 0; i < n; ++i)
      if (bp[i] <= K + 1 && (m == 0 || bp[m - 1] != bp[i])) bp[m++] = bp[i];
    return m;
  };
  for (const Term& t : terms) {
    int bp[8];
    const int nb = breakpoints(t, bp);
    for (int i = 0; i + 1 < nb; ++i) {
      const int b0 = bp[i], b1 = std::min(bp[i + 1] - 1, K);
      if (b0 > K) break;
      touch(lab.at(t, b0), b0, b1);
    }
  }
  const double e_const = d.part == 2 ? 0.0 : d.e_const;  // the constant belongs to H0
  if (e_const != 0.0) {
    touch(kLabelI, 0, 0);
    touch(kLabelH, 1, K);
  }
  // ---- channel indices per bond
  std::vector<std::vector<uint64_t>> chans(K + 1);
  for (const auto& kv : range)
    for (int b = kv.second.first; b <= kv.second.second; ++b) chans[b].push_back(kv.first);
  std::vector<std::unordered_map<uint64_t, int>> index(K + 1);
  out.K = K;
  out.dq.assign(K + 1, {});
  out.kind.assign(K + 1, {});
  for (int b = 0; b <= K; ++b) {
    std::sort(chans[b].begin(), chans[b].end(), channel_less);
    index[b].reserve(chans[b].size() * 2);
    for (size_t i = 0; i < chans[b].size(); ++i) {
      index[b][chans[b][i]] = (int)i;
      out.dq[b].push_back(label_dq(chans[b][i]));
      out.kind[b].push_back((int8_t)label_kind(chans[b][i]));
    }
  }
  if (chans[0].size() != 1 || chans[K].size() != 1) return "internal: boundary bonds must hold one channel";

  // ---- pass 2: entries
  out.W.assign(K, {});
  std::vector<std::unordered_map<uint64_t, size_t>> where(K);
  const Mat4 F = parity4();
  auto entry = [&](int site, int a, int b) -> MpoEntry& {
    const uint64_t key = (uint64_t)a << 32 | (uint32_t)b;
    auto it = where[site].find(key);
    if (it != where[site].end()) return out.W[site][it->second];
    where[site].emplace(key, out.W[site].size());
    MpoEntry e;
    e.win = a;
    e.wout = b;
    std::memset(e.m, 0, sizeof(e.m));
    out.W[site].push_back(e);
    return out.W[site].back();
  };
  std::string err;
  for (const Term& t : terms) {
    // event sites: sites holding operators and the site just left of the switch bond
    int ev[6], ne = 0;
    for (int i = 0; i < t.n; ++i) {
      const int s = op_site(t.ops[i]);
      if (ne == 0 || ev[ne - 1] != s) ev[ne++] = s;
    }
    if (sw - 1 >= 0 && sw - 1 < K) {
      bool have = false;
      for (int i = 0; i < ne; ++i) have |= ev[i] == sw - 1;
      if (!have) ev[ne++] = sw - 1;
    }
    for (int e = 0; e < ne; ++e) {
      const int j = ev[e];
      const uint64_t lin = lab.at(t, j), lout = lab.at(t, j + 1);
      const bool has_op = [&] {
        for (int i = 0; i < t.n; ++i)
          if (op_site(t.ops[i]) == j) return true;
        return false;
      }();
      if (!has_op && lin == lout) continue;  // plain pass-through, added below
      Mat4 m = identity4();
      int after = 0;
      for (int i = 0; i < t.n; ++i) {
        if (op_site(t.ops[i]) == j) m = mul4(m, local_matrix(op_spin(t.ops[i]), op_dag(t.ops[i])));
        after += op_site(t.ops[i]) > j;
      }
      if (after & 1) m = mul4(m, F);
      const int kin = label_kind(lin), kout = label_kind(lout);
      const bool applies_coef = (kin == 0 || kin == 2) && (kout == 1 || kout == 3);
      MpoEntry& w = entry(j, index[j].at(lin), index[j + 1].at(lout));
      if (applies_coef) {
        for (int q = 0; q < 16; ++q) w.m[q] += t.coef * m.a[q];
      } else {
        bool fresh = true;
        for (int q = 0; q < 16; ++q) fresh &= w.m[q] == 0.0;
        if (!fresh) {
          for (int q = 0; q < 16; ++q)
            if (w.m[q] != m.a[q]) err = "internal: inconsistent label transition";
        }
        std::memcpy(w.m, m.a, sizeof(w.m));
      }
    }
  }
  if (!err.empty()) return err;
  if (e_const != 0.0) {
    MpoEntry& w = entry(0, index[0].at(kLabelI), index[1].at(kLabelH));
    for (int q = 0; q < 4; ++q) w.m[q * 4 + q] += e_const;
  }
  // pass-through of every channel across the sites inside its range
  for (const auto& kv : range) {
    const uint64_t key = kv.first;
    const int kind = label_kind(key);
    const int count = (int)((key >> 60) & 3);
    const bool odd = (kind >= 2) && (count & 1);
    for (int b = kv.second.first; b < kv.second.second; ++b) {
      MpoEntry& w = entry(b, index[b].at(key), index[b + 1].at(key));
      const Mat4 m = odd ? F : identity4();
      std::memcpy(w.m, m.a, sizeof(w.m));
    }
  }
  // drop entries that cancelled to zero
  for (int j = 0; j < K; ++j) {
    auto& v = out.W[j];
    v.erase(std::remove_if(v.begin(), v.end(), [](const MpoEntry& e) {
              for (double x : e.m)
                if (x != 0.0) return false;
              return true;
            }),
            v.end());
  }
  return "";
}

}  // namespace lcc
