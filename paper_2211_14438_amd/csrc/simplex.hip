// Host-side index tables of the total-degree coefficient layout.
#include "simplex.hpp"
#include "common.hpp"

#include <algorithm>

namespace bern {

static int64_t binom64(int64_t n, int64_t k) {
  if (k < 0 || n < 0 || k > n) return 0;
  if (k > n - k) k = n - k;
  int64_t r = 1;
  for (int64_t i = 1; i <= k; ++i) r = r * (n - k + i) / i;  // exact at every step
  return r;
}

int64_t ssize(int n, int D, int64_t cap) {
  if (D < 0) return 0;
  // C(n + D, n) = prod_{i=1..k} (n + D - k + i) / i, k = min(n, D); every
  // partial product is itself a binomial coefficient, so the division is
  // exact, and r <= cap < 2^41 keeps r * f far from overflow
  int64_t r = 1;
  const int k = std::min(n, D);
  for (int i = 1; i <= k; ++i) {
    r = r * ((int64_t)n + D - k + i) / i;
    if (r > cap) return -1;
  }
  return r;
}

static void enum_degree(int n, int d, int pos, std::vector<uint16_t> &cur, std::vector<uint16_t> &out) {
  if (pos == n - 1) {
    cur[pos] = (uint16_t)d;
    out.insert(out.end(), cur.begin(), cur.end());
    return;
  }
  for (int v = d; v >= 0; --v) {  // descending lexicographic
    cur[pos] = (uint16_t)v;
    enum_degree(n, d - v, pos + 1, cur, out);
  }
}

std::vector<uint16_t> simplex_exponents(int n, int D) {
  std::vector<uint16_t> out, cur(n, 0);
  for (int d = 0; d <= D; ++d) enum_degree(n, d, 0, cur, out);
  return out;
}

int64_t simplex_rank(int n, const uint16_t *e) {
  int d = 0;
  for (int i = 0; i < n; ++i) d += e[i];
  int64_t r = d > 0 ? binom64(n + d - 1, n) : 0;  // all monomials of total degree < d
  int rem = d;
  for (int i = 0; i + 1 < n; ++i) {
    const int m = n - 2 - i;  // digits after position i, minus the last
    for (int v = e[i] + 1; v <= rem; ++v) r += binom64(rem - v + m, m);
    rem -= e[i];
  }
  return r;
}

SimplexTables::~SimplexTables() {
  for (auto &kv : dense) (void)hipFree(kv.second);
  for (auto &kv : prod) {
    (void)hipFree(kv.second.off);
    (void)hipFree(kv.second.pairs);
    (void)hipFree(kv.second.diag);
  }
  for (auto &kv : prefixes) (void)hipFree(kv.second.first);
  for (auto &kv : trees) (void)hipFree(kv.second.buf);
}

hipError_t tree_table(SimplexTables &t, int D, const TreeTable **out) {
  std::lock_guard<std::mutex> g(t.mu);
  auto it = t.trees.find(D);
  if (it != t.trees.end()) {
    *out = &it->second;
    return hipSuccess;
  }
  if (no_alloc_active()) return hipErrorNotReady;
  const int n = t.n;
  if (D < 1 || D > 15 || n < 2 || n > kMaxTreeDims) return hipErrorInvalidValue;
  if (ssize(n, D, (int64_t)1 << 24) < 0) return hipErrorInvalidValue;
  TreeTable tt;
  std::vector<int> buf;
  for (int d = 2; d <= n; ++d) {
    const std::vector<uint16_t> ec = simplex_exponents(d - 1, D);
    const int64_t Sc = ssize(d - 1, D);
    tt.base[d] = (int)buf.size();
    const size_t off0 = buf.size();
    buf.resize(buf.size() + (size_t)Sc + 1);
    std::vector<uint16_t> tup((size_t)d);
    for (int64_t r = 0; r < Sc; ++r) {
      buf[off0 + (size_t)r] = (int)buf.size();
      int deg = 0;
      for (int a = 0; a < d - 1; ++a) {
        tup[(size_t)a + 1] = ec[(size_t)(r * (d - 1) + a)];
        deg += tup[(size_t)a + 1];
      }
      for (int j = 0; j + deg <= D; ++j) {
        tup[0] = (uint16_t)j;
        buf.push_back((int)simplex_rank(d, tup.data()));
      }
    }
    buf[off0 + (size_t)Sc] = (int)buf.size();
  }
  tt.len = (int)buf.size();
  hipError_t err = hipMalloc(&tt.buf, buf.size() * sizeof(int));
  if (err == hipSuccess) err = hipMemcpy(tt.buf, buf.data(), buf.size() * sizeof(int), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(tt.buf);
    return err;
  }
  auto res = t.trees.emplace(D, tt);
  *out = &res.first->second;
  return hipSuccess;
}

hipError_t dense_index_table(SimplexTables &t, int D, const int **out) {
  std::lock_guard<std::mutex> g(t.mu);
  auto it = t.dense.find(D);
  if (it != t.dense.end()) {
    *out = it->second;
    return hipSuccess;
  }
  if (no_alloc_active()) return hipErrorNotReady;
  const int n = t.n;
  const int64_t S = ssize(n, D, (int64_t)1 << 31);
  if (S < 0) return hipErrorInvalidValue;
  double dense = 1.0;
  for (int a = 0; a < n; ++a) dense *= D + 1;
  if (dense > 2147483647.0) return hipErrorInvalidValue;
  const std::vector<uint16_t> e = simplex_exponents(n, D);
  std::vector<int> idx(S);
  for (int64_t r = 0; r < S; ++r) {
    int64_t v = 0;
    for (int a = 0; a < n; ++a) v = v * (D + 1) + e[r * n + a];
    idx[r] = (int)v;
  }
  int *d = nullptr;
  RET_IF(hipMalloc(&d, S * sizeof(int)));
  hipError_t err = hipMemcpy(d, idx.data(), S * sizeof(int), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(d);
    return err;
  }
  t.dense[D] = d;
  *out = d;
  return hipSuccess;
}

hipError_t product_table(SimplexTables &t, int da, int db, bool sym, const ProdTable **out) {
  std::lock_guard<std::mutex> g(t.mu);
  const auto key = std::make_tuple(da, db, sym ? 1 : 0);
  auto it = t.prod.find(key);
  if (it != t.prod.end()) {
    *out = &it->second;
    return hipSuccess;
  }
  if (no_alloc_active()) return hipErrorNotReady;
  if (sym && da != db) return hipErrorInvalidValue;
  const int n = t.n;
  const int64_t Sa = ssize(n, da, (int64_t)1 << 31), Sb = ssize(n, db, (int64_t)1 << 31);
  const int64_t Sc = ssize(n, da + db, (int64_t)1 << 31);
  if (Sa < 0 || Sb < 0 || Sc < 0 || (sym ? Sa * (Sa - 1) / 2 : Sa * Sb) > kMaxPairs) return hipErrorInvalidValue;
  const std::vector<uint16_t> ea = simplex_exponents(n, da), eb = simplex_exponents(n, db);
  std::vector<int64_t> cnt(Sc + 1, 0);
  std::vector<int> diag(sym ? Sc : 0, -1);
  std::vector<uint16_t> k(n);
  std::vector<int> rk((size_t)Sa * (size_t)Sb, -1);  // output rank of every listed pair
  for (int64_t i = 0; i < Sa; ++i) {
    for (int64_t j = sym ? i : 0; j < Sb; ++j) {
      for (int q = 0; q < n; ++q) k[q] = (uint16_t)(ea[i * n + q] + eb[j * n + q]);
      const int64_t r = simplex_rank(n, k.data());
      if (sym && i == j) {
        diag[r] = (int)i;
        continue;
      }
      rk[(size_t)i * Sb + j] = (int)r;
      ++cnt[r + 1];
    }
  }
  for (int64_t r = 0; r < Sc; ++r) cnt[r + 1] += cnt[r];
  const int64_t P = cnt[Sc];
  std::vector<int> off(Sc + 1);
  for (int64_t r = 0; r <= Sc; ++r) off[r] = (int)cnt[r];
  std::vector<int2> pairs(std::max<int64_t>(P, 1));
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t i = 0; i < Sa; ++i)
    for (int64_t j = sym ? i + 1 : 0; j < Sb; ++j) {
      const int r = rk[(size_t)i * Sb + j];
      pairs[fill[r]++] = make_int2((int)i, (int)j);
    }
  ProdTable pt;
  pt.npairs = P;
  hipError_t err = hipMalloc(&pt.off, (Sc + 1) * sizeof(int));
  if (err == hipSuccess) err = hipMalloc(&pt.pairs, pairs.size() * sizeof(int2));
  if (err == hipSuccess && sym) err = hipMalloc(&pt.diag, Sc * sizeof(int));
  if (err == hipSuccess) err = hipMemcpy(pt.off, off.data(), (Sc + 1) * sizeof(int), hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipMemcpy(pt.pairs, pairs.data(), pairs.size() * sizeof(int2), hipMemcpyHostToDevice);
  if (err == hipSuccess && sym) err = hipMemcpy(pt.diag, diag.data(), Sc * sizeof(int), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(pt.off);
    (void)hipFree(pt.pairs);
    (void)hipFree(pt.diag);
    return err;
  }
  auto res = t.prod.emplace(key, pt);
  *out = &res.first->second;
  return hipSuccess;
}

hipError_t prefix_table(SimplexTables &t, int D, int na, const int **out, int *len) {
  std::lock_guard<std::mutex> g(t.mu);
  const auto key = std::make_pair(D, na);
  auto it = t.prefixes.find(key);
  if (it != t.prefixes.end()) {
    *out = it->second.first;
    *len = it->second.second;
    return hipSuccess;
  }
  if (no_alloc_active()) return hipErrorNotReady;
  if (na < 1 || D < 0) return hipErrorInvalidValue;
  std::vector<int> off(na + 1), vals;
  for (int a = 0; a < na; ++a) {
    off[a] = (int)vals.size();
    double lim = 1.0;
    for (int q = 0; q < a; ++q) lim *= D + 1;
    if (lim > 1e7) return hipErrorInvalidValue;
    for (int64_t v = 0; v < (int64_t)lim; ++v) {
      int64_t r = v;
      int sum = 0;
      for (int q = 0; q < a; ++q) {
        sum += (int)(r % (D + 1));
        r /= D + 1;
      }
      if (sum <= D) vals.push_back((int)v);
    }
  }
  off[na] = (int)vals.size();
  std::vector<int> all(off);
  for (size_t q = 0; q < all.size(); ++q) all[q] += na + 1;  // offsets into the whole table
  all.insert(all.end(), vals.begin(), vals.end());
  int *d = nullptr;
  RET_IF(hipMalloc(&d, all.size() * sizeof(int)));
  hipError_t err = hipMemcpy(d, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(d);
    return err;
  }
  t.prefixes[key] = std::make_pair(d, (int)all.size());
  *out = d;
  *len = (int)all.size();
  return hipSuccess;
}

}  // namespace bern
