// Total-degree coefficient layout.
//
// Every polynomial the path produces has total degree at most its
// per-variable degree D: layer-1 pre-activations are affine in t, the affine
// maps only add, an order-k approximant composed with a polynomial of total
// degree D has total degree k*D, and the linear fallback is affine. So of the
// (D+1)^n monomials t^J of a per-variable degree-D tensor only those with
// |J| = j_1 + ... + j_n <= D can be nonzero: S(n, D) = C(n+D, n) of them.
// Tensors are stored with exactly these coefficients.
//
// Order: graded by total degree (all |J| = 0, then |J| = 1, ...), and within
// one total degree by descending lexicographic exponent tuple. The monomials
// of total degree <= D' < D are then the first S(n, D') coefficients, so
// lifting a polynomial to a higher degree (Prop. 4 elevation) appends zeros,
// and a lower-degree tensor is read inside a higher-degree one by its prefix.
// Rank 0 is the constant; ranks 1..n are t_1..t_n.
//
// The basis change to Bernstein form still runs on the dense per-variable
// degree-D tensor in LDS (Def. 2 needs every tensor-product Bernstein
// coefficient); products run over index-pair tables. Both tables are built on
// the host once per (n, degrees) and kept on the device by the network.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace bern {

constexpr int kMaxTreeDims = 16;  // variables of a tree table (the input count limit)

// C(n + D, n), or -1 above `cap`.
int64_t ssize(int n, int D, int64_t cap = (int64_t)1 << 40);

// Exponent tuples of the S(n, D) monomials in layout order: [S][n].
std::vector<uint16_t> simplex_exponents(int n, int D);

// Layout rank of an exponent tuple of n digits (total degree any).
int64_t simplex_rank(int n, const uint16_t *e);

// Device tables of one product of a degree-da and a degree-db polynomial
// (output degree da + db): for output coefficient K, the input index pairs
// pairs[off[K] .. off[K+1]) with I + J = K. For a square (sym) only pairs
// with rank(I) < rank(J) are listed and diag[K] is the rank of K/2 (or -1).
struct ProdTable {
  int *off = nullptr;
  int2 *pairs = nullptr;
  int *diag = nullptr;
  int64_t npairs = 0;
};

// Child tables of the tree read-off (fixing the leading variable at a
// Bernstein index, one variable at a time). For every d = 2 .. n: the
// (d-1)-variable layout of degree D is the child of the d-variable one (the
// leading variable dropped); for each child coefficient r and j = 0 .. D-|r|
// the table lists the parent rank of (j, r). One int buffer; dimension d
// starts at base[d]: off[S(d-1) + 1] (absolute starts in the buffer), then
// the parent ranks, S(d) of them (each parent coefficient exactly once).
struct TreeTable {
  int base[kMaxTreeDims + 2] = {};
  int len = 0;
  int *buf = nullptr;
};

struct SimplexTables {
  int n = 0;
  std::mutex mu;
  std::map<int, int *> dense;                      // D -> [S(n,D)] index in the (D+1)^n tensor
  std::map<std::tuple<int, int, int>, ProdTable> prod;  // (da, db, sym)
  std::map<int, TreeTable> trees;  // D
  std::map<std::pair<int, int>, std::pair<int *, int>> prefixes;  // (D, na) -> (table, ints)
  ~SimplexTables();
};

// True while the calling thread runs an entry point that must not allocate
// (bern_bounds_noalloc): a table that is not built yet is then not built,
// and its builder returns hipErrorNotReady.
bool no_alloc_active();

// Largest number of index pairs a product table may hold.
constexpr int64_t kMaxPairs = (int64_t)1 << 25;

// Build (once) and return the tables; errors: hipErrorInvalidValue when a
// table would exceed its limit, or the allocation / copy error.
hipError_t dense_index_table(SimplexTables &t, int D, const int **out);
hipError_t product_table(SimplexTables &t, int da, int db, bool sym, const ProdTable **out);
hipError_t tree_table(SimplexTables &t, int D, const TreeTable **out);

// Valid fibre prefixes of the per-axis basis change of a tensor whose
// nonzero coefficients all have exponent sum <= D: converting axis a (axes
// after a already converted), a fibre is zero unless the exponents of the
// axes before a sum to at most D. Table of ints: off[0 .. na] (off[a] =
// start of the list for a leading axes, off[na] = end), then the lists: the
// dense indices (base D+1, a digits) of those leading exponents, ascending.
hipError_t prefix_table(SimplexTables &t, int D, int na, const int **out, int *len);

}  // namespace bern
