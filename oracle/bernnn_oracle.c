/*
 * BERN-NN bound propagation: plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT. Only the test suite, the
 * smoke entry point and the benchmark's CPU-baseline leg may load this file's
 * library. It shares no code, header, table or helper with the HIP library:
 * the two are written independently from the paper and meet only in the tests.
 *
 * Representation: the paper's own one. A polynomial in n variables over the
 * input box, of per-variable degree d, is the tensor of its (d+1)^n Bernstein
 * coefficients (Section 4.1, "Ten(B_{g,L})", Example 1), last variable
 * fastest. Every step is the paper's definition, written out plainly:
 *   Def. 1, eqs. (bernpol)-(bernpolcoeff2)   Bernstein polynomial of g on a box
 *   Def. 2, eq. (range_enclosing_property)   bounds = min / max coefficient
 *   Prop. 3, eqs. (scaled_bern_tensor1)-(prod_original_bern)
 *                                            Prod_Bern: scale by C_L, Prod, unscale
 *   Section 4.2 (after Prop. 3)              Pow_Bern: repeated Prod_Bern
 *   Prop. 4, eqs. (L_sum)-(tensor_sum)       Sum_Bern: elevate with a ones tensor, add
 *   Section 5.1, Steps 1-3                   one neuron
 *   Section 5.2, eqs. (upper_bounds_layer), (lower_bounds_layer)   one layer
 *   Section 5.3                              input initialisation and the layer loop
 *
 * Readings of points the paper leaves open (each one is listed with its reason
 * in the design notes of the repository):
 *   R1  bounds of a pre-activation are read at the degree the tensor carries
 *       (1, L, L^2, ... in the plain rule), never re-elevated;
 *   R2  the bias "+ b" of the layer equations is added to every Bernstein
 *       coefficient (Bernstein basis functions sum to one);
 *   R3  "*" with the weight matrices in the layer equations is the contraction
 *       over the neurons of the previous layer;
 *   R4  stable neurons: hi <= 0 gives the zero polynomial (checked first),
 *       lo >= 0 gives the identity; only lo < 0 < hi uses the approximant;
 *   R5  the power series of Step 2 is taken in u = (y - lo)/(hi - lo) in [0,1];
 *   R6  the under-approximant is the same series composed with the lower
 *       polynomial, shifted down by its value at y = 0 (Prop. 2);
 *   R7  plain rule: every neuron of hidden layer i is stored at degree L*D_i
 *       (Section 5.4, elevation to the highest expected degree);
 *   R8  given per-neuron plans: unstable neuron with code c >= 1 uses a
 *       degree-c approximant (degree c*D), active neuron keeps degree D,
 *       inactive neuron is the zero polynomial (degree 0), code 0 is the
 *       linear fallback (degree 1); all neurons of a layer are then elevated
 *       to the largest of these degrees (Prop. 4);
 *   R9  linear fallback: the degree-1 approximant's post polynomials, replaced
 *       by their least-squares affine fit to the Bernstein control net plus the
 *       largest (upper) or smallest (lower) remainder coefficient; sound by
 *       Def. 2 for any affine function;
 *   R13 periodic linearisation Lin (Section 5.4: the post polynomials are
 *       dropped to degree (1,...,1) every Lin hidden layers; the cited
 *       linearisation is not given): after every hidden layer whose index
 *       (1-based) is a multiple of Lin, each neuron's stored post polynomials
 *       (at the layer's degree, after the elevation of R7/R8) are replaced by
 *       the R9 construction -- least-squares affine fit of the Bernstein
 *       control net plus the extreme remainder -- so the next layer starts
 *       at degree 1. Lin = 0 switches it off (the paper's experiments).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_BOX (-3)
#define ORC_E_DEGREE (-4)
#define ORC_E_TOO_LARGE (-5)
#define ORC_E_OOM (-6)

/* ---------------------------------------------------------------- helpers */

/* Binomial coefficient C(n, k) (notation of Section 2.1), exact in FP64 for
 * the degrees used here. */
double orc_binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  if (k > n - k) k = n - k;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = nearbyint(r * (double)(n - k + i) / (double)i);
  return r;
}

/* Number of coefficients (d+1)^n of a hypercube tensor; -1 on overflow. */
long long orc_tsize(int n, int d) {
  long long s = 1;
  for (int a = 0; a < n; ++a) {
    if (s > (long long)4e15 / (d + 1)) return -1;
    s *= (d + 1);
  }
  return s;
}

/* Multi-index K of flat position idx (last variable fastest). */
static void digits(long long idx, int n, int d, int *k) {
  for (int a = n - 1; a >= 0; --a) {
    k[a] = (int)(idx % (d + 1));
    idx /= (d + 1);
  }
}

/* C_d tensor of Prop. 3: (C_d)_K = prod_a C(d, k_a). */
static void binom_tensor(int n, int d, double *out) {
  long long c = orc_tsize(n, d);
  int k[16];
  for (long long i = 0; i < c; ++i) {
    digits(i, n, d, k);
    double v = 1.0;
    for (int a = 0; a < n; ++a) v *= orc_binom(d, k[a]);
    out[i] = v;
  }
}

/* ----------------------------------------------- Section 4 tensor algebra */

/* Prod (Section 4.2): power-series product of two polynomials given by their
 * coefficient tensors, i.e. out_K = sum_{I+J=K} A_I B_J (an n-d convolution).
 * The output has per-variable degree da+db. */
int orc_prod(int n, int da, const double *A, int db, const double *B, double *out) {
  int dout = da + db;
  long long ca = orc_tsize(n, da), cb = orc_tsize(n, db), co = orc_tsize(n, dout);
  if (ca < 0 || cb < 0 || co < 0) return ORC_E_TOO_LARGE;
  long long *offA = (long long *)malloc(sizeof(long long) * (size_t)ca);
  long long *offB = (long long *)malloc(sizeof(long long) * (size_t)cb);
  if (!offA || !offB) { free(offA); free(offB); return ORC_E_OOM; }
  int k[16];
  /* position of I+J in the output tensor = position of I + position of J,
   * both written with the output's per-variable stride (dout+1). */
  for (long long i = 0; i < ca; ++i) {
    digits(i, n, da, k);
    long long o = 0;
    for (int a = 0; a < n; ++a) o = o * (dout + 1) + k[a];
    offA[i] = o;
  }
  for (long long j = 0; j < cb; ++j) {
    digits(j, n, db, k);
    long long o = 0;
    for (int a = 0; a < n; ++a) o = o * (dout + 1) + k[a];
    offB[j] = o;
  }
  memset(out, 0, sizeof(double) * (size_t)co);
  for (long long i = 0; i < ca; ++i)
    for (long long j = 0; j < cb; ++j) out[offA[i] + offB[j]] += A[i] * B[j];
  free(offA);
  free(offB);
  return ORC_OK;
}

/* Prod_Bern, Prop. 3: Bernstein tensors A (degree da) and B (degree db) ->
 * Bernstein tensor of the product at degree da+db:
 *   A~ = A * C_da, B~ = B * C_db, out = Prod(A~, B~) * (1 / C_{da+db}). */
int orc_prod_bern(int n, int da, const double *A, int db, const double *B, double *out) {
  long long ca = orc_tsize(n, da), cb = orc_tsize(n, db), co = orc_tsize(n, da + db);
  if (ca < 0 || cb < 0 || co < 0) return ORC_E_TOO_LARGE;
  double *As = (double *)malloc(sizeof(double) * (size_t)ca);
  double *Bs = (double *)malloc(sizeof(double) * (size_t)cb);
  double *Cs = (double *)malloc(sizeof(double) * (size_t)(ca > cb ? (ca > co ? ca : co) : (cb > co ? cb : co)));
  if (!As || !Bs || !Cs) { free(As); free(Bs); free(Cs); return ORC_E_OOM; }
  binom_tensor(n, da, Cs);
  for (long long i = 0; i < ca; ++i) As[i] = A[i] * Cs[i];
  binom_tensor(n, db, Cs);
  for (long long i = 0; i < cb; ++i) Bs[i] = B[i] * Cs[i];
  int st = orc_prod(n, da, As, db, Bs, out);
  if (st == ORC_OK) {
    binom_tensor(n, da + db, Cs);
    for (long long i = 0; i < co; ++i) out[i] = out[i] / Cs[i];
  }
  free(As); free(Bs); free(Cs);
  return st;
}

/* Degree elevation, Prop. 4 eqs. (degree_elevation_1/2): Prod_Bern of A
 * (degree d) with the ones tensor of degree e-d. */
int orc_elevate(int n, int d, const double *A, int e, double *out) {
  if (e < d) return ORC_E_DEGREE;
  long long cd = orc_tsize(n, d);
  if (cd < 0) return ORC_E_TOO_LARGE;
  if (e == d) { memcpy(out, A, sizeof(double) * (size_t)cd); return ORC_OK; }
  long long c1 = orc_tsize(n, e - d);
  if (c1 < 0) return ORC_E_TOO_LARGE;
  double *ones = (double *)malloc(sizeof(double) * (size_t)c1);
  if (!ones) return ORC_E_OOM;
  for (long long i = 0; i < c1; ++i) ones[i] = 1.0;
  int st = orc_prod_bern(n, d, A, e - d, ones, out);
  free(ones);
  return st;
}

/* Pow_Bern (Section 4.2): the i-th power of A (degree d) as a Bernstein
 * tensor of degree i*d, by repeated Prod_Bern. i = 0 gives the constant 1
 * at degree 0. */
int orc_pow_bern(int n, int d, const double *A, int i, double *out) {
  if (i < 0) return ORC_E_DEGREE;
  if (i == 0) { out[0] = 1.0; return ORC_OK; }
  long long cmax = orc_tsize(n, i * d);
  if (cmax < 0) return ORC_E_TOO_LARGE;
  long long cd = orc_tsize(n, d);
  memcpy(out, A, sizeof(double) * (size_t)cd);
  if (i == 1) return ORC_OK;
  double *tmp = (double *)malloc(sizeof(double) * (size_t)cmax);
  if (!tmp) return ORC_E_OOM;
  int st = ORC_OK;
  for (int p = 2; p <= i && st == ORC_OK; ++p) {
    st = orc_prod_bern(n, (p - 1) * d, out, d, A, tmp);
    memcpy(out, tmp, sizeof(double) * (size_t)orc_tsize(n, p * d));
  }
  free(tmp);
  return st;
}

/* Sum_Bern, Prop. 4: out (degree max(da,db)) = A + B after elevating both. */
int orc_sum_bern(int n, int da, const double *A, int db, const double *B, double *out) {
  int ds = da > db ? da : db;
  long long cs = orc_tsize(n, ds);
  if (cs < 0) return ORC_E_TOO_LARGE;
  double *ea = (double *)malloc(sizeof(double) * (size_t)cs);
  double *eb = (double *)malloc(sizeof(double) * (size_t)cs);
  if (!ea || !eb) { free(ea); free(eb); return ORC_E_OOM; }
  int st = orc_elevate(n, da, A, ds, ea);
  if (st == ORC_OK) st = orc_elevate(n, db, B, ds, eb);
  if (st == ORC_OK)
    for (long long i = 0; i < cs; ++i) out[i] = ea[i] + eb[i];
  free(ea); free(eb);
  return st;
}

/* Value of a Bernstein tensor at t in [0,1]^n: eq. (bernpol) with the basis
 * of eq. (bernpolcoeff) written in the box-normalised coordinate t. */
double orc_bern_eval(int n, int d, const double *B, const double *t) {
  long long c = orc_tsize(n, d);
  int k[16];
  double s = 0.0;
  for (long long i = 0; i < c; ++i) {
    digits(i, n, d, k);
    double v = B[i];
    for (int a = 0; a < n; ++a)
      v *= orc_binom(d, k[a]) * pow(t[a], k[a]) * pow(1.0 - t[a], d - k[a]);
    s += v;
  }
  return s;
}

/* Power (monomial, in t) coefficients -> Bernstein coefficients at degree d:
 * the textbook identity t^j = sum_{k>=j} C(k,j)/C(d,j) Ber_{k,d}(t), applied
 * along every variable. Used by the tests to check the GPU's basis change. */
int orc_power_to_bern(int n, int d, const double *a, double *b) {
  long long c = orc_tsize(n, d);
  if (c < 0) return ORC_E_TOO_LARGE;
  double *cur = (double *)malloc(sizeof(double) * (size_t)c);
  if (!cur) return ORC_E_OOM;
  memcpy(cur, a, sizeof(double) * (size_t)c);
  long long stride = 1;
  for (int ax = n - 1; ax >= 0; --ax) {
    /* fibres along variable ax: index = outer*(d+1)*stride + k*stride + inner */
    long long outer = c / ((long long)(d + 1) * stride);
    for (long long o = 0; o < outer; ++o)
      for (long long in = 0; in < stride; ++in) {
        long long base = o * (d + 1) * stride + in;
        for (int k = 0; k <= d; ++k) {
          double s = 0.0;
          for (int j = 0; j <= k; ++j)
            s += orc_binom(k, j) / orc_binom(d, j) * cur[base + (long long)j * stride];
          b[base + (long long)k * stride] = s;
        }
      }
    memcpy(cur, b, sizeof(double) * (size_t)c);
    stride *= (d + 1);
  }
  memcpy(b, cur, sizeof(double) * (size_t)c);
  free(cur);
  return ORC_OK;
}

/* ------------------------------------------------ Section 3: ReLU approximant */

/* Bernstein coefficients of sigma = ReLU on [lo, hi], eq. (bernpolcoeff2):
 * b_k = sigma(lo + (hi - lo) k / L), k = 0..L. */
void orc_relu_bern_coefs(double lo, double hi, int L, double *b) {
  for (int k = 0; k <= L; ++k) {
    double y = lo + (hi - lo) * (double)k / (double)L;
    b[k] = y > 0.0 ? y : 0.0;
  }
}

/* Step 2: univariate Bernstein coefficients b_0..b_L on [0,1] -> power
 * coefficients c_j of the same polynomial in u:
 *   c_j = C(L,j) sum_{k<=j} (-1)^(j-k) C(j,k) b_k. */
void orc_bern_to_power_1d(int L, const double *b, double *c) {
  for (int j = 0; j <= L; ++j) {
    double s = 0.0;
    for (int k = 0; k <= j; ++k)
      s += (((j - k) & 1) ? -1.0 : 1.0) * orc_binom(j, k) * b[k];
    c[j] = orc_binom(L, j) * s;
  }
}

/* Univariate Bernstein polynomial of degree L at u in [0,1], eq. (bernpol). */
double orc_bern_eval_1d(int L, const double *b, double u) {
  double s = 0.0;
  for (int k = 0; k <= L; ++k)
    s += b[k] * orc_binom(L, k) * pow(u, k) * pow(1.0 - u, L - k);
  return s;
}

/* Over-approximant of Prop. 1 as a power series in u = (y-lo)/(hi-lo)
 * (coefficients c[0..L]) and the shift e = B(0) of Prop. 2 (eq. max_error),
 * evaluated at u0 = -lo/(hi-lo) from the Bernstein form. */
void orc_relu_poly(double lo, double hi, int L, double *c, double *e) {
  double b[65];
  orc_relu_bern_coefs(lo, hi, L, b);
  orc_bern_to_power_1d(L, b, c);
  *e = orc_bern_eval_1d(L, b, -lo / (hi - lo));
}

/* ------------------------------------------------ Section 5: propagation */

typedef struct {
  int d;      /* per-variable degree */
  double *U;  /* [h][(d+1)^n] Bernstein coefficients, upper polynomials */
  double *Lw; /* same, lower polynomials */
} layer_t;

/* Step 3 for one polynomial P (degree d, Bernstein): sum_j c_j nu(P)^j with
 * nu(P) = (P - lo)/(hi - lo), computed with Pow_Bern and Sum_Bern; the result
 * has degree Lr*d and is written to out. */
static int compose(int n, int d, const double *P, double lo, double hi, int Lr,
                   const double *c, double *out) {
  long long cd = orc_tsize(n, d), co = orc_tsize(n, Lr * d);
  if (cd < 0 || co < 0) return ORC_E_TOO_LARGE;
  double *nu = (double *)malloc(sizeof(double) * (size_t)cd);
  double *pw = (double *)malloc(sizeof(double) * (size_t)co);
  double *acc = (double *)malloc(sizeof(double) * (size_t)co);
  double *tmp = (double *)malloc(sizeof(double) * (size_t)co);
  if (!nu || !pw || !acc || !tmp) { free(nu); free(pw); free(acc); free(tmp); return ORC_E_OOM; }
  /* nu = (P - lo) / (hi - lo): affine map of the coefficients (partition of unity) */
  for (long long i = 0; i < cd; ++i) nu[i] = (P[i] - lo) / (hi - lo);
  int st = ORC_OK;
  int dacc = 0;
  acc[0] = 0.0;
  for (int j = 0; j <= Lr && st == ORC_OK; ++j) {
    st = orc_pow_bern(n, d, nu, j, pw); /* degree j*d */
    if (st != ORC_OK) break;
    long long cj = orc_tsize(n, j * d);
    for (long long i = 0; i < cj; ++i) pw[i] *= c[j];
    st = orc_sum_bern(n, dacc, acc, j * d, pw, tmp);
    dacc = dacc > j * d ? dacc : j * d;
    memcpy(acc, tmp, sizeof(double) * (size_t)orc_tsize(n, dacc));
  }
  if (st == ORC_OK) {
    /* d == 0 gives dacc == 0 == Lr*d */
    memcpy(out, acc, sizeof(double) * (size_t)co);
  }
  free(nu); free(pw); free(acc); free(tmp);
  return st;
}

/* Least-squares affine fit of a Bernstein control net {(K/d, b_K)} (reading
 * R9). Returns beta[0] = mean, beta[1+a] = slope along variable a, so that
 * l(t) = beta0 + sum_a beta_a (t_a - 1/2). The centred grid makes the normal
 * equations diagonal. */
static void ls_affine(int n, int d, const double *B, double *beta) {
  long long c = orc_tsize(n, d);
  int k[16];
  for (int a = 0; a <= n; ++a) beta[a] = 0.0;
  double ss[16] = {0};
  for (long long i = 0; i < c; ++i) {
    beta[0] += B[i];
    if (d == 0) continue;
    digits(i, n, d, k);
    for (int a = 0; a < n; ++a) {
      double s = (double)k[a] / d - 0.5;
      beta[1 + a] += B[i] * s;
      ss[a] += s * s;
    }
  }
  beta[0] /= (double)c;
  for (int a = 0; a < n; ++a) beta[1 + a] = (d == 0) ? 0.0 : beta[1 + a] / ss[a];
}

/* Exported for the tests (pins of reading R9). */
void orc_ls_affine(int n, int d, const double *B, double *beta) { ls_affine(n, d, B, beta); }

/* Affine function l given by beta, evaluated at t. */
static double ls_eval(int n, const double *beta, const double *t) {
  double v = beta[0];
  for (int a = 0; a < n; ++a) v += beta[1 + a] * (t[a] - 0.5);
  return v;
}

/* Linear fallback (reading R9) of a degree-d polynomial P: returns the
 * degree-1 Bernstein tensor of l + max_K(P_K - l(K/d)) (upper, sign=+1) or
 * l + min_K(...) (lower, sign=-1). */
static void linearize(int n, int d, const double *P, int sign, double *out) {
  double beta[17];
  ls_affine(n, d, P, beta);
  long long c = orc_tsize(n, d);
  int k[16];
  double t[16];
  double ext = sign > 0 ? -INFINITY : INFINITY;
  for (long long i = 0; i < c; ++i) {
    digits(i, n, d, k);
    for (int a = 0; a < n; ++a) t[a] = d == 0 ? 0.5 : (double)k[a] / d;
    double r = P[i] - ls_eval(n, beta, t);
    if (sign > 0 ? r > ext : r < ext) ext = r;
  }
  long long c1 = orc_tsize(n, 1);
  for (long long i = 0; i < c1; ++i) {
    digits(i, n, 1, k);
    for (int a = 0; a < n; ++a) t[a] = (double)k[a];
    out[i] = ls_eval(n, beta, t) + ext; /* linear precision: Bernstein coef = value at corner */
  }
}

void orc_linearize(int n, int d, const double *P, int sign, double *out) { linearize(n, d, P, sign, out); }

static double tmin(const double *x, long long c) {
  double m = x[0];
  for (long long i = 1; i < c; ++i) if (x[i] < m) m = x[i];
  return m;
}
static double tmax(const double *x, long long c) {
  double m = x[0];
  for (long long i = 1; i < c; ++i) if (x[i] > m) m = x[i];
  return m;
}

static int g_threads = 0;
void orc_set_threads(int t) { g_threads = t; }
int orc_get_threads(void) {
#ifdef _OPENMP
  return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
  return 1;
#endif
}

/* Whole network over one box (Problem 1, Section 5.3).
 *   H            number of affine layers; widths[0..H] = n, h_1, ..., h_H
 *   W, bias      all layers concatenated; W^(i) row-major h_i x h_{i-1}
 *   box_lo/hi    the input box I_n(d_lo, d_hi)
 *   L            ReLU approximation order (plain rule)
 *   plan         NULL: plain rule (R7); else one code per hidden neuron (R8)
 *   neuron_lo/hi pre-activation bounds [lo, hi] of every hidden neuron (Step 1)
 *   out_lo/hi    output bounds: min / max Bernstein coefficient (Def. 2)
 *   rel_vol      (nullable) relative volume of Section 6: mean over the box of
 *                upper minus lower output polynomial, in closed form from the
 *                Bernstein coefficients (each basis function integrates to 1/(d+1)^n)
 *   out_deg      (nullable) degree of the output polynomials
 *   out_U/out_L  (nullable) output Bernstein tensors, capacity out_cap doubles each
 *   used_plan    (nullable) per hidden neuron: the ReLU degree actually used
 *                (0 inactive/zero, -1 active/identity, -2 linear fallback, >=1 degree)
 *   lin          periodic linearisation (reading R13): 0 off, k >= 1 after
 *                every k-th hidden layer
 */
int orc_network(int H, const int *widths, const double *W, const double *bias,
                const double *box_lo, const double *box_hi, int L, const int8_t *plan,
                double *neuron_lo, double *neuron_hi, double *out_lo, double *out_hi,
                double *rel_vol, int *out_deg, double *out_U, double *out_L,
                long long out_cap, int8_t *used_plan, int lin) {
  if (H < 1 || !widths || !W || !bias || !box_lo || !box_hi || lin < 0) return ORC_E_ARG;
  int n = widths[0];
  if (n < 1 || n > 16) return ORC_E_ARG;
  for (int i = 0; i <= H; ++i) if (widths[i] < 1) return ORC_E_ARG;
  if (!plan && (L < 1 || L > 64)) return ORC_E_DEGREE;
  for (int a = 0; a < n; ++a)
    if (!(box_lo[a] <= box_hi[a]) || !isfinite(box_lo[a]) || !isfinite(box_hi[a])) return ORC_E_BOX;
  if (plan) {
    long long nh = 0;
    for (int i = 1; i < H; ++i) nh += widths[i];
    for (long long j = 0; j < nh; ++j)
      if (plan[j] < 0 || plan[j] > 8) return ORC_E_DEGREE;
  }
#ifdef _OPENMP
  if (g_threads > 0) omp_set_num_threads(g_threads);
#endif

  /* Section 5.3 input initialisation: x_a at degree (1,...,1) is the Kronecker
   * product [d_lo_a; d_hi_a] (x) [1;1] ... with the box interval on axis a. */
  layer_t prev;
  prev.d = 1;
  long long c1 = orc_tsize(n, 1);
  prev.U = (double *)malloc(sizeof(double) * (size_t)(n * c1));
  prev.Lw = (double *)malloc(sizeof(double) * (size_t)(n * c1));
  if (!prev.U || !prev.Lw) return ORC_E_OOM;
  {
    int k[16];
    for (int a = 0; a < n; ++a)
      for (long long i = 0; i < c1; ++i) {
        digits(i, n, 1, k);
        prev.U[a * c1 + i] = k[a] ? box_hi[a] : box_lo[a];
        prev.Lw[a * c1 + i] = prev.U[a * c1 + i];
      }
  }

  int st = ORC_OK;
  long long woff = 0, boff = 0, noff = 0;
  for (int layer = 1; layer <= H && st == ORC_OK; ++layer) {
    int hin = widths[layer - 1], h = widths[layer];
    int d = prev.d;
    long long cd = orc_tsize(n, d);
    if (cd < 0) { st = ORC_E_TOO_LARGE; break; }
    const double *Wl = W + woff, *bl = bias + boff;
    double *Uh = (double *)malloc(sizeof(double) * (size_t)(h * cd));
    double *Lh = (double *)malloc(sizeof(double) * (size_t)(h * cd));
    if (!Uh || !Lh) { free(Uh); free(Lh); st = ORC_E_OOM; break; }

    /* Section 5.2: U^ = W+ U + W- L + b, L^ = W+ L + W- U + b (R2, R3). */
#pragma omp parallel for schedule(dynamic)
    for (int j = 0; j < h; ++j) {
      for (long long i = 0; i < cd; ++i) {
        double su = bl[j], sl = bl[j];
        for (int k = 0; k < hin; ++k) {
          double w = Wl[(long long)j * hin + k];
          double wp = w > 0.0 ? w : 0.0, wm = w < 0.0 ? w : 0.0;
          su += wp * prev.U[k * cd + i] + wm * prev.Lw[k * cd + i];
          sl += wp * prev.Lw[k * cd + i] + wm * prev.U[k * cd + i];
        }
        Uh[j * cd + i] = su;
        Lh[j * cd + i] = sl;
      }
    }
    free(prev.U);
    free(prev.Lw);
    prev.U = prev.Lw = NULL;

    if (layer == H) {
      /* outputs: Def. 2 on the output polynomials */
      for (int j = 0; j < h; ++j) {
        out_lo[j] = tmin(Lh + j * cd, cd);
        out_hi[j] = tmax(Uh + j * cd, cd);
        if (rel_vol) {
          double s = 0.0;
          for (long long i = 0; i < cd; ++i) s += Uh[j * cd + i] - Lh[j * cd + i];
          rel_vol[j] = s / (double)cd;
        }
      }
      if (out_deg) *out_deg = d;
      if (out_U && out_L && out_cap >= (long long)h * cd) {
        memcpy(out_U, Uh, sizeof(double) * (size_t)(h * cd));
        memcpy(out_L, Lh, sizeof(double) * (size_t)(h * cd));
      }
      free(Uh); free(Lh);
      break;
    }

    /* Step 1 for every neuron, then the degree each neuron's post takes. */
    double *lo = (double *)malloc(sizeof(double) * h), *hi = (double *)malloc(sizeof(double) * h);
    int *deg = (int *)malloc(sizeof(int) * h), *kind = (int *)malloc(sizeof(int) * h);
    int dpost = 0;
    for (int j = 0; j < h; ++j) {
      lo[j] = tmin(Lh + j * cd, cd);
      hi[j] = tmax(Uh + j * cd, cd);
      neuron_lo[noff + j] = lo[j];
      neuron_hi[noff + j] = hi[j];
      if (hi[j] <= 0.0) { kind[j] = 0; deg[j] = 0; }            /* inactive (R4) */
      else if (lo[j] >= 0.0) { kind[j] = -1; deg[j] = d; }      /* active (R4) */
      else if (!plan) { kind[j] = L; deg[j] = L * d; }          /* unstable, plain */
      else if (plan[noff + j] >= 1) { kind[j] = plan[noff + j]; deg[j] = plan[noff + j] * d; }
      else { kind[j] = -2; deg[j] = 1; }                        /* linear fallback (R9) */
      if (used_plan) used_plan[noff + j] = (int8_t)kind[j];
      if (deg[j] > dpost) dpost = deg[j];
    }
    if (!plan) dpost = L * d; /* R7: uniform elevation */
    long long cp = orc_tsize(n, dpost);
    if (cp < 0) { st = ORC_E_TOO_LARGE; free(lo); free(hi); free(deg); free(kind); free(Uh); free(Lh); break; }
    prev.d = dpost;
    prev.U = (double *)malloc(sizeof(double) * (size_t)(h * cp));
    prev.Lw = (double *)malloc(sizeof(double) * (size_t)(h * cp));
    if (!prev.U || !prev.Lw) { st = ORC_E_OOM; free(lo); free(hi); free(deg); free(kind); free(Uh); free(Lh); break; }

    int stl = ORC_OK;
#pragma omp parallel for schedule(dynamic) reduction(min : stl)
    for (int j = 0; j < h; ++j) {
      double *pu = prev.U + j * cp, *pl = prev.Lw + j * cp;
      long long cmx = orc_tsize(n, deg[j] > d ? deg[j] : d);
      double *tu = (double *)malloc(sizeof(double) * (size_t)cmx);
      double *tl = (double *)malloc(sizeof(double) * (size_t)cmx);
      int s = ORC_OK;
      if (!tu || !tl) s = ORC_E_OOM;
      else if (kind[j] == 0) {
        tu[0] = tl[0] = 0.0; /* zero polynomial at degree 0 */
      } else if (kind[j] == -1) {
        memcpy(tu, Uh + j * cd, sizeof(double) * (size_t)cd);
        memcpy(tl, Lh + j * cd, sizeof(double) * (size_t)cd);
      } else {
        int Lr = kind[j] >= 1 ? kind[j] : 1;
        double c[65], e;
        orc_relu_poly(lo[j], hi[j], Lr, c, &e);
        s = compose(n, d, Uh + j * cd, lo[j], hi[j], Lr, c, tu);          /* eq. (post_bounds_2) */
        if (s == ORC_OK) s = compose(n, d, Lh + j * cd, lo[j], hi[j], Lr, c, tl); /* eq. (post_bounds_1) */
        if (s == ORC_OK) {
          long long cl = orc_tsize(n, Lr * d);
          for (long long i = 0; i < cl; ++i) tl[i] -= e; /* Prop. 2 shift, all coefficients */
        }
        if (s == ORC_OK && kind[j] == -2) {
          /* R9: linearise the degree-1 approximant's post polynomials */
          double *lu = (double *)malloc(sizeof(double) * (size_t)orc_tsize(n, 1));
          double *ll = (double *)malloc(sizeof(double) * (size_t)orc_tsize(n, 1));
          linearize(n, d, tu, +1, lu);
          linearize(n, d, tl, -1, ll);
          memcpy(tu, lu, sizeof(double) * (size_t)orc_tsize(n, 1));
          memcpy(tl, ll, sizeof(double) * (size_t)orc_tsize(n, 1));
          free(lu); free(ll);
        }
      }
      /* stack: elevate to the layer's post degree (Prop. 4, Section 5.4) */
      if (s == ORC_OK) s = orc_elevate(n, deg[j], tu, dpost, pu);
      if (s == ORC_OK) s = orc_elevate(n, deg[j], tl, dpost, pl);
      free(tu); free(tl);
      if (s < stl) stl = s;
    }
    st = stl;
    /* R13: every lin-th hidden layer, every neuron's stored post polynomials
     * (degree dpost) become their linearisation at degree 1 */
    if (st == ORC_OK && lin > 0 && layer % lin == 0) {
      long long c1n = orc_tsize(n, 1);
      double *lu = (double *)malloc(sizeof(double) * (size_t)(h * c1n));
      double *ll = (double *)malloc(sizeof(double) * (size_t)(h * c1n));
      if (!lu || !ll) {
        free(lu); free(ll);
        st = ORC_E_OOM;
      } else {
        for (int j = 0; j < h; ++j) {
          linearize(n, dpost, prev.U + j * cp, +1, lu + j * c1n);
          linearize(n, dpost, prev.Lw + j * cp, -1, ll + j * c1n);
        }
        free(prev.U);
        free(prev.Lw);
        prev.U = lu;
        prev.Lw = ll;
        prev.d = 1;
      }
    }
    free(lo); free(hi); free(deg); free(kind);
    free(Uh); free(Lh);
    woff += (long long)h * hin;
    boff += h;
    noff += h;
  }
  free(prev.U);
  free(prev.Lw);
  return st;
}

/* Several boxes, one after the other (boxes are independent). */
int orc_network_boxes(int H, const int *widths, const double *W, const double *bias,
                      long long n_boxes, const double *box_lo, const double *box_hi, int L,
                      const int8_t *plan, double *neuron_lo, double *neuron_hi,
                      double *out_lo, double *out_hi) {
  int n = widths[0];
  long long nh = 0;
  for (int i = 1; i < H; ++i) nh += widths[i];
  int o = widths[H];
  for (long long bx = 0; bx < n_boxes; ++bx) {
    int st = orc_network(H, widths, W, bias, box_lo + bx * n, box_hi + bx * n, L,
                         plan ? plan + bx * nh : NULL, neuron_lo + bx * nh, neuron_hi + bx * nh,
                         out_lo + bx * o, out_hi + bx * o, NULL, NULL, NULL, NULL, 0, NULL, 0);
    if (st != ORC_OK) return st;
  }
  return ORC_OK;
}
