/* Runs the oracle's entry points on small seeded inputs so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer checks every access and
 * every integer operation they make. Exit status 0 when every call returns
 * its expected status; the sanitizers abort on any error they find. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

long long orc_tsize(int n, int d);
int orc_prod(int n, int da, const double *A, int db, const double *B, double *out);
int orc_prod_bern(int n, int da, const double *A, int db, const double *B, double *out);
int orc_elevate(int n, int d, const double *A, int e, double *out);
int orc_pow_bern(int n, int d, const double *A, int i, double *out);
int orc_sum_bern(int n, int da, const double *A, int db, const double *B, double *out);
double orc_bern_eval(int n, int d, const double *B, const double *t);
int orc_power_to_bern(int n, int d, const double *a, double *b);
void orc_relu_bern_coefs(double lo, double hi, int L, double *b);
void orc_relu_poly(double lo, double hi, int L, double *c, double *e);
void orc_ls_affine(int n, int d, const double *B, double *beta);
void orc_linearize(int n, int d, const double *P, int sign, double *out);
void orc_set_threads(int t);
int orc_network(int H, const int *widths, const double *W, const double *bias, const double *box_lo,
                const double *box_hi, int L, const int8_t *plan, double *neuron_lo, double *neuron_hi,
                double *out_lo, double *out_hi, double *rel_vol, int *out_deg, double *out_U, double *out_L,
                long long out_cap, int8_t *used_plan, int lin);
int orc_network_boxes(int H, const int *widths, const double *W, const double *bias, long long n_boxes,
                      const double *box_lo, const double *box_hi, int L, const int8_t *plan, double *neuron_lo,
                      double *neuron_hi, double *out_lo, double *out_hi);

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* xorshift64*, uniform in [-1, 1) */
  g_state ^= g_state >> 12;
  g_state ^= g_state << 25;
  g_state ^= g_state >> 27;
  return (double)((g_state * 0x2545F4914F6CDD1Dull) >> 11) / 4503599627370496.0 - 1.0;
}

static double *vec(long long m) {
  double *v = malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
  for (long long i = 0; i < m; ++i) v[i] = urand();
  return v;
}

static int fails = 0;
#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      fprintf(stderr, "failed: %s (line %d)\n", #cond, __LINE__); \
      ++fails;                                                    \
    }                                                             \
  } while (0)

static void primitives(void) {
  for (int n = 1; n <= 3; ++n)
    for (int d = 0; d <= 3; ++d) {
      const long long C = orc_tsize(n, d), C2 = orc_tsize(n, 2 * d), Ce = orc_tsize(n, d + 2);
      double *A = vec(C), *B = vec(C), *P = vec(C2), *E = vec(Ce), *Q = vec(C), *S = vec(C);
      double t[3] = {0.25, 0.5, 0.75}, beta[4], lin[8]; /* lin: degree-1 Bernstein tensor, 2^n */
      EXPECT(orc_prod(n, d, A, d, B, P) == 0);
      EXPECT(orc_prod_bern(n, d, A, d, B, P) == 0);
      EXPECT(orc_elevate(n, d, A, d + 2, E) == 0);
      EXPECT(orc_pow_bern(n, d, A, 2, P) == 0);
      EXPECT(orc_sum_bern(n, d, A, d, B, S) == 0);
      EXPECT(isfinite(orc_bern_eval(n, d, A, t)));
      EXPECT(orc_power_to_bern(n, d, A, Q) == 0);
      if (d >= 1) {
        orc_ls_affine(n, d, A, beta);
        orc_linearize(n, d, A, 1, lin);
        orc_linearize(n, d, A, -1, lin);
      }
      free(A); free(B); free(P); free(E); free(Q); free(S);
    }
  for (int L = 1; L <= 8; ++L) {
    double b[9], c[9], e;
    orc_relu_bern_coefs(-1.5, 2.0, L, b);
    orc_relu_poly(-1.5, 2.0, L, c, &e);
    EXPECT(isfinite(e));
  }
}

static void network(const int *widths, int H, int L, int with_plan, int lin) {
  const int n = widths[0], o = widths[H];
  long long nw = 0, nb = 0, nh = 0;
  for (int i = 1; i <= H; ++i) {
    nw += (long long)widths[i] * widths[i - 1];
    nb += widths[i];
    if (i < H) nh += widths[i];
  }
  double *W = vec(nw), *b = vec(nb), lo[16], hi[16];
  for (int a = 0; a < n; ++a) {
    const double c = urand(), w = 0.05 + 0.3 * (urand() + 1.0);
    lo[a] = c - w;
    hi[a] = c + w;
  }
  int8_t *plan = NULL, *used = malloc((size_t)(nh > 0 ? nh : 1));
  if (with_plan) {
    plan = malloc((size_t)(nh > 0 ? nh : 1));
    for (long long j = 0; j < nh; ++j) plan[j] = (int8_t)(j % 4); /* codes 0 (fallback) .. 3 */
  }
  double *nlo = vec(nh), *nhi = vec(nh), *olo = vec(o), *ohi = vec(o), *rv = vec(o);
  const long long cap = 1 << 16;
  double *U = vec(cap * o), *Lw = vec(cap * o);
  int deg = -1;
  const int st = orc_network(H, widths, W, b, lo, hi, L, plan, nlo, nhi, olo, ohi, rv, &deg, U, Lw, cap, used, lin);
  EXPECT(st == 0);
  for (int k = 0; k < o && st == 0; ++k) EXPECT(olo[k] <= ohi[k] && rv[k] >= 0.0);
  /* several boxes through the batch entry */
  double blo[2 * 16], bhi[2 * 16];
  for (int q = 0; q < 2; ++q)
    for (int a = 0; a < n; ++a) {
      blo[q * n + a] = lo[a];
      bhi[q * n + a] = hi[a];
    }
  int8_t *plan2 = NULL;
  if (plan) {
    plan2 = malloc((size_t)(2 * (nh > 0 ? nh : 1)));
    for (long long j = 0; j < 2 * nh; ++j) plan2[j] = plan[j % (nh > 0 ? nh : 1)];
  }
  double *nlo2 = vec(2 * nh), *nhi2 = vec(2 * nh), *olo2 = vec(2 * o), *ohi2 = vec(2 * o);
  EXPECT(orc_network_boxes(H, widths, W, b, 2, blo, bhi, L, plan2, nlo2, nhi2, olo2, ohi2) == 0);
  free(W); free(b); free(plan); free(plan2); free(used); free(nlo); free(nhi); free(olo); free(ohi); free(rv);
  free(U); free(Lw); free(nlo2); free(nhi2); free(olo2); free(ohi2);
}

static void rejects(void) {
  const int widths[3] = {2, 3, 1};
  double W[9] = {0}, b[4] = {0}, lo[2] = {1.0, 0.0}, hi[2] = {0.0, 1.0}, nl[3], nh[3], ol[1], oh[1];
  EXPECT(orc_network(2, widths, W, b, lo, hi, 2, NULL, nl, nh, ol, oh, NULL, NULL, NULL, NULL, 0, NULL, 0) != 0);
  lo[0] = -1.0;
  hi[0] = 1.0;
  EXPECT(orc_network(2, widths, W, b, lo, hi, 0, NULL, nl, nh, ol, oh, NULL, NULL, NULL, NULL, 0, NULL, 0) != 0);
  EXPECT(orc_network(2, widths, W, b, lo, hi, 2, NULL, nl, nh, ol, oh, NULL, NULL, NULL, NULL, 0, NULL, -1) != 0);
  const int8_t bad[3] = {9, 0, 0};
  EXPECT(orc_network(2, widths, W, b, lo, hi, 2, bad, nl, nh, ol, oh, NULL, NULL, NULL, NULL, 0, NULL, 0) != 0);
}

int main(void) {
  orc_set_threads(2);
  primitives();
  const int w1[4] = {2, 5, 5, 1}, w2[5] = {3, 6, 5, 4, 2}, w3[3] = {1, 4, 1};
  network(w1, 3, 1, 0, 0);
  network(w1, 3, 2, 0, 0);
  network(w1, 3, 3, 0, 0);
  network(w2, 4, 2, 0, 0);
  network(w2, 4, 3, 1, 0);
  network(w2, 4, 2, 0, 1);
  network(w2, 4, 3, 1, 2);
  network(w3, 2, 8, 0, 0);
  rejects();
  if (fails) {
    fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  printf("oracle driver: all calls clean\n");
  return 0;
}
