/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow CPU FP64 reference for the potential of charges in a layered
 * medium (Wang, Zhang & Cai, "Fast multipole method for 3-D Laplace equation
 * in layered media", arXiv:1908.10863).  Only tests/, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file's library.  It shares
 * no code with the GPU path.
 *
 * What is computed (Sec. 3.1, eqs. totalinteraction / freereactioncomponents):
 *   Phi_i = sum_{j != i, same layer} q_j / (4 pi |r_i - r_j|)
 *         + sum_{j (all, incl. j = i)} q_j sum_{valid ab} u^{ab}(r_i, r_j)
 *   u^{ab}(r, r') = 1/(4 pi) int_0^inf J0(k rho) exp(-k zeta^{ab}) sigma^{ab}(k) dk
 * with zeta^{ab} the interface-relative exponent of eq. zexponential and the
 * 1/(8 pi^2) double integral of eq. generalcomponents reduced to J0 by the
 * Bessel integral of Sec. 3.4.
 *
 * Conventions (layer l is d_l < z < d_{l-1}; layer 0 on top, layer L at the
 * bottom; interfaces d_0 > d_1 > ... > d_{L-1}):
 *   a = 1 : target-side wave from the target layer's bottom interface d_l
 *   a = 2 : target-side wave from its top interface d_{l-1}
 *   b = 1 : source wave towards the source layer's bottom interface d_l'
 *   b = 2 : source wave towards its top interface d_{l'-1}
 * Output arrays of four sigmas are indexed [2*(a-1) + (b-1)].
 *
 * Parity pins for every function live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
#define OR_MAXL 16

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of later parallel loops (a single-core timing of the oracle uses 1). */
void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

static int valid_side(int L, int layer, int side) {
  return side == 1 ? (layer <= L - 1) : (layer >= 1);
}

/* ------------------------------------------------------------------------ */
/* Reaction densities by a direct solve of the interface system (App. A).    */
/*                                                                          */
/* In layer i the reaction part of the transformed field (normalised by the  */
/* free-space factor) is  s1_i exp(-k(z - d_i)) + s2_i exp(-k(d_{i-1} - z)), */
/* with s2_0 = s1_L = 0 for decay at +-infinity.  The source's own free wave */
/* reaches its bottom interface with amplitude g1 and its top one with g2.   */
/* Continuity of u and eps du/dz at every interface d_i gives 2L equations   */
/* for the 2L unknowns; b = 1 is the response to (g1,g2) = (1,0) and b = 2   */
/* the response to (0,1).  Gaussian elimination with partial pivoting.       */
/* ------------------------------------------------------------------------ */
/* Densities for the general interface conditions a_{i} u_i = a_{i+1} u_{i+1}
 * and b_i du_i/dz = b_{i+1} du_{i+1}/dz at z = d_i (the general conditions of
 * App. A; a == NULL means a_i = 1, and b = eps gives the classic transmission
 * conditions).  The same direct solve as the classic case, row by row. */
int oracle_sigma_ab(int L, const double* d, const double* acoef, const double* eps, int lt,
                    int ls, double k, double* out) {
  if (L < 1 || L > OR_MAXL || lt < 0 || lt > L || ls < 0 || ls > L) return -1;
  const int n = 2 * L;
  double A[2 * OR_MAXL][2 * OR_MAXL];
  double R[2 * OR_MAXL][2];
  memset(A, 0, sizeof(A));
  memset(R, 0, sizeof(R));
  /* unknown columns: s1_i (i = 0..L-1) -> i ; s2_i (i = 1..L) -> L + i - 1 */
#define C1(i) (i)
#define C2(i) (L + (i) - 1)
  for (int i = 0; i < L; ++i) {
    /* e_i = exp(-k D_i), D_i = d_{i-1} - d_i : thickness of layer i (i >= 1) */
    const double ei = (i >= 1) ? exp(-k * (d[i - 1] - d[i])) : 0.0;
    const double ei1 = (i + 1 <= L - 1) ? exp(-k * (d[i] - d[i + 1])) : 0.0;
    const int rc = 2 * i, rf = 2 * i + 1;
    const double a0 = acoef ? acoef[i] : 1.0, a1 = acoef ? acoef[i + 1] : 1.0;
    /* continuity of a u at z = d_i */
    A[rc][C1(i)] += a0;
    if (i >= 1) A[rc][C2(i)] += a0 * ei;
    if (i + 1 <= L - 1) A[rc][C1(i + 1)] -= a1 * ei1;
    A[rc][C2(i + 1)] -= a1;
    if (ls == i) R[rc][0] -= a0;     /* g1 on the upper side */
    if (ls == i + 1) R[rc][1] += a1; /* g2 on the lower side */
    /* continuity of eps du/dz at z = d_i (divided by -k) */
    A[rf][C1(i)] += eps[i];
    if (i >= 1) A[rf][C2(i)] -= eps[i] * ei;
    if (i + 1 <= L - 1) A[rf][C1(i + 1)] -= eps[i + 1] * ei1;
    A[rf][C2(i + 1)] += eps[i + 1];
    if (ls == i) R[rf][0] += eps[i];
    if (ls == i + 1) R[rf][1] += eps[i + 1];
  }
  /* elimination with partial pivoting */
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
    if (A[piv][c] == 0.0) return -2;
    if (piv != c) {
      for (int j = 0; j < n; ++j) { double t = A[c][j]; A[c][j] = A[piv][j]; A[piv][j] = t; }
      for (int j = 0; j < 2; ++j) { double t = R[c][j]; R[c][j] = R[piv][j]; R[piv][j] = t; }
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r][c] / A[c][c];
      if (f == 0.0) continue;
      for (int j = c; j < n; ++j) A[r][j] -= f * A[c][j];
      R[r][0] -= f * R[c][0];
      R[r][1] -= f * R[c][1];
    }
  }
  double X[2 * OR_MAXL][2];
  for (int c = n - 1; c >= 0; --c) {
    for (int j = 0; j < 2; ++j) {
      double s = R[c][j];
      for (int m = c + 1; m < n; ++m) s -= A[c][m] * X[m][j];
      X[c][j] = s / A[c][c];
    }
  }
  for (int a = 1; a <= 2; ++a)
    for (int b = 1; b <= 2; ++b) {
      double v = 0.0;
      if (valid_side(L, lt, a) && valid_side(L, ls, b)) {
        const int col = (a == 1) ? C1(lt) : C2(lt);
        v = X[col][b - 1];
      }
      out[2 * (a - 1) + (b - 1)] = v;
    }
#undef C1
#undef C2
  return 0;
}

int oracle_sigma(int L, const double* d, const double* eps, int lt, int ls,
                 double k, double* out) {
  return oracle_sigma_ab(L, d, NULL, eps, lt, ls, k, out);
}

/* ------------------------------------------------------------------------ */
/* Closed-form densities of a three-layer medium (App. A, eqs.               */
/* densitythreelayer1-3), written with x = exp(-k D), D = d_0 - d_1, as      */
/* sigma = (n0 + n1 x + n2 x^2) / (2 kappa),                                 */
/* kappa = [(e0+e1)(e1+e2) + (e0-e1)(e1-e2) x^2] / 2.                        */
/* Two printed entries are read differently (see the reading list kept with  */
/* the design notes): the x^2 term of kappa carries (e1 - e2) and the two    */
/* numerator terms of sigma^{22}_{22} pair as (e2-e1)(e0+e1) + (e1-e0)(e1+e2)x^2, */
/* so that every density tends to its nearest-interface limit as k -> inf.   */
/* ------------------------------------------------------------------------ */
static void sigma3_numerators(const double* e, int lt, int ls, int a, int b,
                              double* n0, double* n1, double* n2) {
  const double e0 = e[0], e1 = e[1], e2 = e[2];
  *n0 = *n1 = *n2 = 0.0;
  const int code = lt * 1000 + ls * 100 + a * 10 + b;
  switch (code) {
    /* source in the top layer */
    case 11: *n0 = (e0 - e1) * (e1 + e2); *n2 = (e0 + e1) * (e1 - e2); break; /* s^{11}_{00} */
    case 1021: *n0 = 2.0 * e0 * (e1 + e2); break;                              /* s^{21}_{10} */
    case 1011: *n1 = 2.0 * e0 * (e1 - e2); break;                              /* s^{11}_{10} */
    case 2021: *n1 = 4.0 * e0 * e1; break;                                     /* s^{21}_{20} */
    /* source in the middle layer */
    case 112: *n0 = 2.0 * e1 * (e1 + e2); break;                               /* s^{12}_{01} */
    case 111: *n1 = 2.0 * e1 * (e1 - e2); break;                               /* s^{11}_{01} */
    case 1111: *n0 = (e1 - e2) * (e1 + e0); break;                             /* s^{11}_{11} */
    case 1121: *n1 = (e1 - e2) * (e1 - e0); break;                             /* s^{21}_{11} */
    case 1112: *n1 = (e1 - e2) * (e1 - e0); break;                             /* s^{12}_{11} */
    case 1122: *n0 = (e1 + e2) * (e1 - e0); break;                             /* s^{22}_{11} */
    case 2122: *n1 = 2.0 * e1 * (e1 - e0); break;                              /* s^{22}_{21} */
    case 2121: *n0 = 2.0 * e1 * (e0 + e1); break;                              /* s^{21}_{21} */
    /* source in the bottom layer */
    case 212: *n1 = 4.0 * e1 * e2; break;                                      /* s^{12}_{02} */
    case 1222: *n1 = 2.0 * e2 * (e1 - e0); break;                              /* s^{22}_{12} */
    case 1212: *n0 = 2.0 * e2 * (e0 + e1); break;                              /* s^{12}_{12} */
    case 2222: *n0 = (e2 - e1) * (e0 + e1); *n2 = (e1 - e0) * (e1 + e2); break; /* s^{22}_{22} */
    default: break;
  }
}

int oracle_sigma3(const double* d, const double* eps, int lt, int ls, double k,
                  double* out) {
  if (lt < 0 || lt > 2 || ls < 0 || ls > 2) return -1;
  const double x = exp(-k * (d[0] - d[1]));
  const double kap = 0.5 * ((eps[0] + eps[1]) * (eps[1] + eps[2]) +
                            (eps[0] - eps[1]) * (eps[1] - eps[2]) * x * x);
  for (int a = 1; a <= 2; ++a)
    for (int b = 1; b <= 2; ++b) {
      double n0, n1, n2;
      sigma3_numerators(eps, lt, ls, a, b, &n0, &n1, &n2);
      out[2 * (a - 1) + (b - 1)] = (n0 + n1 * x + n2 * x * x) / (2.0 * kap);
    }
  return 0;
}

/* Image series of a three-layer density: expanding 1/kappa as a geometric    */
/* series in x^2 gives sigma(k) = sum_t c_t exp(-k s_t D) with s_t integer,   */
/* hence u^{ab} = sum_t c_t / (4 pi sqrt(rho^2 + (zeta + s_t D)^2)).          */
/* Fills up to maxterm (coef, shift) pairs; returns the count.                */
int oracle_image3_terms(const double* eps, int lt, int ls, int a, int b,
                        int maxterm, double* coef, int* shift) {
  double n0, n1, n2;
  sigma3_numerators(eps, lt, ls, a, b, &n0, &n1, &n2);
  const double P = (eps[0] + eps[1]) * (eps[1] + eps[2]);
  const double Rr = (eps[0] - eps[1]) * (eps[1] - eps[2]);
  const double ratio = -Rr / P; /* 1/kappa = (2/P) sum_j ratio^j x^{2j} */
  /* sigma = (1/P) sum_j ratio^j (n0 x^{2j} + n1 x^{2j+1} + n2 x^{2j+2}) */
  int cnt = 0;
  double rj = 1.0;
  for (int j = 0; j < 400 && cnt + 3 <= maxterm; ++j) {
    const double mag = fabs(rj) * (fabs(n0) + fabs(n1) + fabs(n2)) / P;
    if (j > 0 && mag < 1e-19) break;
    if (n0 != 0.0) { coef[cnt] = rj * n0 / P; shift[cnt] = 2 * j; ++cnt; }
    if (n1 != 0.0) { coef[cnt] = rj * n1 / P; shift[cnt] = 2 * j + 1; ++cnt; }
    if (n2 != 0.0) { coef[cnt] = rj * n2 / P; shift[cnt] = 2 * j + 2; ++cnt; }
    rj *= ratio;
    if (rj == 0.0) break;
  }
  return cnt;
}

/* ------------------------------------------------------------------------ */
/* Fixed composite Gauss-Legendre rule on [0, kmax] for the Sommerfeld       */
/* integrals.  Nodes are shared by every pair of one call so that sigma(k)   */
/* is evaluated once per node.  A density is a sum of exponentials           */
/* exp(-c k) (multiple reflections in the finite layers), so panels start    */
/* small at k = 0 and grow geometrically (ratio 1.2, width ~ k/5): any       */
/* exponential is then integrated to full precision where it is not         */
/* negligible.  The panel width is capped so that 20 points cover at most a  */
/* full period of J0(k rho_max), ten e-folds of exp(-k zeta_min) and a tenth */
/* of the multiple-reflection scale of the thinnest finite layer.            */
/* ------------------------------------------------------------------------ */
#define GL_NPT 20
static void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double t = cos(OR_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int j = 2; j <= n; ++j) {
        double p2 = ((2.0 * j - 1.0) * t * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      /* p1 = P_n(t), p0 = P_{n-1}(t) */
      double dp = n * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (fabs(dt) < 1e-16) break;
    }
    double p0 = 1.0, p1 = t;
    for (int j = 2; j <= n; ++j) {
      double p2 = ((2.0 * j - 1.0) * t * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (t * p1 - p0) / (t * t - 1.0);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

typedef struct {
  int nn;
  double* k;
  double* w;
} rule_t;

static int make_rule(double rho_max, double zeta_min, double dmin, rule_t* r) {
  double gx[GL_NPT], gw[GL_NPT];
  gauss_legendre(GL_NPT, gx, gw);
  const double kmax = 45.0 / zeta_min;
  double hmax = 10.0 / zeta_min;
  if (rho_max > 0.0 && 2.0 * OR_PI / rho_max < hmax) hmax = 2.0 * OR_PI / rho_max;
  if (dmin > 0.0 && 5.0 * dmin < hmax) hmax = 5.0 * dmin;
  double scale = zeta_min < 1.0 ? zeta_min : 1.0;
  if (dmin > 0.0 && dmin < scale) scale = dmin;
  const double h0 = 1e-3 * scale;
  /* count panels */
  int npan = 0;
  for (double k0 = 0.0, h = h0; k0 < kmax; ++npan) {
    k0 += h;
    h = (h * 1.2 < hmax) ? h * 1.2 : hmax;
  }
  r->nn = npan * GL_NPT;
  r->k = (double*)malloc(sizeof(double) * r->nn);
  r->w = (double*)malloc(sizeof(double) * r->nn);
  if (!r->k || !r->w) return -1;
  double k0 = 0.0, h = h0;
  for (int p = 0; p < npan; ++p) {
    for (int i = 0; i < GL_NPT; ++i) {
      r->k[p * GL_NPT + i] = k0 + 0.5 * h * (gx[i] + 1.0);
      r->w[p * GL_NPT + i] = 0.5 * h * gw[i];
    }
    k0 += h;
    h = (h * 1.2 < hmax) ? h * 1.2 : hmax;
  }
  return 0;
}

/* smallest thickness of a finite layer, 0 when there is none */
static double min_thickness(int L, const double* d) {
  double m = 0.0;
  for (int i = 1; i < L; ++i) {
    const double t = d[i - 1] - d[i];
    if (m == 0.0 || t < m) m = t;
  }
  return m;
}

static void free_rule(rule_t* r) {
  free(r->k);
  free(r->w);
}

/* One reaction component by quadrature: 1/(4pi) int J0(k rho) e^{-k zeta} sigma dk.
 * sigma from the direct solve (or sigma == 1 when L == 0). */
double oracle_reaction_quad(int L, const double* d, const double* eps, int lt,
                            int ls, int a, int b, double rho, double zeta) {
  rule_t r;
  if (make_rule(rho, zeta, L > 0 ? min_thickness(L, d) : 0.0, &r)) return NAN;
  double acc = 0.0, cmp = 0.0;
  for (int i = 0; i < r.nn; ++i) {
    double sg = 1.0;
    if (L > 0) {
      double s4[4];
      oracle_sigma(L, d, eps, lt, ls, r.k[i], s4);
      sg = s4[2 * (a - 1) + (b - 1)];
    }
    const double f = r.w[i] * j0(r.k[i] * rho) * exp(-r.k[i] * zeta) * sg;
    /* Neumaier summation */
    const double t = acc + f;
    if (fabs(acc) >= fabs(f)) cmp += (acc - t) + f; else cmp += (f - t) + acc;
    acc = t;
  }
  free_rule(&r);
  return (acc + cmp) / (4.0 * OR_PI);
}

double oracle_reaction_image3(const double* d, const double* eps, int lt, int ls,
                              int a, int b, double rho, double zeta) {
  double coef[1200];
  int shift[1200];
  const int nt = oracle_image3_terms(eps, lt, ls, a, b, 1200, coef, shift);
  const double D = d[0] - d[1];
  double acc = 0.0;
  for (int t = nt - 1; t >= 0; --t) {
    const double zz = zeta + shift[t] * D;
    acc += coef[t] / sqrt(rho * rho + zz * zz);
  }
  return acc / (4.0 * OR_PI);
}

/* exponent zeta^{ab} of eq. zexponential (interface-relative distances) */
static double zeta_of(const double* d, int lt, int ls, int a, int b, double z,
                      double zs) {
  const double t = (a == 1) ? (z - d[lt]) : (d[lt - 1] - z);
  const double s = (b == 1) ? (zs - d[ls]) : (d[ls - 1] - zs);
  return t + s;
}

/* ------------------------------------------------------------------------ */
/* Tabulated reaction kernels (method 2), for direct sums too large for the  */
/* per-pair quadrature.  For every component the kernel                      */
/*   K(rho, zeta) = 1/(4pi) int J0(k rho) e^{-k zeta} sigma(k) dk            */
/* is computed by the shared rule at the nodes of a tensor grid over the     */
/* pairs' (rho, zeta) box and interpolated by polynomials of degree KT_DEG   */
/* in each variable (barycentric formula, Chebyshev-Lobatto points).  rho    */
/* panels have width at most zeta_min (K's singularities lie at least        */
/* zeta_min off the real rho axis); zeta panels double in width from         */
/* zeta_min, as their distance to the singularity at zeta = 0 does.  Before  */
/* use, the interpolant is certified at KT_CHECK random points per component */
/* against the shared rule applied directly: the largest deviation must stay */
/* below KT_TOL times the component's largest node value, else the call      */
/* fails (returns -5).                                                       */
/* ------------------------------------------------------------------------ */
#define KT_DEG 24
#define KT_NP (KT_DEG + 1)
#define KT_CHECK 48
#define KT_TOL 1e-12
#define KT_MAXPAN 256

typedef struct {
  int npr, npz;
  double hr, zmin, zmax;
  double xk[KT_NP], wk[KT_NP]; /* nodes cos(j pi / KT_DEG) and barycentric weights */
  double* val;                 /* [comp][npr * KT_NP][npz * KT_NP] (NULL for invalid components) */
  double* cmax;                /* [comp] largest |node value| */
} ktab_t;

static double kt_zlo(const ktab_t* T, int pz) { return T->zmin * ldexp(1.0, pz); }
static double kt_zhi(const ktab_t* T, int pz) {
  const double h = T->zmin * ldexp(1.0, pz + 1);
  return (pz == T->npz - 1 || h > T->zmax) ? T->zmax : h;
}

/* barycentric basis at local coordinate u in [-1, 1] */
static void kt_basis(const ktab_t* T, double u, double* l) {
  double s = 0.0;
  for (int j = 0; j < KT_NP; ++j) {
    const double du = u - T->xk[j];
    if (du == 0.0) {
      for (int i = 0; i < KT_NP; ++i) l[i] = (i == j) ? 1.0 : 0.0;
      return;
    }
    l[j] = T->wk[j] / du;
    s += l[j];
  }
  for (int j = 0; j < KT_NP; ++j) l[j] /= s;
}

static void kt_locate(const ktab_t* T, double rho, double zeta, int* pr, int* pz, double* lr, double* lz) {
  int a = (int)(rho / T->hr);
  if (a < 0) a = 0;
  if (a > T->npr - 1) a = T->npr - 1;
  int b = (int)floor(log2(zeta / T->zmin));
  if (b < 0) b = 0;
  if (b > T->npz - 1) b = T->npz - 1;
  kt_basis(T, 2.0 * (rho - a * T->hr) / T->hr - 1.0, lr);
  const double lo = kt_zlo(T, b), hi = kt_zhi(T, b);
  kt_basis(T, 2.0 * (zeta - lo) / (hi - lo) - 1.0, lz);
  *pr = a;
  *pz = b;
}

static double kt_eval(const ktab_t* T, int c, int pr, int pz, const double* lr, const double* lz) {
  const int nz = T->npz * KT_NP;
  const double* v = T->val + (size_t)c * (size_t)(T->npr * KT_NP) * nz;
  double acc = 0.0;
  for (int a = 0; a < KT_NP; ++a) {
    const double* row = v + (size_t)(pr * KT_NP + a) * nz + pz * KT_NP;
    double r = 0.0;
    for (int b = 0; b < KT_NP; ++b) r += lz[b] * row[b];
    acc += lr[a] * r;
  }
  return acc;
}

/* the shared rule applied to one (rho, zeta) of component c */
static double kt_direct(const rule_t* rule, const double* sg, double rho, double zeta) {
  double acc = 0.0, cmp = 0.0;
  for (int kk = 0; kk < rule->nn; ++kk) {
    const double f = rule->w[kk] * j0(rule->k[kk] * rho) * exp(-rule->k[kk] * zeta) * sg[kk];
    const double t = acc + f;
    if (fabs(acc) >= fabs(f)) cmp += (acc - t) + f; else cmp += (f - t) + acc;
    acc = t;
  }
  return (acc + cmp) / (4.0 * OR_PI);
}

/* valid[c] marks the components to tabulate; sig [comp][nn] from the rule */
static int kt_build(ktab_t* T, const rule_t* rule, const double* sig, const int* valid, int ncomp,
                    double rho_max, double zmin, double zmax) {
  T->val = NULL;
  T->cmax = NULL;
  if (!(zmin > 0.0) || !(zmax >= zmin)) return -5;
  T->npr = (int)ceil(rho_max / zmin);
  if (T->npr < 1) T->npr = 1;
  if (T->npr > KT_MAXPAN) return -5; /* pairs too close to an interface for a table: use quadrature */
  T->hr = (rho_max > 0.0 ? rho_max : zmin) / T->npr;
  T->zmin = zmin;
  T->zmax = zmax;
  T->npz = 1;
  while (T->zmin * ldexp(1.0, T->npz) < zmax) ++T->npz;
  for (int j = 0; j < KT_NP; ++j) {
    T->xk[j] = cos(OR_PI * j / KT_DEG);
    T->wk[j] = ((j & 1) ? -1.0 : 1.0) * ((j == 0 || j == KT_DEG) ? 0.5 : 1.0);
  }
  const int nr = T->npr * KT_NP, nz = T->npz * KT_NP, nn = rule->nn;
  double* rn = (double*)malloc(sizeof(double) * nr);
  double* zn = (double*)malloc(sizeof(double) * nz);
  double* J = (double*)malloc(sizeof(double) * (size_t)nr * nn);
  double* E = (double*)malloc(sizeof(double) * (size_t)nz * nn);
  T->val = (double*)calloc((size_t)ncomp * nr * nz, sizeof(double));
  T->cmax = (double*)calloc(ncomp, sizeof(double));
  if (!rn || !zn || !J || !E || !T->val || !T->cmax) {
    free(rn); free(zn); free(J); free(E);
    return -3;
  }
  for (int a = 0; a < T->npr; ++a)
    for (int j = 0; j < KT_NP; ++j) rn[a * KT_NP + j] = (a + 0.5 + 0.5 * T->xk[j]) * T->hr;
  for (int b = 0; b < T->npz; ++b) {
    const double lo = kt_zlo(T, b), hi = kt_zhi(T, b);
    for (int j = 0; j < KT_NP; ++j) zn[b * KT_NP + j] = 0.5 * (lo + hi) + 0.5 * (hi - lo) * T->xk[j];
  }
#pragma omp parallel for schedule(static)
  for (int i = 0; i < nr; ++i)
    for (int kk = 0; kk < nn; ++kk) J[(size_t)i * nn + kk] = rule->w[kk] * j0(rule->k[kk] * rn[i]);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < nz; ++i)
    for (int kk = 0; kk < nn; ++kk) E[(size_t)i * nn + kk] = exp(-rule->k[kk] * zn[i]);
  /* node values: K[c][i][j] = sum_k J[i][k] sigma_c[k] E[j][k] / (4 pi) */
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
  for (int c = 0; c < ncomp; ++c)
    for (int i = 0; i < nr; ++i) {
      if (!valid[c]) continue;
      const double* sg = sig + (size_t)c * nn;
      const double* Ji = J + (size_t)i * nn;
      double* out = T->val + ((size_t)c * nr + i) * nz;
      for (int j = 0; j < nz; ++j) {
        const double* Ej = E + (size_t)j * nn;
        double acc = 0.0;
        for (int kk = 0; kk < nn; ++kk) acc += Ji[kk] * sg[kk] * Ej[kk];
        out[j] = acc / (4.0 * OR_PI);
      }
    }
  free(rn); free(zn); free(J); free(E);
  for (int c = 0; c < ncomp; ++c) {
    if (!valid[c]) continue;
    const double* v = T->val + (size_t)c * nr * nz;
    for (size_t i = 0; i < (size_t)nr * nz; ++i)
      if (fabs(v[i]) > T->cmax[c]) T->cmax[c] = fabs(v[i]);
  }
  /* certification at seeded random points (a 64-bit linear congruential stream) */
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int c = 0; c < ncomp; ++c) {
    if (!valid[c]) continue;
    uint64_t st = 0x9E3779B97F4A7C15ull ^ (uint64_t)(c + 1);
    for (int t = 0; t < KT_CHECK; ++t) {
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      const double u1 = (double)(st >> 11) * 0x1.0p-53;
      st = st * 6364136223846793005ull + 1442695040888963407ull;
      const double u2 = (double)(st >> 11) * 0x1.0p-53;
      const double rho = u1 * T->npr * T->hr, zeta = zmin + u2 * (zmax - zmin);
      int pr, pz;
      double lr[KT_NP], lz[KT_NP];
      kt_locate(T, rho, zeta, &pr, &pz, lr, lz);
      const double got = kt_eval(T, c, pr, pz, lr, lz);
      const double ref = kt_direct(rule, sig + (size_t)c * nn, rho, zeta);
      if (!(fabs(got - ref) <= KT_TOL * T->cmax[c])) {
#pragma omp atomic write
        bad = 1;
      }
    }
  }
  return bad ? -5 : 0;
}

static void kt_free(ktab_t* T) {
  free(T->val);
  free(T->cmax);
}

/* ------------------------------------------------------------------------ */
/* Direct potential at selected targets.                                     */
/*   method 0: reaction kernels by quadrature (any number of layers)         */
/*   method 1: reaction kernels by the three-layer image series (L == 2)     */
/*   method 2: reaction kernels from certified tables (any number of layers) */
/*   parts   : bit 0 free space, bit 1 reaction                              */
/* Targets are indices into the N points; phi_out has nt entries.            */
/* ------------------------------------------------------------------------ */
/* Direct sum at the selected targets.  With mat_out non-null the pair values
 * themselves are stored as well, mat_out[ti * n + j] = the potential at
 * target ti of a unit charge at j (0 where no part applies); q may then be
 * NULL (unit charges). */
static int potential_impl(int L, const double* d, const double* acoef, const double* eps, int64_t n,
                          const double* x, const double* y, const double* z,
                          const int32_t* layer, const double* q, int64_t nt,
                          const int64_t* targets, int method, int parts,
                          double* phi_out, double* mat_out) {
  if (L < 1 || L > OR_MAXL) return -1;
  if (method == 1 && (L != 2 || acoef)) return -1;
  const int ncomp = (L + 1) * (L + 1) * 4;
  /* quadrature set-up: shared rule, sigma tabulated per component at nodes */
  rule_t rule = {0, NULL, NULL};
  double* sig = NULL;
  ktab_t ktab;
  memset(&ktab, 0, sizeof(ktab));
  double zeta_hi = 0.0, rho_span = 0.0;
  if ((parts & 2) && (method == 0 || method == 2)) {
    double rho_max = 0.0, zeta_min = INFINITY;
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    for (int64_t j = 0; j < n; ++j) {
      if (x[j] < xmin) xmin = x[j];
      if (x[j] > xmax) xmax = x[j];
      if (y[j] < ymin) ymin = y[j];
      if (y[j] > ymax) ymax = y[j];
      const int l = layer[j];
      if (l <= L - 1 && z[j] - d[l] < zeta_min) zeta_min = z[j] - d[l];
      if (l >= 1 && d[l - 1] - z[j] < zeta_min) zeta_min = d[l - 1] - z[j];
      if (l <= L - 1 && z[j] - d[l] > zeta_hi) zeta_hi = z[j] - d[l];
      if (l >= 1 && d[l - 1] - z[j] > zeta_hi) zeta_hi = d[l - 1] - z[j];
    }
    rho_max = hypot(xmax - xmin, ymax - ymin);
    rho_span = rho_max;
    zeta_hi *= 2.0;
    zeta_min *= 2.0; /* every exponent is a target part plus a source part */
    if (make_rule(rho_max, zeta_min, min_thickness(L, d), &rule)) return -3;
    sig = (double*)malloc(sizeof(double) * (size_t)ncomp * rule.nn);
    if (!sig) return -3;
    for (int i = 0; i < rule.nn; ++i)
      for (int lt = 0; lt <= L; ++lt)
        for (int ls = 0; ls <= L; ++ls) {
          double s4[4];
          oracle_sigma_ab(L, d, acoef, eps, lt, ls, rule.k[i], s4);
          for (int c = 0; c < 4; ++c)
            sig[(size_t)((lt * (L + 1) + ls) * 4 + c) * rule.nn + i] = s4[c];
        }
    if (method == 2) {
      int* valid = (int*)calloc(ncomp, sizeof(int));
      if (!valid) return -3;
      for (int lt = 0; lt <= L; ++lt)
        for (int ls = 0; ls <= L; ++ls)
          for (int a = 1; a <= 2; ++a)
            for (int b = 1; b <= 2; ++b)
              valid[(lt * (L + 1) + ls) * 4 + 2 * (a - 1) + (b - 1)] = valid_side(L, lt, a) && valid_side(L, ls, b);
      const int rc = kt_build(&ktab, &rule, sig, valid, ncomp, rho_span, zeta_min, zeta_hi);
      free(valid);
      if (rc) {
        kt_free(&ktab);
        free(sig);
        free_rule(&rule);
        return rc;
      }
    }
  }
  /* image-series coefficients per component */
  double* icoef = NULL;
  int* ishift = NULL;
  int* icnt = NULL;
  const int MAXT = 1200;
  if ((parts & 2) && method == 1) {
    icoef = (double*)malloc(sizeof(double) * ncomp * MAXT);
    ishift = (int*)malloc(sizeof(int) * ncomp * MAXT);
    icnt = (int*)calloc(ncomp, sizeof(int));
    if (!icoef || !ishift || !icnt) return -3;
    for (int lt = 0; lt <= L; ++lt)
      for (int ls = 0; ls <= L; ++ls)
        for (int a = 1; a <= 2; ++a)
          for (int b = 1; b <= 2; ++b) {
            const int c = (lt * (L + 1) + ls) * 4 + 2 * (a - 1) + (b - 1);
            if (valid_side(L, lt, a) && valid_side(L, ls, b))
              icnt[c] = oracle_image3_terms(eps, lt, ls, a, b, MAXT, icoef + c * MAXT,
                                            ishift + c * MAXT);
          }
  }
  const double D = (L == 2) ? d[0] - d[1] : 0.0;
  double* jbuf_all = NULL;
  int nthr = oracle_num_threads();
  if ((parts & 2) && method == 0) {
    jbuf_all = (double*)malloc(sizeof(double) * (size_t)rule.nn * nthr);
    if (!jbuf_all) return -3;
  }
  int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t ti = 0; ti < nt; ++ti) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    const int64_t i = targets[ti];
    if (i < 0 || i >= n) { err = -4; continue; }
    const double xi = x[i], yi = y[i], zi = z[i];
    const int li = layer[i];
    double fs = 0.0, fc = 0.0; /* free part, Neumaier */
    double rs = 0.0, rc = 0.0; /* reaction part, Neumaier */
    double* mrow = mat_out ? mat_out + ti * n : NULL;
    for (int64_t j = 0; j < n; ++j) {
      const double dx = xi - x[j], dy = yi - y[j];
      const int lj = layer[j];
      const double qj = q ? q[j] : 1.0;
      if (mrow) mrow[j] = 0.0;
      if ((parts & 1) && lj == li && j != i) {
        const double dz = zi - z[j];
        const double g = 1.0 / (4.0 * OR_PI * sqrt(dx * dx + dy * dy + dz * dz));
        if (mrow) mrow[j] += g;
        const double f = qj / (4.0 * OR_PI * sqrt(dx * dx + dy * dy + dz * dz));
        const double t = fs + f;
        if (fabs(fs) >= fabs(f)) fc += (fs - t) + f; else fc += (f - t) + fs;
        fs = t;
      }
      if (parts & 2) {
        const double rho = sqrt(dx * dx + dy * dy);
        double v = 0.0;
        if (method == 0) {
          double* jb = jbuf_all + (size_t)tid * rule.nn;
          for (int kk = 0; kk < rule.nn; ++kk) jb[kk] = rule.w[kk] * j0(rule.k[kk] * rho);
          for (int a = 1; a <= 2; ++a)
            for (int b = 1; b <= 2; ++b) {
              if (!valid_side(L, li, a) || !valid_side(L, lj, b)) continue;
              const double zeta = zeta_of(d, li, lj, a, b, zi, z[j]);
              const double* sg =
                  sig + (size_t)((li * (L + 1) + lj) * 4 + 2 * (a - 1) + (b - 1)) * rule.nn;
              double acc = 0.0;
              for (int kk = rule.nn - 1; kk >= 0; --kk)
                acc += jb[kk] * exp(-rule.k[kk] * zeta) * sg[kk];
              v += acc / (4.0 * OR_PI);
            }
        } else if (method == 2) {
          for (int a = 1; a <= 2; ++a)
            for (int b = 1; b <= 2; ++b) {
              if (!valid_side(L, li, a) || !valid_side(L, lj, b)) continue;
              const double zeta = zeta_of(d, li, lj, a, b, zi, z[j]);
              const int c = (li * (L + 1) + lj) * 4 + 2 * (a - 1) + (b - 1);
              int pr, pz;
              double lr[KT_NP], lz[KT_NP];
              kt_locate(&ktab, rho, zeta, &pr, &pz, lr, lz);
              v += kt_eval(&ktab, c, pr, pz, lr, lz);
            }
        } else {
          for (int a = 1; a <= 2; ++a)
            for (int b = 1; b <= 2; ++b) {
              if (!valid_side(L, li, a) || !valid_side(L, lj, b)) continue;
              const double zeta = zeta_of(d, li, lj, a, b, zi, z[j]);
              const int c = (li * (L + 1) + lj) * 4 + 2 * (a - 1) + (b - 1);
              double acc = 0.0;
              for (int t = icnt[c] - 1; t >= 0; --t) {
                const double zz = zeta + ishift[c * MAXT + t] * D;
                acc += icoef[c * MAXT + t] / sqrt(rho * rho + zz * zz);
              }
              v += acc / (4.0 * OR_PI);
            }
        }
        if (mrow) mrow[j] += v;
        const double f = qj * v;
        const double t = rs + f;
        if (fabs(rs) >= fabs(f)) rc += (rs - t) + f; else rc += (f - t) + rs;
        rs = t;
      }
    }
    phi_out[ti] = (fs + fc) + (rs + rc);
  }
  free(jbuf_all);
  kt_free(&ktab);
  free(sig);
  free_rule(&rule);
  free(icoef);
  free(ishift);
  free(icnt);
  return err;
}

int oracle_potential(int L, const double* d, const double* eps, int64_t n,
                     const double* x, const double* y, const double* z,
                     const int32_t* layer, const double* q, int64_t nt,
                     const int64_t* targets, int method, int parts,
                     double* phi_out) {
  return potential_impl(L, d, NULL, eps, n, x, y, z, layer, q, nt, targets, method, parts, phi_out, NULL);
}

/* The direct sum for the general interface conditions (coefficients a, b;
 * quadrature only). */
int oracle_potential_ab(int L, const double* d, const double* acoef, const double* bcoef, int64_t n,
                        const double* x, const double* y, const double* z,
                        const int32_t* layer, const double* q, int64_t nt,
                        const int64_t* targets, int parts, double* phi_out) {
  return potential_impl(L, d, acoef, bcoef, n, x, y, z, layer, q, nt, targets, 0, parts, phi_out, NULL);
}

/* The dense matrix of eq. totalinteraction: G[ti * n + j] is the potential at
 * target ti of a unit charge at j (free part for j != i in the same layer, the
 * reaction part for every j).  phi_scratch: nt doubles. */
int oracle_matrix(int L, const double* d, const double* eps, int64_t n,
                  const double* x, const double* y, const double* z,
                  const int32_t* layer, int64_t nt, const int64_t* targets,
                  int method, int parts, double* phi_scratch, double* G) {
  return potential_impl(L, d, NULL, eps, n, x, y, z, layer, NULL, nt, targets, method, parts, phi_scratch, G);
}
