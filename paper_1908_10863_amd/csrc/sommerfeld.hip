// Reaction densities and Sommerfeld-type integrals on the GPU (plan time).
//
// * Densities sigma^{ab}_{l l'}(k) of App. A at complex k: the interface
//   conditions (u and eps du/dz continuous) are resolved by the stable
//   generalized-reflection recursion (downward and upward reflection
//   coefficients seen through every layer stack, then transmission from the
//   source layer to the target layer), valid for Re k >= 0.
// * Initial values S^n I_{n,0} (n <= nmax) and S^n I_{n,1} (1 <= n <= nmax) of
//   eq. scaledsommerfeldint: composite Gauss-Legendre quadrature with panels
//   graded geometrically towards 0, along the real axis when rho <= z + zinf,
//   otherwise along the imaginary axis in the K_m form of eq. contourchange
//   (Sec. 3.4), zinf being the density's decay length (eq. densityasymptotic).
// * The remaining orders by the forward recurrence of eq. recurrence.
// * Reaction near-field kernels (1/4pi) I_{00} for particle pairs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "fmm_internal.h"

namespace fmmlm {
namespace {

constexpr int kGL = 16;
// The first panel [0, h0] is replaced by [0, h0 2^-Z] and [h0 2^-k, h0 2^-(k-1)],
// k = Z..1, which integrates the logarithmic singularity of K_0 at 0 to full accuracy.
constexpr int kZoom = 40;
__constant__ double c_glx[kGL];
__constant__ double c_glw[kGL];

// ---------------------------------------------------------------- densities
struct Scatter {
  double Rdn[kMaxL], Tdn[kMaxL], Rup[kMaxL], Tup[kMaxL];
};

__device__ void local_coeffs(const Medium& md, Scatter& sc) {
  for (int i = 0; i < md.L; ++i) {
    const double e0 = md.eps[i], e1 = md.eps[i + 1], s = e0 + e1;
    sc.Rdn[i] = (e0 - e1) / s;  // downgoing wave in layer i reflected at d_i
    sc.Tdn[i] = 2.0 * e0 / s;   // ... transmitted into layer i+1
    sc.Rup[i] = (e1 - e0) / s;  // upgoing wave in layer i+1 reflected at d_i
    sc.Tup[i] = 2.0 * e1 / s;   // ... transmitted into layer i
  }
}

// sigma^{ab}_{lt,ls}(k) of the classic conditions for md.eps; k complex with
// Re k >= 0.
__device__ cplx density_classic(const Medium& md, const Scatter& sc, int lt, int ls, int a, int b, cplx k) {
  const int L = md.L;
  // propagation factor across finite layer i (1 <= i <= L-1): e_i = exp(-k D_i)
  cplx e[kMaxL + 1], e2[kMaxL + 1];
  for (int i = 0; i <= L; ++i) {
    if (i >= 1 && i <= L - 1) {
      const double D = md.d[i - 1] - md.d[i];
      e[i] = cexp_dev(cmk(-k.re * D, -k.im * D));
    } else {
      e[i] = cmk(0.0, 0.0);
    }
    e2[i] = e[i] * e[i];
  }
  // generalized reflection looking down from layer i at d_i, and looking up
  // from layer i+1 at d_i
  cplx Gdn[kMaxL], Gup[kMaxL];
  Gdn[L - 1] = cmk(sc.Rdn[L - 1], 0.0);
  for (int i = L - 2; i >= 0; --i) {
    const cplx x = e2[i + 1] * Gdn[i + 1];
    const cplx num = (sc.Tdn[i] * sc.Tup[i]) * x;
    const cplx den = cmk(1.0, 0.0) - sc.Rup[i] * x;
    Gdn[i] = cmk(sc.Rdn[i], 0.0) + cdiv(num, den);
  }
  Gup[0] = cmk(sc.Rup[0], 0.0);
  for (int i = 1; i <= L - 1; ++i) {
    const cplx x = e2[i] * Gup[i - 1];
    const cplx num = (sc.Tup[i] * sc.Tdn[i]) * x;
    const cplx den = cmk(1.0, 0.0) - sc.Rdn[i] * x;
    Gup[i] = cmk(sc.Rup[i], 0.0) + cdiv(num, den);
  }
  // amplitudes in the source layer: u (upgoing at d_ls), w (downgoing at d_{ls-1})
  const cplx zero = cmk(0.0, 0.0), one = cmk(1.0, 0.0);
  const cplx Rd = (ls <= L - 1) ? Gdn[ls] : zero;
  const cplx Ru = (ls >= 1) ? Gup[ls - 1] : zero;
  const cplx es = e[ls];
  const cplx den = one - Rd * Ru * e2[ls];
  cplx u, w;
  if (b == 1) {
    u = cdiv(Rd, den);
    w = Ru * es * u;
  } else {
    w = cdiv(Ru, den);
    u = Rd * es * w;
  }
  if (lt == ls) return (a == 1) ? u : w;
  if (lt < ls) {
    // upgoing amplitude s1 at the bottom interface of each layer above the source
    cplx inc = (b == 2 ? one : zero) + es * u;  // upgoing at d_{ls-1} inside the source layer
    cplx s1 = zero;
    for (int i = ls - 1; i >= lt; --i) {
      const cplx g = (i >= 1) ? Gup[i - 1] : zero;
      const cplx dd = one - sc.Rdn[i] * (e2[i] * g);
      s1 = cdiv(sc.Tup[i] * inc, dd);
      inc = e[i] * s1;
    }
    if (a == 1) return s1;
    return (lt >= 1) ? Gup[lt - 1] * (e[lt] * s1) : zero;
  }
  // lt > ls: downgoing amplitude s2 at the top interface of each layer below
  cplx inc = (b == 1 ? one : zero) + es * w;  // downgoing at d_ls inside the source layer
  cplx s2 = zero;
  for (int i = ls + 1; i <= lt; ++i) {
    const cplx g = (i <= L - 1) ? Gdn[i] : zero;
    const cplx dd = one - sc.Rup[i - 1] * (e2[i] * g);
    s2 = cdiv(sc.Tdn[i - 1] * inc, dd);
    inc = e[i] * s2;
  }
  if (a == 2) return s2;
  return (lt <= L - 1) ? Gdn[lt] * (e[lt] * s2) : zero;
}

// sigma^{ab}_{lt,ls}(k) of the medium's interface conditions (factor a_ls / a_lt,
// exactly 1 for the classic conditions)
__device__ cplx density(const Medium& md, const Scatter& sc, int lt, int ls, int a, int b, cplx k) {
  if (md.L == 0) return cmk(1.0, 0.0);
  return (md.acoef[ls] / md.acoef[lt]) * density_classic(md, sc, lt, ls, a, b, k);
}

// ---------------------------------------------------------------- Bessel K_0, K_1
// K_m(x) = int_0^inf exp(-x cosh t) cosh(m t) dt (DLMF 10.32.9), trapezoidal
// rule with step 1/8: the integrand is analytic in |Im t| < pi/2 and decays
// double-exponentially, so the rule is accurate to roughly exp(-pi^2 / h).
__device__ void bessel_k01(double x, double* k0, double* k1) {
  const double h = 0.125;
  const double eh = exp(h);
  double E = 1.0;  // exp(t)
  double s0 = 0.5 * exp(-x), s1 = 0.5 * exp(-x);
  for (int i = 1; i < 4000; ++i) {
    E *= eh;
    const double ch = 0.5 * (E + 1.0 / E);
    const double f = exp(-x * ch);
    s0 += f;
    s1 += f * ch;
    if (x * ch > 745.0) break;
  }
  *k0 = h * s0;
  *k1 = h * s1;
}

// ---------------------------------------------------------------- quadrature
struct Panels {
  double h0, ratio, hmax, kmax;
};

// geometric grading from h0 (ratio 1.25) up to hmax, then uniform to kmax
__device__ inline double next_h(double h, const Panels& pn) {
  const double t = h * pn.ratio;
  return t < pn.hmax ? t : pn.hmax;
}

__device__ double min_thickness(const Medium& md) {
  double m = 0.0;
  for (int i = 1; i < md.L; ++i) {
    const double t = md.d[i - 1] - md.d[i];
    if (m == 0.0 || t < m) m = t;
  }
  return m;
}

__device__ double max_thickness(const Medium& md) {
  double m = 0.0;
  for (int i = 1; i < md.L; ++i) {
    const double t = md.d[i - 1] - md.d[i];
    if (t > m) m = t;
  }
  return m;
}

// amp S^n P~_n^m(Z/R) / R^{n+1}, R = sqrt(rho^2 + Z^2), added to o0[n] (m = 0,
// n <= nmax) and o1[n] (m = 1, 1 <= n <= nmax; o1 may be null).  This is the
// normalised integral of the density amp e^{-k Zi} at z = Z - Zi (Sec. 3.4:
// int_0^inf J_m(k rho) k^n e^{-k Z} dk = (n-m)! P_n^m(Z/R) / R^{n+1}, P_n^m without the
// Condon-Shortley phase), with P~_n^m = sqrt((n-m)!/(n+m)!) P_n^m.
__device__ void image_values(double amp, double S, double rho, double Z, int nmax, double* o0,
                             double* o1) {
  const double R = sqrt(rho * rho + Z * Z);
  const double x = Z / R, sn = rho / R, t = S / R;
  double pw = amp / R;
  double q0 = 0.0, p0 = 1.0;  // P_{n-1}^0, P_n^0
  double q1 = 0.0, p1 = sn;   // P_{n-1}^1, P_n^1 (n >= 1)
  for (int n = 0; n <= nmax; ++n) {
    o0[n] += pw * p0;
    if (o1 != nullptr && n >= 1) {
      o1[n] += pw * p1 / sqrt((double)n * (n + 1));
      const double r1 = ((2.0 * n + 1.0) * x * p1 - (n + 1.0) * q1) / n;
      q1 = p1;
      p1 = r1;
    }
    const double r0 = ((2.0 * n + 1.0) * x * p0 - n * q0) / (n + 1.0);
    q0 = p0;
    p0 = r0;
    pw *= t;
  }
}

// S^n I_{n,0} -> out0[n] (n <= nmax), S^n I_{n,1} -> out1[n] (1 <= n <= nmax).
// out1 may be null (only m = 0 wanted).  1/sqrt((n+m)!(n-m)!) included.
// The density's leading term sinf e^{-k zinf} (eq. densityasymptotic) is
// integrated in closed form by image_values; only the remainder
// sigma(k) - sinf e^{-k zinf}, which decays like e^{-k (zinf + 2 dmin)}, goes
// through the quadrature.  With one interface the remainder is zero.
__device__ void initial_values(const Medium& md, const Scatter& sc, const CompInfo& c, double S,
                               double rho, double z, int nmax, double* out0, double* out1,
                               bool with_image = true) {
  constexpr int kMaxN = 2 * kPMax + 1;
  const bool want1 = (out1 != nullptr) && rho > 0.0;
  for (int n = 0; n <= nmax; ++n) {
    out0[n] = 0.0;
    if (out1 != nullptr) out1[n] = 0.0;
  }
  if (with_image) image_values(c.sinf, S, rho, z + c.zinf, nmax, out0, want1 ? out1 : nullptr);
  if (md.L < 2) return;
  double acc0[kMaxN], acc1[kMaxN];
  for (int n = 0; n <= nmax; ++n) acc0[n] = acc1[n] = 0.0;
  const double dmin = min_thickness(md);
  const double zq = z + c.zinf + 2.0 * dmin;  // decay length of the remainder
  const bool contour = rho > zq;
  double small = 1.0;
  if (zq < small) small = zq;
  if (dmin < small) small = dmin;
  if (contour && rho < small) small = rho;
  Panels pn;
  pn.ratio = 1.25;
  pn.h0 = 1e-3 * small;
  if (!contour) {
    // real axis: J_m(k rho) (kS)^n e^{-kz} (sigma(k) - sinf e^{-k zinf})
    // panel widths are inverse lengths: the remainder decays on 1/zq (and
    // zq >= 2 dmin, so thin layers shrink it), J_m(k rho) oscillates on pi/rho
    pn.kmax = (2.0 * nmax + 50.0) / zq;
    double hmax = 2.0 / zq;
    if (rho > 0.0 && 3.14159265358979 / rho < hmax) hmax = 3.14159265358979 / rho;
    pn.hmax = hmax;
    double k0 = 0.0, h = pn.h0;
    int zoom = kZoom + 1;  // first panel [0, h0] split geometrically towards 0
    while (k0 < pn.kmax) {
      double a0 = k0, hh = h;
      if (zoom > 0) {
        hh = (zoom > kZoom) ? ldexp(pn.h0, -kZoom) : ldexp(pn.h0, -zoom);
        a0 = (zoom > kZoom) ? 0.0 : hh;
      }
      for (int g = 0; g < kGL; ++g) {
        const double k = a0 + 0.5 * hh * (c_glx[g] + 1.0);
        const double w = 0.5 * hh * c_glw[g];
        const double sg = density(md, sc, c.lt, c.ls, c.a, c.b, cmk(k, 0.0)).re - c.sinf * exp(-k * c.zinf);
        const double base = w * exp(-k * z) * sg;
        const double j0v = (rho > 0.0) ? j0(k * rho) : 1.0;
        const double j1v = want1 ? j1(k * rho) : 0.0;
        double pw = 1.0;  // (kS)^n
        const double ks = k * S;
        for (int n = 0; n <= nmax; ++n) {
          acc0[n] += base * j0v * pw;
          acc1[n] += base * j1v * pw;
          pw *= ks;
        }
      }
      if (zoom > 0) {
        --zoom;
        if (zoom > 0) continue;
      }
      k0 += h;
      h = next_h(h, pn);
    }
  } else {
    // imaginary axis: (2/pi) K_m(eta rho) (S eta)^n x {(-1)^{(n-m)/2} Re w, (-1)^{(n-m+1)/2} Im w},
    // w = e^{-i eta z} (sigma(i eta) - sinf e^{-i eta zinf})
    pn.kmax = (2.0 * nmax + 50.0) / rho;
    double hmax = 2.0 / rho;
    // sigma(i eta) does not decay along the imaginary axis: a wave reflected
    // through the whole stack oscillates like e^{-2 i eta (stack thickness)},
    // so the panels resolve two round trips through the stack (for three
    // layers the stack is the one finite layer)
    const double stack = md.L >= 2 ? md.d[0] - md.d[md.L - 1] : 0.0;
    const double osc = z + c.zinf + 4.0 * fmax(max_thickness(md), stack);
    if (3.14159265358979 / osc < hmax) hmax = 3.14159265358979 / osc;
    pn.hmax = hmax;
    double k0 = 0.0, h = pn.h0;
    int zoom = kZoom + 1;
    while (k0 < pn.kmax) {
      double a0 = k0, hh = h;
      if (zoom > 0) {
        hh = (zoom > kZoom) ? ldexp(pn.h0, -kZoom) : ldexp(pn.h0, -zoom);
        a0 = (zoom > kZoom) ? 0.0 : hh;
      }
      for (int g = 0; g < kGL; ++g) {
        const double et = a0 + 0.5 * hh * (c_glx[g] + 1.0);
        const double wq = 0.5 * hh * c_glw[g] * (2.0 / 3.14159265358979323846);
        cplx sg = density(md, sc, c.lt, c.ls, c.a, c.b, cmk(0.0, et));
        double sn, cs, si, ci;
        sincos(et * z, &sn, &cs);
        sincos(et * c.zinf, &si, &ci);
        sg.re -= c.sinf * ci;
        sg.im += c.sinf * si;
        const cplx wv = cmk(cs, -sn) * sg;
        double kk0, kk1;
        bessel_k01(et * rho, &kk0, &kk1);
        double pw = 1.0;
        const double es = et * S;
        for (int n = 0; n <= nmax; ++n) {
          // m = 0: n even -> (-1)^{n/2} Re w ; n odd -> (-1)^{(n+1)/2} Im w
          const double f0 = (n & 1) ? (((n + 1) / 2) & 1 ? -wv.im : wv.im)
                                    : ((n / 2) & 1 ? -wv.re : wv.re);
          acc0[n] += wq * kk0 * pw * f0;
          if (want1 && n >= 1) {
            // m = 1: n - 1 even -> (-1)^{(n-1)/2} Re w ; odd -> (-1)^{n/2} Im w
            const double f1 = ((n - 1) & 1) ? ((n / 2) & 1 ? -wv.im : wv.im)
                                            : (((n - 1) / 2) & 1 ? -wv.re : wv.re);
            acc1[n] += wq * kk1 * pw * f1;
          }
          pw *= es;
        }
      }
      if (zoom > 0) {
        --zoom;
        if (zoom > 0) continue;
      }
      k0 += h;
      h = next_h(h, pn);
    }
  }
  // normalisation 1/sqrt((n+m)!(n-m)!)
  double fn = 1.0;  // n!
  for (int n = 0; n <= nmax; ++n) {
    if (n > 0) fn *= n;
    out0[n] += acc0[n] / fn;
    // (n+1)! (n-1)! = n!^2 (n+1)/n
    if (want1 && n >= 1) out1[n] += acc1[n] / (fn * sqrt((n + 1.0) / n));
  }
}

// Orders M >= 2 of a table [cidx(n, m)] from M = 0, 1 by eq. recurrence.
__device__ void recurrence_fill(double S, double rho, int nmax, double* o) {
  // S^n I_{n,m+1} = (2m / a_{n+m}) (S / rho) S^{n-1} I_{n-1,m} - (a_{n-m} / a_{n+m}) S^n I_{n,m-1}
  for (int m = 1; m + 1 <= nmax; ++m) {
    for (int n = m + 1; n <= nmax; ++n) {
      double v = 0.0;
      if (rho > 0.0) {
        const double anpm = sqrt((double)(n + m) * (n + m + 1));
        const double anmm = sqrt((double)(n - m) * (n - m + 1));
        v = (2.0 * m / anpm) * (S / rho) * o[cidx(n - 1, m)] - (anmm / anpm) * o[cidx(n, m - 1)];
      }
      o[cidx(n, m + 1)] = v;
    }
  }
}

// One thread per task: initial values, then eq. recurrence for M >= 2.
__global__ void sommerfeld_table_kernel(Medium md, const CompInfo* __restrict__ comps,
                                        const SommTask* __restrict__ tasks, int ntask, int nmax,
                                        double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntask) return;
  Scatter sc;
  local_coeffs(md, sc);
  const SommTask tk = tasks[t];
  const CompInfo c = comps[tk.comp];
  constexpr int kMaxN = 2 * kPMax + 1;
  double i0[kMaxN], i1[kMaxN];
  initial_values(md, sc, c, tk.S, tk.rho, tk.z, nmax, i0, i1);
  double* o = out + (int64_t)t * ncoef(nmax);
  for (int n = 0; n <= nmax; ++n) {
    o[cidx(n, 0)] = i0[n];
    if (n >= 1) o[cidx(n, 1)] = i1[n];
  }
  recurrence_fill(tk.S, tk.rho, nmax, o);
}

__global__ void nearfield_kernel(Medium md, const CompInfo* __restrict__ comps,
                                 const int32_t* __restrict__ tpt, const int32_t* __restrict__ spt,
                                 const int32_t* __restrict__ cmp, int64_t npairs,
                                 const double* __restrict__ px, const double* __restrict__ py,
                                 const double* __restrict__ ph, double* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npairs) return;
  Scatter sc;
  local_coeffs(md, sc);
  const int32_t a = tpt[i], b = spt[i];
  const double dx = px[a] - px[b], dy = py[a] - py[b];
  const double rho = sqrt(dx * dx + dy * dy);
  const double zeta = ph[a] + ph[b];
  double v0;
  initial_values(md, sc, comps[cmp[i]], 1.0, rho, zeta, 0, &v0, nullptr);
  val[i] = v0 * (1.0 / (4.0 * 3.14159265358979323846));
}

// ---------------------------------------------------------------- learned form
// The density's remainder sigma(k) e^{k zinf} - sinf is approximated first by a
// ladder of exponentials sum_j c_j e^{-k j delta} (j = 1..kLadder, delta = 2 dmin,
// fitted once per component), each rung integrating in closed form like the
// leading term, as an image at zeta + zinf + j delta.  The network learns what
// the ladder leaves.
//
// Counter-based generator (splitmix64 finaliser of seed, stream and counter).
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ inline double rng_unit(uint64_t seed, uint64_t stream, uint64_t i) {
  const uint64_t z = mix64(seed ^ mix64(stream + 0x9E3779B97F4A7C15ull * (i + 1)));
  return (double)(z >> 11) * 0x1.0p-53;
}

// Adds sign * sum_j c_j S^n P~_n^m / R_j^{n+1} (rungs at Z + j delta) to o0, o1.
__device__ inline void ladder_values(const double* __restrict__ c, double delta, double sign, double S,
                                     double rho, double Z, int nmax, double* o0, double* o1) {
  for (int j = 0; j < kLadder; ++j)
    image_values(sign * c[j], S, rho, Z + (j + 1) * delta, nmax, o0, o1);
}

// Network inputs for one (component, rho, zeta): with Z2 = zeta + zinf + 2 dmin
// and R2 = |(rho, Z2)|, f = (2 rho/rho_max - 1, 2 zeta/zeta_max - 1,
// 2 Z2/R2 - 1, 4 dmin/R2 - 1).  Returns R2.
__device__ inline double surrogate_features(const SurrogateDomain& dm, double zinf, double rho,
                                            double zeta, float4* f) {
  const double Z2 = zeta + zinf + 2.0 * dm.dmin;
  const double R2 = sqrt(rho * rho + Z2 * Z2);
  f->x = (float)(2.0 * rho / dm.rho_max - 1.0);
  f->y = (float)(2.0 * zeta / dm.zeta_max - 1.0);
  f->z = (float)(2.0 * Z2 / R2 - 1.0);
  f->w = (float)(4.0 * dm.dmin / R2 - 1.0);
  return R2;
}

__device__ inline bool surrogate_in_domain(const SurrogateDomain& dm, double rho, double zeta) {
  return rho >= 0.0 && rho <= dm.rho_max && zeta > 0.0 && zeta <= dm.zeta_max;
}

// Training samples: component uniform; (rho, zeta) half uniform over the
// domain, half concentrated towards 0 (cubes of uniforms), where the
// reaction near field and the finest M2L levels sit.  Target of output j
// (degree n_j, order m_j: j <= nmax -> (j, 0), else (j - nmax, 1)) is what the
// leading term and the ladder leave of the initial value (S = 1), times
// kSurDecay^{n_j} R2^{n_j + 1} / yscale: the weights follow how fast an error
// of degree n fades in the M2L result (the scaled multipole moments of a box
// fall off like (0.87 S / R)^n, S <= R / 2).
__global__ void surrogate_sample_kernel(Medium md, const CompInfo* __restrict__ comps, int ncomp,
                                        const double* __restrict__ lad, SurrogateDomain dm, int nmax,
                                        uint64_t seed, int64_t n, int32_t* __restrict__ comp_out,
                                        float4* __restrict__ feat, float* __restrict__ y,
                                        double* __restrict__ rz) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Scatter sc;
  local_coeffs(md, sc);
  int c = (int)(rng_unit(seed, 1, i) * ncomp);
  if (c >= ncomp) c = ncomp - 1;
  double u = rng_unit(seed, 2, i), v = rng_unit(seed, 3, i);
  if (rng_unit(seed, 4, i) < 0.5) {
    u = u * u * u;
    v = v * v * v;
  }
  const double rho = u * dm.rho_max;
  const double zeta = fmax(v, 1e-6) * dm.zeta_max;
  const CompInfo ci = comps[c];
  float4 f;
  const double R2 = surrogate_features(dm, ci.zinf, rho, zeta, &f);
  constexpr int kMaxN = 2 * kPMax + 1;
  double i0[kMaxN], i1[kMaxN];
  initial_values(md, sc, ci, 1.0, rho, zeta, nmax, i0, i1, false);
  ladder_values(lad + (int64_t)c * kLadder, dm.delta, -1.0, 1.0, rho, zeta + ci.zinf, nmax, i0,
                rho > 0.0 ? i1 : nullptr);
  const int nout = 2 * nmax + 1;
  float* yo = y + i * nout;
  double pw = R2 / dm.yscale;  // kSurDecay^n R2^{n+1} / yscale
  for (int nn = 0; nn <= nmax; ++nn) {
    yo[nn] = (float)(i0[nn] * pw);
    if (nn >= 1) yo[nmax + nn] = (float)(i1[nn] * pw);
    pw *= R2 * kSurDecay;
  }
  comp_out[i] = c;
  feat[i] = f;
  if (rz) {
    rz[2 * i] = rho;
    rz[2 * i + 1] = zeta;
  }
}

// Features of the plan's Sommerfeld tasks (rho, z of a task are unscaled).
__global__ void surrogate_task_features_kernel(const CompInfo* __restrict__ comps,
                                               const int32_t* __restrict__ smap, SurrogateDomain dm,
                                               const SommTask* __restrict__ tasks, int ntask,
                                               int32_t* __restrict__ comp_out, float4* __restrict__ feat) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntask) return;
  const SommTask tk = tasks[t];
  float4 f;
  surrogate_features(dm, comps[tk.comp].zinf, tk.rho, tk.z, &f);
  comp_out[t] = smap[tk.comp];
  feat[t] = f;
}

// Initial values of a task inside the learned form's domain: the leading term
// and the ladder (lad: this component's rungs) in closed form plus the
// remainder S^n yscale rem(j) / (kSurDecay^n R2^{n+1}) for m = 0, 1, where
// rem(j) is output j in output units (j = n for m = 0, ynmax + n for m = 1).
template <class Rem>
__device__ void learned_task_values(const CompInfo& c, const double* __restrict__ lad, const SurrogateDomain& dm,
                                    const SommTask& tk, int nmax, int ynmax, Rem rem, double* i0, double* i1) {
  for (int n = 0; n <= nmax; ++n) i0[n] = i1[n] = 0.0;
  double* o1 = tk.rho > 0.0 ? i1 : nullptr;
  image_values(c.sinf, tk.S, tk.rho, tk.z + c.zinf, nmax, i0, o1);
  ladder_values(lad, dm.delta, 1.0, tk.S, tk.rho, tk.z + c.zinf, nmax, i0, o1);
  const double Z2 = tk.z + c.zinf + 2.0 * dm.dmin;
  const double R2 = sqrt(tk.rho * tk.rho + Z2 * Z2);
  double pw = dm.yscale / R2;  // yscale S^n / (kSurDecay^n R2^{n+1})
  for (int n = 0; n <= nmax; ++n) {
    i0[n] += pw * rem(n);
    if (n >= 1 && tk.rho > 0.0) i1[n] += pw * rem(ynmax + n);
    pw *= tk.S / (R2 * kSurDecay);
  }
}

// The learned form's near-field value I_00 (S = 1) without the 1/(4 pi): the
// closed-form parts plus yscale rem0 / R2.
__device__ inline double learned_pair_value(const CompInfo& c, const double* __restrict__ lad,
                                            const SurrogateDomain& dm, double rho, double zeta, double rem0) {
  double v0 = 0.0;
  image_values(c.sinf, 1.0, rho, zeta + c.zinf, 0, &v0, nullptr);
  ladder_values(lad, dm.delta, 1.0, 1.0, rho, zeta + c.zinf, 0, &v0, nullptr);
  const double Z2 = zeta + c.zinf + 2.0 * dm.dmin;
  return v0 + dm.yscale * rem0 / sqrt(rho * rho + Z2 * Z2);
}

// S^n I_{n,m} for a task: the leading term and the ladder in closed form plus
// the network's remainder S^n yscale y_j / (kSurDecay^n R2^{n+1}) (FP32
// network, FP64 here) for m = 0, 1; the quadrature when (rho, z) lies outside
// the trained domain; then eq. recurrence.
__global__ void surrogate_table_kernel(Medium md, const CompInfo* __restrict__ comps,
                                       const int32_t* __restrict__ scomp, const double* __restrict__ lad,
                                       SurrogateDomain dm, const SommTask* __restrict__ tasks, int ntask,
                                       int nmax, const float* __restrict__ y, int ldy, int ynmax,
                                       double* __restrict__ out, int32_t* __restrict__ used) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntask) return;
  const SommTask tk = tasks[t];
  const CompInfo c = comps[tk.comp];
  constexpr int kMaxN = 2 * kPMax + 1;
  double i0[kMaxN], i1[kMaxN];
  const bool net = surrogate_in_domain(dm, tk.rho, tk.z);
  if (net) {
    const float* yy = y + (int64_t)t * ldy;
    learned_task_values(c, lad + (int64_t)scomp[t] * kLadder, dm, tk, nmax, ynmax,
                        [&](int j) { return (double)yy[j]; }, i0, i1);
  } else {
    Scatter sc;
    local_coeffs(md, sc);
    initial_values(md, sc, c, tk.S, tk.rho, tk.z, nmax, i0, i1);
  }
  double* o = out + (int64_t)t * ncoef(nmax);
  for (int n = 0; n <= nmax; ++n) {
    o[cidx(n, 0)] = i0[n];
    if (n >= 1) o[cidx(n, 1)] = i1[n];
  }
  recurrence_fill(tk.S, tk.rho, nmax, o);
  if (used) used[t] = net ? 1 : 0;
}

// Reaction near field through the network: per pair (component, rho, zeta)
// and in-domain flag; out-of-domain pairs take the quadrature.
__global__ void surrogate_pair_features_kernel(const CompInfo* __restrict__ comps,
                                               const int32_t* __restrict__ smap, SurrogateDomain dm,
                                               const int32_t* __restrict__ tpt, const int32_t* __restrict__ spt,
                                               const int32_t* __restrict__ cmp, int64_t npairs,
                                               const double* __restrict__ px, const double* __restrict__ py,
                                               const double* __restrict__ ph, int32_t* __restrict__ comp_out,
                                               float4* __restrict__ feat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npairs) return;
  const int32_t a = tpt[i], b = spt[i];
  const double dx = px[a] - px[b], dy = py[a] - py[b];
  const double rho = sqrt(dx * dx + dy * dy);
  const double zeta = ph[a] + ph[b];
  float4 f;
  surrogate_features(dm, comps[cmp[i]].zinf, rho, zeta, &f);
  comp_out[i] = smap[cmp[i]];
  feat[i] = f;
}

__global__ void surrogate_nearfield_kernel(Medium md, const CompInfo* __restrict__ comps,
                                           const int32_t* __restrict__ scomp, const double* __restrict__ lad,
                                           SurrogateDomain dm, const int32_t* __restrict__ tpt,
                                           const int32_t* __restrict__ spt, const int32_t* __restrict__ cmp,
                                           int64_t npairs, const double* __restrict__ px,
                                           const double* __restrict__ py, const double* __restrict__ ph,
                                           const float* __restrict__ y, int ldy, double* __restrict__ val,
                                           unsigned long long* __restrict__ nfallback) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npairs) return;
  const int32_t a = tpt[i], b = spt[i];
  const double dx = px[a] - px[b], dy = py[a] - py[b];
  const double rho = sqrt(dx * dx + dy * dy);
  const double zeta = ph[a] + ph[b];
  const CompInfo c = comps[cmp[i]];
  double v0;
  if (surrogate_in_domain(dm, rho, zeta)) {
    v0 = learned_pair_value(c, lad + (int64_t)scomp[i] * kLadder, dm, rho, zeta, (double)y[i * ldy]);
  } else {
    Scatter sc;
    local_coeffs(md, sc);
    initial_values(md, sc, c, 1.0, rho, zeta, 0, &v0, nullptr);
    atomicAdd(nfallback, 1ull);
  }
  val[i] = v0 * (1.0 / (4.0 * 3.14159265358979323846));
}

// ---------------------------------------------------------------- table form
// Pre-computed 2-D tables for the initial values (the Remark after Table 3.1):
// per component, the remainder the network would learn (what the leading term
// and the ladder leave, times kSurDecay^n R2^{n+1}, a smooth O(1) function of
// (rho, zeta)) is tabulated on a grid of npr x npz panels over the domain, at
// kTabK Chebyshev points of the first kind per panel and direction, and
// interpolated by the barycentric formula (tensor product, degree kTabK - 1 in
// rho and in zeta: exact on polynomials of that degree).  Layout: component,
// panel (pr * npz + pz), output j, node (a * kTabK + b; a in rho, b in zeta).
__constant__ double c_chx[kTabK];  // cos((2k + 1) pi / (2 kTabK))
__constant__ double c_chw[kTabK];  // barycentric weights (-1)^k sin((2k + 1) pi / (2 kTabK))

// Lagrange basis values l[k] at x in [-1, 1] (barycentric formula; exact at nodes)
__device__ inline void cheb_lagrange(double x, double* l) {
  int hit = -1;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kTabK; ++k) {
    const double dx = x - c_chx[k];
    if (dx == 0.0) hit = k;
    const double t = c_chw[k] / (dx == 0.0 ? 1.0 : dx);
    l[k] = t;
    s += t;
  }
  if (hit >= 0) {
#pragma unroll
    for (int k = 0; k < kTabK; ++k) l[k] = (k == hit) ? 1.0 : 0.0;
    return;
  }
  const double is = 1.0 / s;
#pragma unroll
  for (int k = 0; k < kTabK; ++k) l[k] *= is;
}

// panel of (rho, zeta) (clamped to the grid) and the basis values in both directions
__device__ inline int table_cell(const TableGrid& g, double rho, double zeta, double* lr, double* lz) {
  int pr = (int)(rho / g.hr), pz = (int)(zeta / g.hz);
  pr = pr < 0 ? 0 : (pr >= g.npr ? g.npr - 1 : pr);
  pz = pz < 0 ? 0 : (pz >= g.npz ? g.npz - 1 : pz);
  cheb_lagrange(2.0 * (rho - pr * g.hr) / g.hr - 1.0, lr);
  cheb_lagrange(2.0 * (zeta - pz * g.hz) / g.hz - 1.0, lz);
  return pr * g.npz + pz;
}

// output j of a panel block [nout][kTabK * kTabK]
__device__ inline double table_value(const double* __restrict__ blk, int j, const double* lr, const double* lz) {
  const double* f = blk + (int64_t)j * kTabK * kTabK;
  double acc = 0.0;
#pragma unroll
  for (int a = 0; a < kTabK; ++a) {
    double r = 0.0;
#pragma unroll
    for (int b = 0; b < kTabK; ++b) r += lz[b] * f[a * kTabK + b];
    acc += lr[a] * r;
  }
  return acc;
}

// One thread per (component, panel, node): the remainder's scaled initial values
// by the quadrature (the same targets as the network's training samples).
__global__ void table_fill_kernel(Medium md, const CompInfo* __restrict__ comps, int ncomp,
                                  const double* __restrict__ lad, SurrogateDomain dm, TableGrid g, int nmax,
                                  double* __restrict__ tab) {
  constexpr int KK = kTabK * kTabK;
  const int64_t per = (int64_t)g.npr * g.npz * KK;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= per * ncomp) return;
  const int c = (int)(i / per);
  const int64_t r = i % per;
  const int cell = (int)(r / KK), ab = (int)(r % KK);
  const int pr = cell / g.npz, pz = cell % g.npz, a = ab / kTabK, b = ab % kTabK;
  const double rho = (pr + 0.5 + 0.5 * c_chx[a]) * g.hr;
  const double zeta = (pz + 0.5 + 0.5 * c_chx[b]) * g.hz;
  Scatter sc;
  local_coeffs(md, sc);
  const CompInfo ci = comps[c];
  constexpr int kMaxN = 2 * kPMax + 1;
  double i0[kMaxN], i1[kMaxN];
  initial_values(md, sc, ci, 1.0, rho, zeta, nmax, i0, i1, false);
  ladder_values(lad + (int64_t)c * kLadder, dm.delta, -1.0, 1.0, rho, zeta + ci.zinf, nmax, i0, i1);
  const double Z2 = zeta + ci.zinf + 2.0 * dm.dmin;
  const double R2 = sqrt(rho * rho + Z2 * Z2);
  const int nout = 2 * nmax + 1;
  double* blk = tab + ((int64_t)c * g.npr * g.npz + cell) * nout * KK;
  double pw = R2 / dm.yscale;  // kSurDecay^n R2^{n+1} / yscale
  for (int n = 0; n <= nmax; ++n) {
    blk[(int64_t)n * KK + ab] = i0[n] * pw;
    if (n >= 1) blk[(int64_t)(nmax + n) * KK + ab] = i1[n] * pw;
    pw *= R2 * kSurDecay;
  }
}

// S^n I_{n,m} of tasks through the tables (quadrature outside the domain), then eq. recurrence.
__global__ void table_task_kernel(Medium md, const CompInfo* __restrict__ comps, const int32_t* __restrict__ smap,
                                  const double* __restrict__ lad, SurrogateDomain dm, TableGrid g,
                                  const double* __restrict__ tab, int ynmax, const SommTask* __restrict__ tasks,
                                  int ntask, int nmax, double* __restrict__ out, int32_t* __restrict__ used) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntask) return;
  const SommTask tk = tasks[t];
  const CompInfo c = comps[tk.comp];
  constexpr int kMaxN = 2 * kPMax + 1;
  double i0[kMaxN], i1[kMaxN];
  const bool in = surrogate_in_domain(dm, tk.rho, tk.z);
  if (in) {
    const int sc = smap[tk.comp];
    double lr[kTabK], lz[kTabK];
    const int cell = table_cell(g, tk.rho, tk.z, lr, lz);
    const double* blk = tab + ((int64_t)sc * g.npr * g.npz + cell) * (2 * ynmax + 1) * kTabK * kTabK;
    learned_task_values(c, lad + (int64_t)sc * kLadder, dm, tk, nmax, ynmax,
                        [&](int j) { return table_value(blk, j, lr, lz); }, i0, i1);
  } else {
    Scatter scat;
    local_coeffs(md, scat);
    initial_values(md, scat, c, tk.S, tk.rho, tk.z, nmax, i0, i1);
  }
  double* o = out + (int64_t)t * ncoef(nmax);
  for (int n = 0; n <= nmax; ++n) {
    o[cidx(n, 0)] = i0[n];
    if (n >= 1) o[cidx(n, 1)] = i1[n];
  }
  recurrence_fill(tk.S, tk.rho, nmax, o);
  if (used) used[t] = in ? 1 : 0;
}

// Reaction near field through the tables (output 0, I_00); quadrature outside the domain.
__global__ void table_nearfield_kernel(Medium md, const CompInfo* __restrict__ comps,
                                       const int32_t* __restrict__ smap, const double* __restrict__ lad,
                                       SurrogateDomain dm, TableGrid g, const double* __restrict__ tab, int nout,
                                       const int32_t* __restrict__ tpt, const int32_t* __restrict__ spt,
                                       const int32_t* __restrict__ cmp, int64_t npairs,
                                       const double* __restrict__ px, const double* __restrict__ py,
                                       const double* __restrict__ ph, double* __restrict__ val,
                                       unsigned long long* __restrict__ nfallback) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npairs) return;
  const int32_t a = tpt[i], b = spt[i];
  const double dx = px[a] - px[b], dy = py[a] - py[b];
  const double rho = sqrt(dx * dx + dy * dy);
  const double zeta = ph[a] + ph[b];
  const CompInfo c = comps[cmp[i]];
  double v0;
  if (surrogate_in_domain(dm, rho, zeta)) {
    const int sc = smap[cmp[i]];
    double lr[kTabK], lz[kTabK];
    const int cell = table_cell(g, rho, zeta, lr, lz);
    const double* blk = tab + ((int64_t)sc * g.npr * g.npz + cell) * nout * kTabK * kTabK;
    v0 = learned_pair_value(c, lad + (int64_t)sc * kLadder, dm, rho, zeta, table_value(blk, 0, lr, lz));
  } else {
    Scatter sc;
    local_coeffs(md, sc);
    initial_values(md, sc, c, 1.0, rho, zeta, 0, &v0, nullptr);
    atomicAdd(nfallback, 1ull);
  }
  val[i] = v0 * (1.0 / (4.0 * 3.14159265358979323846));
}

// The interpolation alone on given node values (tests): out[i][j] for nout outputs.
__global__ void interp2d_kernel(TableGrid g, int nout, const double* __restrict__ nodes, int64_t n,
                                const double* __restrict__ rho, const double* __restrict__ zeta,
                                double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double lr[kTabK], lz[kTabK];
  const int cell = table_cell(g, rho[i], zeta[i], lr, lz);
  const double* blk = nodes + (int64_t)cell * nout * kTabK * kTabK;
  for (int j = 0; j < nout; ++j) out[i * nout + j] = table_value(blk, j, lr, lz);
}

__global__ void density_kernel(Medium md, CompInfo c, int64_t nk, const double* __restrict__ kre,
                               const double* __restrict__ kim, double* __restrict__ ore,
                               double* __restrict__ oim) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nk) return;
  Scatter sc;
  local_coeffs(md, sc);
  const cplx v = density(md, sc, c.lt, c.ls, c.a, c.b, cmk(kre[i], kim[i]));
  ore[i] = v.re;
  oim[i] = v.im;
}

// Gauss-Legendre nodes on [-1, 1] (Newton on the three-term recurrence), host side.
void gl_nodes(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int j = 2; j <= n; ++j) {
        const double p2 = ((2.0 * j - 1.0) * t * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      const double dp = n * (t * p1 - p0) / (t * t - 1.0);
      const double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double p0 = 1.0, p1 = t;
    for (int j = 2; j <= n; ++j) {
      const double p2 = ((2.0 * j - 1.0) * t * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    const double dp = n * (t * p1 - p0) / (t * t - 1.0);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
}

// The node table lives in constant memory, one copy per device: it is
// written once on each device the library runs on.
constexpr int kMaxDevices = 64;
int upload_gl(hipStream_t st) {
  static std::mutex mu;
  static bool done[kMaxDevices] = {};
  (void)st;
  int dev = 0;
  FMM_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return FMMLM_EDEVICE;
  std::lock_guard<std::mutex> lk(mu);
  if (done[dev]) return FMMLM_OK;
  double x[kGL], w[kGL];
  gl_nodes(kGL, x, w);
  FMM_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_glx), x, sizeof(x)));
  FMM_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_glw), w, sizeof(w)));
  double cx[kTabK], cw[kTabK];
  for (int k = 0; k < kTabK; ++k) {
    const double th = M_PI * (2.0 * k + 1.0) / (2.0 * kTabK);
    cx[k] = std::cos(th);
    cw[k] = ((k & 1) ? -1.0 : 1.0) * std::sin(th);
  }
  FMM_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_chx), cx, sizeof(cx)));
  FMM_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(c_chw), cw, sizeof(cw)));
  done[dev] = true;
  return FMMLM_OK;
}

// ---------------------------------------------------------------- allocation-free form
// fmm_layered_sommerfeld_noalloc stages its component and per-point tasks in
// `scratch`, a file-scope device array (each device holds its own copy for the
// life of the process), instead of buffers allocated per call.  Host code
// never passes the array's name to a kernel or a copy: it asks the runtime for
// the array's device address once per device (noalloc_scratch) and uses that.
constexpr size_t kNoAllocCompBytes = 256;  // the CompInfo, padded to keep the tasks aligned
constexpr size_t kNoAllocBytes = kNoAllocCompBytes + (size_t)FMMLM_NOALLOC_MAX_POINTS * sizeof(SommTask);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
static_assert(sizeof(CompInfo) <= kNoAllocCompBytes, "component does not fit its scratch slot");

// Device address of this device's scratch array (looked up once per device).
int noalloc_scratch(unsigned char** out) {
  static std::mutex mu;
  static unsigned char* ptr[kMaxDevices] = {};
  int dev = 0;
  FMM_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return FMMLM_EDEVICE;
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    FMM_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return FMMLM_EDEVICE;
    ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = ptr[dev];
  return FMMLM_OK;
}

// Stages the component and one task per point.  A point with rho < 0, z <= 0
// or a non-finite value gets a harmless task (rho = 0, z = 1, so the
// quadrature stays bounded); noalloc_mark_kernel then writes NaN over its
// outputs.
__device__ inline bool noalloc_valid(double r, double zz) {
  return (r >= 0.0) && (zz > 0.0) && isfinite(r) && isfinite(zz);
}

__global__ void noalloc_tasks_kernel(CompInfo c, double S, const double* __restrict__ rho,
                                     const double* __restrict__ z, int64_t n, CompInfo* __restrict__ comp,
                                     SommTask* __restrict__ tasks) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *comp = c;
  if (i >= n) return;
  const double r = rho[i], zz = z[i];
  tasks[i] = noalloc_valid(r, zz) ? SommTask{0, S, r, zz} : SommTask{0, S, 0.0, 1.0};
}

__global__ void noalloc_mark_kernel(const double* __restrict__ rho, const double* __restrict__ z, int64_t n,
                                    int per, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || noalloc_valid(rho[i], z[i])) return;
  for (int j = 0; j < per; ++j) out[i * per + j] = __builtin_nan("");
}

}  // namespace

// Shortest ray path from the source's exit interface to the target's entry
// interface: the density decays like exp(-k zinf) (eq. densityasymptotic).
double zeta_inf(const Medium& md, int lt, int ls, int a, int b) {
  if (md.L == 0) return 0.0;
  auto D = [&](int l) { return (l >= 1 && l <= md.L - 1) ? md.d[l - 1] - md.d[l] : 0.0; };
  if (lt == ls) return (a == b) ? 0.0 : D(lt);
  if (lt < ls) return (b == 1 ? D(ls) : 0.0) + (md.d[lt] - md.d[ls - 1]) + (a == 2 ? D(lt) : 0.0);
  return (b == 2 ? D(ls) : 0.0) + (md.d[ls] - md.d[lt - 1]) + (a == 1 ? D(lt) : 0.0);
}

// Amplitude of the leading term of the density: the product of the local
// reflection and transmission coefficients met along the shortest ray path of
// zeta_inf (every other path crosses some finite layer twice more, so
// sigma(k) e^{k zinf} - sinf = O(e^{-2 k dmin})).
static double sigma_inf_classic(const Medium& md, int lt, int ls, int a, int b) {
  auto rdn = [&](int i) { return (md.eps[i] - md.eps[i + 1]) / (md.eps[i] + md.eps[i + 1]); };
  auto rup = [&](int i) { return (md.eps[i + 1] - md.eps[i]) / (md.eps[i] + md.eps[i + 1]); };
  auto tdn = [&](int i) { return 2.0 * md.eps[i] / (md.eps[i] + md.eps[i + 1]); };
  auto tup = [&](int i) { return 2.0 * md.eps[i + 1] / (md.eps[i] + md.eps[i + 1]); };
  if (lt == ls) {
    if (a == b) return (b == 1) ? rdn(ls) : rup(ls - 1);
    return rdn(ls) * rup(ls - 1);
  }
  if (lt < ls) {
    double s = (b == 2) ? 1.0 : rdn(ls);  // b = 1: down to d_ls and back up first
    for (int i = ls - 1; i >= lt; --i) s *= tup(i);
    return (a == 1) ? s : rup(lt - 1) * s;
  }
  double s = (b == 1) ? 1.0 : rup(ls - 1);
  for (int i = ls + 1; i <= lt; ++i) s *= tdn(i - 1);
  return (a == 2) ? s : rdn(lt) * s;
}

double sigma_inf(const Medium& md, int lt, int ls, int a, int b) {
  if (md.L == 0) return 1.0;
  return (md.acoef[ls] / md.acoef[lt]) * sigma_inf_classic(md, lt, ls, a, b);
}

int gpu_sommerfeld_tables(const Medium& md, const std::vector<CompInfo>& comps,
                          const std::vector<SommTask>& tasks, int nmax, double* d_out,
                          hipStream_t st) {
  if (tasks.empty()) return FMMLM_OK;
  int rc = upload_gl(st);
  if (rc) return rc;
  CompInfo* dc = nullptr;
  SommTask* dt = nullptr;
  FMM_HIP_TRY(hipMalloc(&dc, comps.size() * sizeof(CompInfo)));
  FMM_HIP_TRY(hipMalloc(&dt, tasks.size() * sizeof(SommTask)));
  FMM_HIP_TRY(hipMemcpyAsync(dc, comps.data(), comps.size() * sizeof(CompInfo), hipMemcpyHostToDevice, st));
  FMM_HIP_TRY(hipMemcpyAsync(dt, tasks.data(), tasks.size() * sizeof(SommTask), hipMemcpyHostToDevice, st));
  const int nt = (int)tasks.size();
  sommerfeld_table_kernel<<<(nt + 63) / 64, 64, 0, st>>>(md, dc, dt, nt, nmax, d_out);
  FMM_HIP_TRY(hipGetLastError());
  FMM_HIP_TRY(hipStreamSynchronize(st));
  hipFree(dc);
  hipFree(dt);
  return FMMLM_OK;
}

int gpu_reaction_nearfield(const Medium& md, const std::vector<CompInfo>& comps,
                           const int32_t* d_tpt, const int32_t* d_spt, const int32_t* d_comp,
                           int64_t npairs, const double* px, const double* py, const double* ph,
                           double* d_val, hipStream_t st) {
  if (npairs == 0) return FMMLM_OK;
  int rc = upload_gl(st);
  if (rc) return rc;
  CompInfo* dc = nullptr;
  FMM_HIP_TRY(hipMalloc(&dc, comps.size() * sizeof(CompInfo)));
  FMM_HIP_TRY(hipMemcpyAsync(dc, comps.data(), comps.size() * sizeof(CompInfo), hipMemcpyHostToDevice, st));
  nearfield_kernel<<<(unsigned)((npairs + 63) / 64), 64, 0, st>>>(md, dc, d_tpt, d_spt, d_comp, npairs,
                                                                  px, py, ph, d_val);
  FMM_HIP_TRY(hipGetLastError());
  FMM_HIP_TRY(hipStreamSynchronize(st));
  hipFree(dc);
  return FMMLM_OK;
}

int gpu_density(const Medium& md, const CompInfo& c, int64_t nk, const double* kre,
                const double* kim, double* ore, double* oim, hipStream_t st) {
  double* buf = nullptr;
  FMM_HIP_TRY(hipMalloc(&buf, 4 * nk * sizeof(double)));
  FMM_HIP_TRY(hipMemcpyAsync(buf, kre, nk * 8, hipMemcpyHostToDevice, st));
  FMM_HIP_TRY(hipMemcpyAsync(buf + nk, kim, nk * 8, hipMemcpyHostToDevice, st));
  density_kernel<<<(unsigned)((nk + 63) / 64), 64, 0, st>>>(md, c, nk, buf, buf + nk, buf + 2 * nk,
                                                            buf + 3 * nk);
  FMM_HIP_TRY(hipGetLastError());
  FMM_HIP_TRY(hipMemcpyAsync(ore, buf + 2 * nk, nk * 8, hipMemcpyDeviceToHost, st));
  FMM_HIP_TRY(hipMemcpyAsync(oim, buf + 3 * nk, nk * 8, hipMemcpyDeviceToHost, st));
  FMM_HIP_TRY(hipStreamSynchronize(st));
  hipFree(buf);
  return FMMLM_OK;
}

int gpu_surrogate_samples(const Medium& md, const std::vector<CompInfo>& comps, const double* d_lad,
                          const SurrogateDomain& dm, int nmax, uint64_t seed, int64_t n, int32_t* d_comp,
                          float* d_feat, float* d_y, hipStream_t st, double* d_rz) {
  if (n == 0) return FMMLM_OK;
  int rc = upload_gl(st);
  if (rc) return rc;
  CompInfo* dc = nullptr;
  FMM_HIP_TRY(hipMalloc(&dc, comps.size() * sizeof(CompInfo)));
  FMM_HIP_TRY(hipMemcpyAsync(dc, comps.data(), comps.size() * sizeof(CompInfo), hipMemcpyHostToDevice, st));
  surrogate_sample_kernel<<<(unsigned)((n + 63) / 64), 64, 0, st>>>(
      md, dc, (int)comps.size(), d_lad, dm, nmax, seed, n, d_comp, reinterpret_cast<float4*>(d_feat), d_y, d_rz);
  FMM_HIP_TRY(hipGetLastError());
  FMM_HIP_TRY(hipStreamSynchronize(st));
  hipFree(dc);
  return FMMLM_OK;
}

int gpu_surrogate_tables(const Medium& md, const std::vector<CompInfo>& comps,
                         const std::vector<int32_t>& smap, const double* d_lad, const SurrogateDomain& dm,
                         const std::vector<SommTask>& tasks, int nmax, const MlpNet& net, double* d_out,
                         int64_t* n_used, hipStream_t st, int32_t* h_used) {
  *n_used = 0;
  if (tasks.empty()) return FMMLM_OK;
  int rc = upload_gl(st);
  if (rc) return rc;
  const int nt = (int)tasks.size();
  const int ynmax = (net.nout - 1) / 2;
  CompInfo* dc = nullptr;
  SommTask* dt = nullptr;
  int32_t *dmap = nullptr, *dcomp = nullptr, *dused = nullptr;
  float *dfeat = nullptr, *dy = nullptr;
  FMM_HIP_TRY(hipMalloc(&dc, comps.size() * sizeof(CompInfo)));
  FMM_HIP_TRY(hipMalloc(&dt, tasks.size() * sizeof(SommTask)));
  FMM_HIP_TRY(hipMalloc(&dmap, smap.size() * sizeof(int32_t)));
  FMM_HIP_TRY(hipMalloc(&dcomp, nt * sizeof(int32_t)));
  FMM_HIP_TRY(hipMalloc(&dused, nt * sizeof(int32_t)));
  FMM_HIP_TRY(hipMalloc(&dfeat, (size_t)nt * 4 * sizeof(float)));
  FMM_HIP_TRY(hipMalloc(&dy, (size_t)nt * net.nout * sizeof(float)));
  FMM_HIP_TRY(hipMemcpyAsync(dc, comps.data(), comps.size() * sizeof(CompInfo), hipMemcpyHostToDevice, st));
  FMM_HIP_TRY(hipMemcpyAsync(dt, tasks.data(), tasks.size() * sizeof(SommTask), hipMemcpyHostToDevice, st));
  FMM_HIP_TRY(hipMemcpyAsync(dmap, smap.data(), smap.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  surrogate_task_features_kernel<<<(nt + 63) / 64, 64, 0, st>>>(dc, dmap, dm, dt, nt, dcomp,
                                                                reinterpret_cast<float4*>(dfeat));
  FMM_HIP_TRY(hipGetLastError());
  rc = gpu_mlp_forward(net, dcomp, dfeat, nt, dy, net.nout, net.nout, nullptr, nullptr, nullptr, st);
  if (rc == FMMLM_OK) {
    surrogate_table_kernel<<<(nt + 63) / 64, 64, 0, st>>>(md, dc, dcomp, d_lad, dm, dt, nt, nmax, dy, net.nout,
                                                          ynmax, d_out, dused);
    FMM_HIP_TRY(hipGetLastError());
    std::vector<int32_t> used(nt);
    FMM_HIP_TRY(hipMemcpyAsync(used.data(), dused, nt * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FMM_HIP_TRY(hipStreamSynchronize(st));
    for (int32_t u : used) *n_used += u;
    if (h_used) std::copy(used.begin(), used.end(), h_used);
  }
  hipFree(dc);
  hipFree(dt);
  hipFree(dmap);
  hipFree(dcomp);
  hipFree(dused);
  hipFree(dfeat);
  hipFree(dy);
  return rc;
}

int gpu_surrogate_nearfield(const Medium& md, const std::vector<CompInfo>& comps,
                            const std::vector<int32_t>& smap, const double* d_lad, const SurrogateDomain& dm,
                            const int32_t* d_tpt, const int32_t* d_spt, const int32_t* d_comp,
                            int64_t npairs, const double* px, const double* py, const double* ph,
                            const MlpNet& net, double* d_val, int64_t* n_fallback, hipStream_t st) {
  *n_fallback = 0;
  if (npairs == 0) return FMMLM_OK;
  int rc = upload_gl(st);
  if (rc) return rc;
  constexpr int64_t kChunk = (int64_t)1 << 22;
  const int64_t cap = std::min(npairs, kChunk);
  CompInfo* dc = nullptr;
  int32_t *dmap = nullptr, *dcomp = nullptr;
  float *dfeat = nullptr, *dy = nullptr;
  unsigned long long* dfb = nullptr;
  FMM_HIP_TRY(hipMalloc(&dc, comps.size() * sizeof(CompInfo)));
  FMM_HIP_TRY(hipMalloc(&dmap, smap.size() * sizeof(int32_t)));
  FMM_HIP_TRY(hipMalloc(&dcomp, cap * sizeof(int32_t)));
  FMM_HIP_TRY(hipMalloc(&dfeat, cap * 4 * sizeof(float)));
  FMM_HIP_TRY(hipMalloc(&dy, cap * sizeof(float)));
  FMM_HIP_TRY(hipMalloc(&dfb, sizeof(unsigned long long)));
  FMM_HIP_TRY(hipMemcpyAsync(dc, comps.data(), comps.size() * sizeof(CompInfo), hipMemcpyHostToDevice, st));
  FMM_HIP_TRY(hipMemcpyAsync(dmap, smap.data(), smap.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
  FMM_HIP_TRY(hipMemsetAsync(dfb, 0, sizeof(unsigned long long), st));
  for (int64_t o = 0; o < npairs && rc == FMMLM_OK; o += kChunk) {
    const int64_t m = std::min(kChunk, npairs - o);
    const unsigned nb = (unsigned)((m + 255) / 256);
    surrogate_pair_features_kernel<<<nb, 256, 0, st>>>(dc, dmap, dm, d_tpt + o, d_spt + o, d_comp + o, m,
                                                       px, py, ph, dcomp, reinterpret_cast<float4*>(dfeat));
    FMM_HIP_TRY(hipGetLastError());
    rc = gpu_mlp_forward(net, dcomp, dfeat, m, dy, 1, 1, nullptr, nullptr, nullptr, st);
    if (rc) break;
    surrogate_nearfield_kernel<<<nb, 256, 0, st>>>(md, dc, dcomp, d_lad, dm, d_tpt + o, d_spt + o, d_comp + o, m,
                                                   px, py, ph, dy, 1, d_val + o, dfb);
    FMM_HIP_TRY(hipGetLastError());
  }
  unsigned long long fb = 0;
  if (rc == FMMLM_OK) {
    FMM_HIP_TRY(hipMemcpyAsync(&fb, dfb, sizeof(fb), hipMemcpyDeviceToHost, st));
    FMM_HIP_TRY(hipStreamSynchronize(st));
  }
  *n_fallback = (int64_t)fb;
  hipFree(dc);
  hipFree(dmap);
  hipFree(dcomp);
  hipFree(dfeat);
  hipFree(dy);
  hipFree(dfb);
  return rc;
}

// ---- table form (host side)
int gpu_table_fill(const Medium& md, const std::vector<CompInfo>& comps, const double* d_lad,
                   const SurrogateDomain& dm, const TableGrid& g, int nmax, double* d_tab, hipStream_t st) {
  int rc = upload_gl(st);
  if (rc) return rc;
  CompInfo* dc = nullptr;
  FMM_HIP_TRY(hipMalloc(&dc, comps.size() * sizeof(CompInfo)));
  FMM_HIP_TRY(hipMemcpyAsync(dc, comps.data(), comps.size() * sizeof(CompInfo), hipMemcpyHostToDevice, st));
  const int64_t n = (int64_t)comps.size() * g.npr * g.npz * kTabK * kTabK;
  table_fill_kernel<<<(unsigned)((n + 63) / 64), 64, 0, st>>>(md, dc, (int)comps.size(), d_lad, dm, g, nmax, d_tab);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipFree(dc);
  if (e != hipSuccess) {
    set_last_error(std::string("table fill: ") + hipGetErrorString(e));
    return FMMLM_EDEVICE;
  }
  return FMMLM_OK;
}

int gpu_table_tasks(const Medium& md, const std::vector<CompInfo>& comps, const std::vector<int32_t>& smap,
                    const double* d_lad, const SurrogateDomain& dm, const TableGrid& g, const double* d_tab,
                    int ynmax, const std::vector<SommTask>& tasks, int nmax, double* d_out, int64_t* n_used,
                    hipStream_t st, int32_t* h_used) {
  *n_used = 0;
  if (tasks.empty()) return FMMLM_OK;
  int rc = upload_gl(st);
  if (rc) return rc;
  const int nt = (int)tasks.size();
  CompInfo* dc = nullptr;
  SommTask* dt = nullptr;
  int32_t *dmap = nullptr, *dused = nullptr;
  hipError_t e = hipMalloc(&dc, comps.size() * sizeof(CompInfo));
  if (e == hipSuccess) e = hipMalloc(&dt, tasks.size() * sizeof(SommTask));
  if (e == hipSuccess) e = hipMalloc(&dmap, smap.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&dused, nt * sizeof(int32_t));
  if (e == hipSuccess)
    e = hipMemcpyAsync(dc, comps.data(), comps.size() * sizeof(CompInfo), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dt, tasks.data(), tasks.size() * sizeof(SommTask), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dmap, smap.data(), smap.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
  std::vector<int32_t> used(nt);
  if (e == hipSuccess) {
    table_task_kernel<<<(nt + 63) / 64, 64, 0, st>>>(md, dc, dmap, d_lad, dm, g, d_tab, ynmax, dt, nt, nmax, d_out,
                                                     dused);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(used.data(), dused, nt * sizeof(int32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipFree(dc);
  hipFree(dt);
  hipFree(dmap);
  hipFree(dused);
  if (e != hipSuccess) {
    set_last_error(std::string("table tasks: ") + hipGetErrorString(e));
    return FMMLM_EDEVICE;
  }
  for (int32_t u : used) *n_used += u;
  if (h_used) std::copy(used.begin(), used.end(), h_used);
  return FMMLM_OK;
}

int gpu_table_nearfield(const Medium& md, const std::vector<CompInfo>& comps, const std::vector<int32_t>& smap,
                        const double* d_lad, const SurrogateDomain& dm, const TableGrid& g, const double* d_tab,
                        int nout, const int32_t* d_tpt, const int32_t* d_spt, const int32_t* d_comp, int64_t npairs,
                        const double* px, const double* py, const double* ph, double* d_val, int64_t* n_fallback,
                        hipStream_t st) {
  *n_fallback = 0;
  if (npairs == 0) return FMMLM_OK;
  int rc = upload_gl(st);
  if (rc) return rc;
  CompInfo* dc = nullptr;
  int32_t* dmap = nullptr;
  unsigned long long* dfb = nullptr;
  hipError_t e = hipMalloc(&dc, comps.size() * sizeof(CompInfo));
  if (e == hipSuccess) e = hipMalloc(&dmap, smap.size() * sizeof(int32_t));
  if (e == hipSuccess) e = hipMalloc(&dfb, sizeof(unsigned long long));
  if (e == hipSuccess)
    e = hipMemcpyAsync(dc, comps.data(), comps.size() * sizeof(CompInfo), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dmap, smap.data(), smap.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(dfb, 0, sizeof(unsigned long long), st);
  unsigned long long fb = 0;
  if (e == hipSuccess) {
    table_nearfield_kernel<<<(unsigned)((npairs + 255) / 256), 256, 0, st>>>(
        md, dc, dmap, d_lad, dm, g, d_tab, nout, d_tpt, d_spt, d_comp, npairs, px, py, ph, d_val, dfb);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&fb, dfb, sizeof(fb), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  hipFree(dc);
  hipFree(dmap);
  hipFree(dfb);
  if (e != hipSuccess) {
    set_last_error(std::string("table near field: ") + hipGetErrorString(e));
    return FMMLM_EDEVICE;
  }
  *n_fallback = (int64_t)fb;
  return FMMLM_OK;
}

int gpu_interp2d(const TableGrid& g, int nout, const double* d_nodes, int64_t n, const double* d_rho,
                 const double* d_zeta, double* d_out, hipStream_t st) {
  int rc = upload_gl(st);
  if (rc) return rc;
  interp2d_kernel<<<(unsigned)((n + 63) / 64), 64, 0, st>>>(g, nout, d_nodes, n, d_rho, d_zeta, d_out);
  FMM_HIP_TRY(hipGetLastError());
  return FMMLM_OK;
}

// S^N I_{N,M} for device arrays rho, z of npts points into out (device),
// asynchronous on st, with no allocation: the per-call staging goes to this
// device's scratch array.  npts <= FMMLM_NOALLOC_MAX_POINTS (checked by the caller).
int gpu_sommerfeld_noalloc(const Medium& md, const CompInfo& c, double S, int64_t npts, const double* rho,
                           const double* z, int nmax, double* out, hipStream_t st) {
  if (npts < 1 || npts > FMMLM_NOALLOC_MAX_POINTS) return FMMLM_EINVAL;
  int rc = upload_gl(st);
  if (rc) return rc;
  unsigned char* base = nullptr;
  if ((rc = noalloc_scratch(&base))) return rc;
  CompInfo* dcomp = reinterpret_cast<CompInfo*>(base);
  SommTask* dtask = reinterpret_cast<SommTask*>(base + kNoAllocCompBytes);
  const unsigned nb = (unsigned)((npts + 63) / 64);
  noalloc_tasks_kernel<<<nb, 64, 0, st>>>(c, S, rho, z, npts, dcomp, dtask);
  FMM_HIP_TRY(hipGetLastError());
  sommerfeld_table_kernel<<<nb, 64, 0, st>>>(md, dcomp, dtask, (int)npts, nmax, out);
  FMM_HIP_TRY(hipGetLastError());
  noalloc_mark_kernel<<<nb, 64, 0, st>>>(rho, z, npts, ncoef(nmax), out);
  FMM_HIP_TRY(hipGetLastError());
  return FMMLM_OK;
}

}  // namespace fmmlm
