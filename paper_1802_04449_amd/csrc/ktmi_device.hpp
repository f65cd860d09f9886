// ktmi_device.hpp -- per-cell device math of the KT + RK2 viscous hydro step
// (arXiv:1802.04449, Secs. II-III) for gfx950: EoS lookup, root solve,
// limiter, local speed, side fluxes, velocity gradients and the IS source.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ktmi {

constexpr double kHbarc = 0.1973269804;  // GeV fm

// Device memory seen through the global address space.  Plain pointers read
// from a table in memory are generic to the compiler, which then emits FLAT
// loads and stores; on CDNA those also count against the LDS / scalar-memory
// wait counter, so every LDS wait would also wait for outstanding HBM loads.
// Pointers of these types compile to global_load / global_store.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) int gint;
typedef __attribute__((address_space(1))) unsigned long long gullong;
typedef __attribute__((address_space(1))) char gchar;

template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gl(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// Parameters copied by value into every launch (kernel argument segment).
struct StepParams {
  int nx, ny, ne, ncell;
  double dx, dy, de;
  double inv_dx, inv_dy, inv_de;  // reciprocals of the spacings
  double h, inv_h;
  double etas;
  double inv_taupi_coef;  // 1 / (b eta/s hbarc): 1/tau_pi = T * inv_taupi_coef (b = 5, Sec. II)
  double eta_taupi;       // 1 / b: eta_v / tau_pi = (e + P) / b
  double lambda1_hat;     // lambda_1 = lambda1_hat / e (0: no second-order term)
  // bulk pressure (eqn. Pitilde): 1/tau_Pi = T * inv_taubulk_coef with tau_Pi =
  // c (zeta/s) hbarc / T, zeta / tau_Pi = (e + P) * zeta_taubulk (= 1/c); both 0
  // without bulk viscosity.  baryon: 1 when the net-baryon density is transported.
  double inv_taubulk_coef, zeta_taubulk;
  int bulk, baryon;
  double eps_cut, theta, newton_tol, pi_reg;
  double c_vac;  // local speed of a vacuum state, sqrt(cs2(0))
  int newton_maxit;
  // 1 when the regulator zeroes pi~ (and Pi, n) wherever e = 0: it is on and the
  // EoS gives P = 0 at e = 0.  Passes then skip the loads that could not change a
  // vacuum cell's result.
  int vac_zero;
  int quiet_r[3];          // quiet-tile skipping: neighbourhood radius in tiles (0: off)
  int guess;               // root-solve start: 0 previous stage, 1 cold (E), 2 network
  int mlp_mfma;            // network forward: 0 FP32 per lane, 1 BF16 matrix cores per wave
  const float* mlp;        // network parameters (FP32), then W2 as BF16
};

struct EosDev {
  int kind;  // 0 ideal gas, 1 uniform table
  int n;
  double c_sb, inv_csb, e0, de, inv_de;
  const double* P;
  const double* T;
  const double* cs2;
  // FP32 copy of the table for the mixed-precision flux and relaxation arithmetic
  float inv_csb_f, e0_f, de_f, inv_de_f;
  const float* Pf;
  const float* Tf;
  const float* cs2f;
};

// Root-solve outcome flags (counted in the diagnostics).  kNeg: K^tau < 0.
enum : int { kFallback = 1, kNonconv = 2, kNan = 4, kVac = 8, kClamp = 16, kNeg = 32 };

// ---------------------------------------------------------------------------
// EoS lookup (Sec. III, EoS options).  The table is uniform in e; values are
// linear between rows; past the last row P keeps the last slope, cs2 is held
// and T scales as ((e+P)/(e_last+P_last))^(1/4).  e < 0 is read as 0.
// ---------------------------------------------------------------------------
struct EosSeg {
  int i;       // row index of the segment (or n-1 past the end)
  double f;    // position inside the segment
  bool beyond;
};

__device__ __forceinline__ EosSeg eos_seg(const EosDev& q, double e) {
  EosSeg s;
  double x = (e - q.e0) * q.inv_de;
  x = x >= 0.0 ? x : 0.0;  // also maps NaN to the first row
  s.beyond = x >= (double)(q.n - 1);
  const double xc = s.beyond ? (double)(q.n - 2) : x;  // keeps the index in [0, n-2]
  int i = (int)floor(xc);
  i = i > q.n - 2 ? q.n - 2 : (i < 0 ? 0 : i);
  s.i = i;
  s.f = xc - (double)i;
  return s;
}

// P and cs2 (flux side states).
__device__ __forceinline__ void eos_p_cs2(const EosDev& q, double e, double& P, double& cs2) {
  e = e > 0.0 ? e : 0.0;
  if (q.kind == 0) {
    P = e * (1.0 / 3.0);
    cs2 = 1.0 / 3.0;
    return;
  }
  EosSeg s = eos_seg(q, e);
  const int n = q.n;
  if (s.beyond) {
    const double slope = (gl(q.P)[n - 1] - gl(q.P)[n - 2]) * q.inv_de;
    const double elast = q.e0 + (double)(n - 1) * q.de;
    P = gl(q.P)[n - 1] + (e - elast) * slope;
    cs2 = gl(q.cs2)[n - 1];
    return;
  }
  const double p0 = gl(q.P)[s.i], p1 = gl(q.P)[s.i + 1];
  const double c0 = gl(q.cs2)[s.i], c1 = gl(q.cs2)[s.i + 1];
  P = p0 + s.f * (p1 - p0);
  cs2 = c0 + s.f * (c1 - c0);
}

// P and the segment slope dP/de (root solve).
__device__ __forceinline__ void eos_p_dp(const EosDev& q, double e, double& P, double& dP) {
  e = e > 0.0 ? e : 0.0;
  if (q.kind == 0) {
    P = e * (1.0 / 3.0);
    dP = 1.0 / 3.0;
    return;
  }
  EosSeg s = eos_seg(q, e);
  const int n = q.n;
  if (s.beyond) {
    dP = (gl(q.P)[n - 1] - gl(q.P)[n - 2]) * q.inv_de;
    const double elast = q.e0 + (double)(n - 1) * q.de;
    P = gl(q.P)[n - 1] + (e - elast) * dP;
    return;
  }
  const double p0 = gl(q.P)[s.i], p1 = gl(q.P)[s.i + 1];
  P = p0 + s.f * (p1 - p0);
  dP = (p1 - p0) * q.inv_de;
}

// P and T (viscous source).
__device__ __forceinline__ void eos_p_t(const EosDev& q, double e, double& P, double& T) {
  e = e > 0.0 ? e : 0.0;
  if (q.kind == 0) {
    P = e * (1.0 / 3.0);
    T = sqrt(sqrt(e * q.inv_csb));
    return;
  }
  EosSeg s = eos_seg(q, e);
  const int n = q.n;
  if (s.beyond) {
    const double slope = (gl(q.P)[n - 1] - gl(q.P)[n - 2]) * q.inv_de;
    const double elast = q.e0 + (double)(n - 1) * q.de;
    P = gl(q.P)[n - 1] + (e - elast) * slope;
    T = gl(q.T)[n - 1] * sqrt(sqrt((e + P) / (elast + gl(q.P)[n - 1])));
    return;
  }
  const double p0 = gl(q.P)[s.i], p1 = gl(q.P)[s.i + 1];
  const double t0 = gl(q.T)[s.i], t1 = gl(q.T)[s.i + 1];
  P = p0 + s.f * (p1 - p0);
  T = t0 + s.f * (t1 - t0);
}

__device__ __forceinline__ double eos_p(const EosDev& q, double e) {
  double P, c;
  eos_p_cs2(q, e, P, c);
  return P;
}

// ---------------------------------------------------------------------------
// Root solve (Sec. III flow chart: T_ideal = T - pi -> e, u).  With
// K = T~^{tau .}/tau - pi~^{tau .}, E = K^tau, M = |K|, the rest-frame energy
// density is the unique root of f(e) = e - E + M^2/(E + P(e)) on
// [max(0, E - M^2/E), E].  Safeguarded Newton (bisection when a step leaves the
// bracket) to |de| <= tol e, then one more Newton step; the cutoff applies to
// the root.  Velocity: u~^i = K^i / sqrt((E+P)(e+P)).
// BK (bulk pressure Pi, eqn. Pitilde): P becomes P + Pi in f, f' and the
// velocity, and the bracket and the cap of M use B = E + min(Pi, 0) in place of
// E (no root when B <= 0: vacuum, flagged as clamped).
// ---------------------------------------------------------------------------
struct Prim {
  double e, u1, u2, u3;
};

__device__ __forceinline__ Prim vacuum() { return Prim{0.0, 0.0, 0.0, 0.0}; }

template <bool BK = false>
__device__ inline Prim con2prim(const EosDev& q, const StepParams& p, double E, double K1,
                                double K2, double K3, double guess, int& iters, int& flags,
                                double Pi = 0.0) {
  iters = 0;
  flags = 0;
  if (isnan(E) || isnan(K1) || isnan(K2) || isnan(K3)) {
    flags = kNan | kVac;
    return vacuum();
  }
  if (!(E >= p.eps_cut)) {
    flags = kVac | (E < 0.0 ? kNeg : 0);
    return vacuum();
  }
  double B = E;
  if constexpr (BK) {
    B = E + (Pi < 0.0 ? Pi : 0.0);
    if (!(B > 0.0)) {
      flags = kVac | kClamp;
      return vacuum();
    }
  }
  double M2 = K1 * K1 + K2 * K2 + K3 * K3;
  const double Mmax = (1.0 - 1e-10) * B;
  if (M2 > Mmax * Mmax) {
    const double s = Mmax / sqrt(M2);
    K1 *= s;
    K2 *= s;
    K3 *= s;
    M2 = K1 * K1 + K2 * K2 + K3 * K3;
    flags |= kClamp;
  }
  double lo = E - M2 / B;
  lo = lo < 0.0 ? 0.0 : lo;
  double hi = E;
  const double lo0 = lo, hi0 = hi;
  double x = guess;
  if (!(x >= lo)) x = lo;
  if (x > hi) x = hi;
  bool conv = false;
  int it;
  for (it = 1; it <= p.newton_maxit; ++it) {
    if (hi < p.eps_cut) {
      iters = it;
      flags |= kVac;
      return vacuum();
    }
    double P, dP;
    eos_p_dp(q, x, P, dP);
    const double r = 1.0 / (BK ? (E + P) + Pi : E + P);  // one division for f and f'
    const double f = x - E + M2 * r;
    const double df = 1.0 - M2 * dP * r * r;
    if (f == 0.0) {
      conv = true;
      break;
    }
    if (f > 0.0)
      hi = x;
    else
      lo = x;
    double xn = x - f / df;
    if (!(xn >= lo && xn <= hi)) {
      xn = 0.5 * (lo + hi);
      flags |= kFallback;
    }
    const double step = fabs(xn - x);
    x = xn;
    if (step <= p.newton_tol * x) {
      conv = true;
      break;
    }
  }
  if (!conv) {
    flags |= kNonconv;
    it = p.newton_maxit;
  }
  {
    double P, dP;
    eos_p_dp(q, x, P, dP);
    const double r = 1.0 / (BK ? (E + P) + Pi : E + P);
    const double f = x - E + M2 * r;
    const double df = 1.0 - M2 * dP * r * r;
    const double xp = x - f / df;
    if (xp >= lo0 && xp <= hi0) x = xp;
  }
  iters = it + 1;
  if (!(x >= p.eps_cut)) {
    flags |= kVac;
    return vacuum();
  }
  const double P = BK ? eos_p(q, x) + Pi : eos_p(q, x);
  const double inv = 1.0 / sqrt((E + P) * (x + P));
  return Prim{x, K1 * inv, K2 * inv, K3 * inv};
}

// ---------------------------------------------------------------------------
// Reconstruction and the KT local speed (Sec. III, eqs. kt and flux_out).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double minmod3(double a, double b, double c) {
  if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
  if (a < 0.0 && b < 0.0 && c < 0.0) return fmax(a, fmax(b, c));
  return 0.0;
}

__device__ __forceinline__ double mm_slope(double th, double qm, double q0, double qp) {
  return minmod3(th * (q0 - qm), 0.5 * (qp - qm), th * (qp - q0));
}

// Largest |eigenvalue| of the ideal flux Jacobian along the face normal for a
// state with u~ = (ut, ux, uy, ue) and sound speed squared cs2:
// lambda = [v_d (1-cs2) +- cs sqrt((1-v^2)(1 - v^2 cs2 - v_d^2 (1-cs2)))]/(1 - v^2 cs2).
__device__ __forceinline__ double local_speed(double ut, double ux, double uy, double ue,
                                              double ud, double cs2) {
  const double inv = 1.0 / ut;
  const double vd = ud * inv;
  const double v2 = (ux * ux + uy * uy + ue * ue) * inv * inv;
  double disc = inv * inv * (1.0 - v2 * cs2 - vd * vd * (1.0 - cs2));
  disc = disc < 0.0 ? 0.0 : disc;
  const double root = sqrt(cs2 * disc);
  const double inv_den = 1.0 / (1.0 - v2 * cs2);
  const double a = vd * (1.0 - cs2);
  return (fabs(a) + root) * inv_den;  // = max(|a + root|, |a - root|) / den, root >= 0
}

// ---------------------------------------------------------------------------
// Precision-generic versions for the flux and relaxation arithmetic: R = double
// (FP64 path) or float (mixed path; table values from the FP32 copy).
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void eos_p_cs2_r(const EosDev& q, R e, R& P, R& cs2);

template <>
__device__ __forceinline__ void eos_p_cs2_r<double>(const EosDev& q, double e, double& P,
                                                     double& cs2) {
  eos_p_cs2(q, e, P, cs2);
}

template <>
__device__ __forceinline__ void eos_p_cs2_r<float>(const EosDev& q, float e, float& P, float& cs2) {
  e = e > 0.0f ? e : 0.0f;
  if (q.kind == 0) {
    P = e * (1.0f / 3.0f);
    cs2 = 1.0f / 3.0f;
    return;
  }
  const int n = q.n;
  float x = (e - q.e0_f) * q.inv_de_f;
  x = x >= 0.0f ? x : 0.0f;
  if (x >= (float)(n - 1)) {
    const float slope = (gl(q.Pf)[n - 1] - gl(q.Pf)[n - 2]) * q.inv_de_f;
    P = gl(q.Pf)[n - 1] + (e - (q.e0_f + (float)(n - 1) * q.de_f)) * slope;
    cs2 = gl(q.cs2f)[n - 1];
    return;
  }
  int i = (int)floorf(x);
  i = i > n - 2 ? n - 2 : (i < 0 ? 0 : i);
  const float f = x - (float)i;
  P = gl(q.Pf)[i] + f * (gl(q.Pf)[i + 1] - gl(q.Pf)[i]);
  cs2 = gl(q.cs2f)[i] + f * (gl(q.cs2f)[i + 1] - gl(q.cs2f)[i]);
}

template <typename R>
__device__ __forceinline__ void eos_p_t_r(const EosDev& q, R e, R& P, R& T);

template <>
__device__ __forceinline__ void eos_p_t_r<double>(const EosDev& q, double e, double& P, double& T) {
  eos_p_t(q, e, P, T);
}

template <>
__device__ __forceinline__ void eos_p_t_r<float>(const EosDev& q, float e, float& P, float& T) {
  e = e > 0.0f ? e : 0.0f;
  if (q.kind == 0) {
    P = e * (1.0f / 3.0f);
    T = sqrtf(sqrtf(e * q.inv_csb_f));
    return;
  }
  const int n = q.n;
  float x = (e - q.e0_f) * q.inv_de_f;
  x = x >= 0.0f ? x : 0.0f;
  if (x >= (float)(n - 1)) {
    const float slope = (gl(q.Pf)[n - 1] - gl(q.Pf)[n - 2]) * q.inv_de_f;
    const float elast = q.e0_f + (float)(n - 1) * q.de_f;
    P = gl(q.Pf)[n - 1] + (e - elast) * slope;
    T = gl(q.Tf)[n - 1] * sqrtf(sqrtf((e + P) / (elast + gl(q.Pf)[n - 1])));
    return;
  }
  int i = (int)floorf(x);
  i = i > n - 2 ? n - 2 : (i < 0 ? 0 : i);
  const float f = x - (float)i;
  P = gl(q.Pf)[i] + f * (gl(q.Pf)[i + 1] - gl(q.Pf)[i]);
  T = gl(q.Tf)[i] + f * (gl(q.Tf)[i + 1] - gl(q.Tf)[i]);
}

// min of the three if all are positive, max if all are negative, else 0,
// written as max(lo, 0) + min(hi, 0) with lo, hi the min and max of the three
// (no compares or selects; the same value for finite arguments, up to the sign
// of a zero result).
template <typename R>
__device__ __forceinline__ R minmod3_r(R a, R b, R c) {
  const R lo = fmin(a, fmin(b, c)), hi = fmax(a, fmax(b, c));
  return fmax(lo, R(0)) + fmin(hi, R(0));
}

template <typename R>
__device__ __forceinline__ R mm_slope_r(R th, R qm, R q0, R qp) {
  return minmod3_r<R>(th * (q0 - qm), R(0.5) * (qp - qm), th * (qp - q0));
}

template <typename R>
__device__ __forceinline__ R local_speed_r(R ut, R ux, R uy, R ue, R ud, R cs2) {
  const R w = R(1) - cs2;
  const R u2 = ux * ux + uy * uy + ue * ue;
  const R up2 = u2 - ud * ud;  // transverse part (>= 0 up to rounding)
  const R disc = R(1) + (up2 > R(0) ? up2 : R(0)) * w;
  return (fabs(ud) * w * ut + sqrt(cs2 * disc)) / (R(1) + u2 * w);
}

// pi~ component index of the symmetric pair (mu, nu).
__host__ __device__ constexpr int sym(int mu, int nu) {
  return mu > nu ? sym(nu, mu)
                 : (mu == 0 ? nu : (mu == 1 ? 3 + nu : (mu == 2 ? 5 + nu : 9)));
}

}  // namespace ktmi
