// Device building blocks of the lattice Boltzmann kernels (gfx950), shared by
// the translation units of the library; everything here is inlined into the
// kernels that use it.
//
// State layout: per sample, q population planes (q = 27 for D3Q27, 19 for
// D3Q19) of n^3 values each plus padding (SoA), cells C-ordered [z][y][x].
// Values are shifted: g_i = f_i - w_i (stored in float or double). The state
// is updated in place with the AA pattern: on an even step a node reads its
// own q slots and writes the post-collision populations back into the
// opposite slots of the same node; on an odd step it reads population i from
// the slot of the opposite velocity at node x - c_i and writes the
// post-collision population i into slot i of node x + c_i. Every slot is read
// and written by exactly one thread per step, so the update is race free, and
// one step moves q loads + q stores per node.
//
// Collision (eqs. (equilibrium), (kbcCollision), (entropyControl), Table 1):
//   rho = 1 + sum g, j = sum c g, u = j / rho,
//   g^eq_i = w_i [drho + 3 c_i.j + rho (4.5 (c_i.u)^2 - 1.5 |u|^2)],
//   f^neq = g - g^eq,
//   shear part ds: the population vector with the traceless normal-stress
//   differences Nxz, Nyz and the off-diagonal stresses of f^neq and no other
//   raw moment: faces (+-1,0,0): (2Nxz - Nyz)/6, (0,+-1,0): (2Nyz - Nxz)/6,
//   (0,0,+-1): -(Nxz + Nyz)/6; edges: cx cy Pxy/4 + cx cz Pxz/4 + cy cz Pyz/4;
//   rest and corners: 0 (the same on both lattices).  Higher-order part
//   dh = f^neq - ds.
//   gamma = 2/omega - (2 - 2/omega) <ds|dh>/<dh|dh>, <X|Y> = sum X_i Y_i / f^eq_i
//   (gamma = 2 when <dh|dh> <= 1e-30),
//   g* = g - omega ds - (omega gamma / 2) dh.
// Everything is computed in the storage precision from the shifted values,
// so the weights w_i never enter a subtraction of nearly equal numbers.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "kernels.h"
#include "lattice.h"

namespace mclbm {
namespace {

template <int I, int N, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// f(i) for every velocity i of the lattice (D3Q27 numbering, ascending)
template <int QN, typename F>
__host__ __device__ __forceinline__ void for_vel(F&& f) {
  static_for<0, Q>([&](auto ic) {
    if constexpr (in_lattice<QN>(decltype(ic)::value)) f(ic);
  });
}

template <int c, typename T>
__device__ __forceinline__ T signed_term(T v) {
  if constexpr (c > 0) return v;
  else return -v;
}

// c_i . (x, y, z) built from the non-zero components only
template <int i, typename T>
__device__ __forceinline__ T cdot(T x, T y, T z) {
  constexpr int a = cx(i), b = cy(i), c = cz(i);
  if constexpr (a == 0 && b == 0 && c == 0) return T(0);
  else if constexpr (b == 0 && c == 0) return signed_term<a>(x);
  else if constexpr (a == 0 && c == 0) return signed_term<b>(y);
  else if constexpr (a == 0 && b == 0) return signed_term<c>(z);
  else if constexpr (c == 0) return signed_term<a>(x) + signed_term<b>(y);
  else if constexpr (b == 0) return signed_term<a>(x) + signed_term<c>(z);
  else if constexpr (a == 0) return signed_term<b>(y) + signed_term<c>(z);
  else return signed_term<a>(x) + signed_term<b>(y) + signed_term<c>(z);
}

template <typename T>
__device__ __forceinline__ T recip(T x) {
  if constexpr (std::is_same<T, float>::value) return __builtin_amdgcn_rcpf(x);
  else return 1.0 / x;
}

template <typename T>
__device__ __forceinline__ T vmin(T a, T b) {
  return a < b ? a : b;
}

template <typename T>
__device__ __forceinline__ T vmax(T a, T b) {
  return a > b ? a : b;
}

// ln(1 + x) for x > -1. float: the hardware base-2 logarithm of u = 1 + x
// (rounded to float) times ln 2, minus the rounding error e = (u - 1) - x of
// u (exact in float): ln(1 + x) = ln(u - e) = ln u - e/u + O(e^2), and
// taking e for e/u errs by e x / u, at most 2^-24 |x|, which is below one
// unit in the last place of ln(1 + x) for small x and of the logarithm's own
// rounding for large x (the correction is the one of the log1p identity in
// Goldberg, "What every computer scientist should know about floating-point
// arithmetic", 1991, Theorem 4, to first order, without its division);
// exactly x where u rounds to 1. double: the library log1p.
template <typename T>
__device__ __forceinline__ T log1p_acc(T x) {
  if constexpr (std::is_same<T, float>::value) {
    const float u = 1.0f + x;
    return __builtin_amdgcn_logf(u) * 0.693147180559945309f - ((u - 1.0f) - x);
  } else {
    return log1p(x);
  }
}

template <typename T>
struct Macro {
  T drho, jx, jy, jz, rho, inv, ux, uy, uz, usq15;
};

template <int QN, typename T>
__device__ __forceinline__ Macro<T> macroscopic(const T (&g)[Q]) {
  T d = T(0), x = T(0), y = T(0), z = T(0);
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    d += g[i];
  });
  // momentum: +direction partial sums minus -direction partial sums
  T xp = T(0), xm = T(0), yp = T(0), ym = T(0), zp = T(0), zm = T(0);
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (cx(i) > 0) xp += g[i];
    if constexpr (cx(i) < 0) xm += g[i];
    if constexpr (cy(i) > 0) yp += g[i];
    if constexpr (cy(i) < 0) ym += g[i];
    if constexpr (cz(i) > 0) zp += g[i];
    if constexpr (cz(i) < 0) zm += g[i];
  });
  x = xp - xm;
  y = yp - ym;
  z = zp - zm;
  Macro<T> m;
  m.drho = d;
  m.jx = x;
  m.jy = y;
  m.jz = z;
  m.rho = T(1) + d;
  m.inv = T(1) / m.rho;
  m.ux = x * m.inv;
  m.uy = y * m.inv;
  m.uz = z * m.inv;
  m.usq15 = T(1.5) * (m.ux * m.ux + m.uy * m.uy + m.uz * m.uz);
  return m;
}

// Velocity of a node (eq. (momentDefin)) from its shifted populations, summed
// in double in velocity order whatever the storage precision: the field the
// FP64 observables transform. The collide-and-stream kernel writes it on
// record ticks and the first pass of the observables computes it from a
// stored state with this same code, so the two fields are bitwise equal.
template <int QN, typename T>
__device__ __forceinline__ void node_velocity(const T (&g)[Q], double& ux, double& uy, double& uz) {
  double d = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const double v = double(g[i]);
    d += v;
    if constexpr (cx(i) != 0) jx += cx(i) * v;
    if constexpr (cy(i) != 0) jy += cy(i) * v;
    if constexpr (cz(i) != 0) jz += cz(i) * v;
  });
  const double rho = 1.0 + d;
  ux = jx / rho;
  uy = jy / rho;
  uz = jz / rho;
}

// shifted equilibrium g^eq_i = f^eq_i - w_i
template <int QN, int i, typename T>
__device__ __forceinline__ T geq(const Macro<T>& m) {
  const T w = T(weight<QN>(i));
  if constexpr (nonzeros(i) == 0) {
    return w * (m.drho - m.rho * m.usq15);
  } else {
    const T cu = cdot<i>(m.ux, m.uy, m.uz);
    const T cj = cdot<i>(m.jx, m.jy, m.jz);
    if constexpr (std::is_same<T, float>::value) {
      // 3 w_i c_i.j with 3 w_i split into a float head and tail: with the
      // rounded weights alone, sum_i 3 w_i c_i c_i = (1 + 7.5e-9) I, a
      // systematic momentum gain in every collision that accumulates over
      // thousands of steps; with the tail the first moment of g^eq is j up
      // to unbiased rounding.
      constexpr double w3 = 3.0 * weight<QN>(i);
      constexpr float w3_hi = float(w3);
      constexpr float w3_lo = float(w3 - double(w3_hi));
      return w * (m.drho + m.rho * (T(4.5) * cu * cu - m.usq15)) + (w3_hi * cj + w3_lo * cj);
    } else {
      return w * (m.drho + T(3) * cj + m.rho * (T(4.5) * cu * cu - m.usq15));
    }
  }
}

template <typename T>
struct Shear {
  T dsx, dsy, dsz, exy, exz, eyz;
};

// shear part of velocity i (faces and edges only)
template <int i, typename T>
__device__ __forceinline__ T shear_part(const Shear<T>& s) {
  constexpr int a = cx(i), b = cy(i), c = cz(i);
  static_assert(nonzeros(i) == 1 || nonzeros(i) == 2, "shear part vanishes on rest and corners");
  if constexpr (nonzeros(i) == 1) {
    if constexpr (a != 0) return s.dsx;
    else if constexpr (b != 0) return s.dsy;
    else return s.dsz;
  } else {
    if constexpr (c == 0) return signed_term<a * b>(s.exy);
    else if constexpr (b == 0) return signed_term<a * c>(s.exz);
    else return signed_term<b * c>(s.eyz);
  }
}

// Second moments of f^neq and the shear coefficients.
template <int QN, typename T>
__device__ __forceinline__ Shear<T> shear_coefficients(const T (&fneq)[Q]) {
  T pxx = T(0), pyy = T(0), pzz = T(0), pxy = T(0), pxz = T(0), pyz = T(0);
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (cx(i) != 0) pxx += fneq[i];
    if constexpr (cy(i) != 0) pyy += fneq[i];
    if constexpr (cz(i) != 0) pzz += fneq[i];
    if constexpr (cx(i) * cy(i) > 0) pxy += fneq[i];
    if constexpr (cx(i) * cy(i) < 0) pxy -= fneq[i];
    if constexpr (cx(i) * cz(i) > 0) pxz += fneq[i];
    if constexpr (cx(i) * cz(i) < 0) pxz -= fneq[i];
    if constexpr (cy(i) * cz(i) > 0) pyz += fneq[i];
    if constexpr (cy(i) * cz(i) < 0) pyz -= fneq[i];
  });
  const T nxz = pxx - pzz, nyz = pyy - pzz;
  const T sixth = T(1) / T(6);
  Shear<T> s;
  s.dsx = (T(2) * nxz - nyz) * sixth;
  s.dsy = (T(2) * nyz - nxz) * sixth;
  s.dsz = -(s.dsx + s.dsy);
  s.exy = T(0.25) * pxy;
  s.exz = T(0.25) * pxz;
  s.eyz = T(0.25) * pyz;
  return s;
}

template <typename T>
struct Relax {
  T omega, two_over_omega, kappa, eps;
};

template <typename T>
__device__ __forceinline__ Relax<T> relax_of(const DevSample& sp) {
  Relax<T> r;
  if constexpr (std::is_same<T, float>::value) {
    r.omega = sp.omega_f;
    r.two_over_omega = sp.two_over_omega_f;
    r.kappa = sp.kappa_f;
    r.eps = sp.eps_f;
  } else {
    r.omega = sp.omega;
    r.two_over_omega = sp.two_over_omega;
    r.kappa = sp.kappa;
    r.eps = sp.eps;
  }
  return r;
}

template <typename T>
struct CellResult {
  Macro<T> m;
  T gamma;
  bool bad;
};

// Exact entropic stabiliser (eq. (kbc_entropy)): with t = omega gamma / 2 the
// post-collision populations are f*_i(t) = b_i - t dh_i, b_i = f_i - omega ds_i,
// and H(t) = sum f*_i ln(f*_i / w_i) is convex in t on the interval where
// every f*_i > 0, with
//   -H'(t) = sum dh_i ln(f*_i / w_i)      (sum dh_i = 0),
//    H''(t) = sum dh_i^2 / f*_i.
// Newton's method from the closed-form t (the first-order solution of
// H'(t) = 0) converges quadratically; a step that would leave the interval is
// replaced by the midpoint towards its edge. A node stops once its step is
// below kExactTolerance of t (the next step would be below the rounding of
// T), after at most kExactNewtonSteps steps; every node decides for itself,
// so the result does not depend on its neighbours in the wave.
// ln(f*_i / w_i) is evaluated as log1p((f*_i - w_i) / w_i) from the shifted
// values, which keeps its relative accuracy for populations near their
// weights. dh carries no mass and no momentum, so H'(t) does not change when
// a + b.c_i is subtracted from every logarithm; the sums subtract
// drho - 1.5 |u|^2 + 3 c_i.u, the part of ln(f^eq_i / w_i) of first order in
// drho and second in u. In exact arithmetic that is a no-op; in rounding it
// keeps the mass and momentum that dh's rounding leaves (near equilibrium,
// where dh is itself at rounding level) from multiplying an O(u) logarithm
// and swamping the third-order balance that fixes t there.
constexpr int kExactNewtonSteps = 4;

template <typename T>
constexpr T exact_tolerance() {
  return std::is_same<T, float>::value ? T(1.0 / (1 << 12)) : T(1e-8);
}

// Below which <dh|dh> counts as equilibrium (gamma = 2, for either
// stabiliser). In FP64 1e-30, where dh vanishes up to rounding. In FP32 the dh
// of a node at equilibrium is the rounding of its populations (the moments
// and g^eq of about 27 float terms: a few units in the last place of
// |g^eq| ~ w |u|): the closed form would report a gamma of that rounding, and
// the exact minimiser acts on any dh, however small, by an amount of third
// order in u. Such a node is taken as at equilibrium, like the FP64 path,
// when <dh|dh> <= 2^-40 (3 |u|^2 + drho^2), about ten times that rounding
// level (sum_i (g^eq_i)^2 / f^eq_i = 3 |u|^2 + drho^2 to leading order);
// resolved flows carry dh far above it.
template <typename T>
__device__ __forceinline__ T equilibrium_threshold(const Macro<T>& m) {
  if constexpr (std::is_same<T, float>::value)
    return fmaxf(1e-30f, 0x1.0p-40f * (2.0f * m.usq15 + m.drho * m.drho));
  else
    return T(1e-30);
}

// The terms of the exact stabiliser, once per node: dh_i = f^neq_i - ds_i and
// bs_i = b_i - w_i = f_i - omega ds_i - w_i, so that f*_i(t) - w_i = bs_i - t dh_i.
// bs is formed as the closed-form update forms the post-collision state,
// (g^eq_i - ds_i) + eps ds_i + dh_i with eps = 2 - omega, which keeps the
// shear relaxation at full relative precision for omega near 2 (a float
// omega alone would carry eps to about 1e-4); the post-collision state is
// then bs_i - t dh_i, and g^eq and f^neq are no longer needed.
template <int QN, typename T>
__device__ __forceinline__ void exact_terms(const T (&geq)[Q], const T (&fneq)[Q], const Shear<T>& s, T eps,
                                            T (&dh)[Q], T (&bs)[Q]) {
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    T ds = T(0);
    if constexpr (nonzeros(i) == 1 || nonzeros(i) == 2) ds = shear_part<i>(s);
    dh[i] = fneq[i] - ds;
    bs[i] = ((geq[i] - ds) + eps * ds) + dh[i];
  });
}

template <int QN, typename T>
__device__ __forceinline__ T exact_entropic_t(const T (&dh)[Q], const T (&bs)[Q], const Macro<T>& m, T t) {
  const T a = m.drho - m.usq15;
  // The interval of t where every f*_i = w_i + bs_i - t dh_i > 0 bounds the
  // Newton iterates; it is formed (27 quotients) only when an iterate leaves
  // the region where every f*_i is positive, which takes 27 products to
  // check. In float the quotients use the hardware reciprocal (about one unit
  // in the last place) and are moved inwards by 2^-20 of their size, so that
  // the interval stays inside the exact one.
  bool have_interval = false;
  T lo = T(-1e30), hi = T(1e30);
  auto interval = [&]() {
    for_vel<QN>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const T base = T(weight<QN>(i)) + bs[i];
      T q;
      if constexpr (std::is_same<T, float>::value) {
        q = base * __builtin_amdgcn_rcpf(dh[i]);
        q = dh[i] > T(0) ? q - fabsf(q) * 0x1.0p-20f : q + fabsf(q) * 0x1.0p-20f;
      } else {
        q = base / dh[i];
      }
      if (dh[i] > T(0)) hi = vmin(hi, q);
      if (dh[i] < T(0)) lo = lo > q ? lo : q;
    });
    have_interval = true;
  };
  auto positive_at = [&](T tt) {
    T fmin = T(1);
    for_vel<QN>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      fmin = vmin(fmin, (T(weight<QN>(i)) + bs[i]) - tt * dh[i]);
    });
    return fmin > T(0);
  };
  // In float the curvature H'' of the first step is kept for the later ones
  // (a chord step: the curvature changes by about |t - t0| |dh| / f* between
  // steps, so each later step still contracts the error by that factor,
  // reaching float resolution in the step that meets the stopping rule); in
  // double every step is a full Newton step.
  // In float the first step also bounds its own error: with q_i = dh_i / f*_i,
  // |d3H/dt3| = |sum dh_i q_i^2| <= max|q| H'', so Newton's error after a
  // step D from t is below (|d3H/dt3| / (2 H'')) D^2 <= max|q| D^2 / 2 to
  // first order in D max|q|; while D max|q| <= 1/16 a node stops once that
  // is below 2^-22 of t, about two units in the last place, without taking
  // the logarithms again to see the next step fall below the tolerance.
  constexpr bool kChord = std::is_same<T, float>::value;
  bool done = false;
  T d2 = T(0), qmax = T(0);
  for (int it = 0; it < kExactNewtonSteps && !done; ++it) {
    T d1 = T(0);
    const bool curvature = !kChord || it == 0;
    if (curvature) d2 = T(0);
    for_vel<QN>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      constexpr double w = weight<QN>(i);
      // f*_i - w_i in shifted form
      const T gs = bs[i] - t * dh[i];
      d1 += dh[i] * (log1p_acc(gs * T(1.0 / w)) - (a + T(3) * cdot<i>(m.ux, m.uy, m.uz)));
      if (curvature) {
        const T qi = dh[i] * recip(T(w) + gs);
        d2 += dh[i] * qi;
        if constexpr (kChord) qmax = vmax(qmax, qi < T(0) ? -qi : qi);
      }
    });
    T tn = t + d1 / d2;
    bool newton = true;
    if (!positive_at(tn)) {
      if (!have_interval) interval();
      if (!(tn < hi)) {
        tn = T(0.5) * (t + hi);
        newton = false;
      }
      if (!(tn > lo)) {
        tn = T(0.5) * (t + lo);
        newton = false;
      }
    }
    const T step = tn - t, astep = step < T(0) ? -step : step;
    done = astep <= exact_tolerance<T>() * fabs(t);
    if constexpr (kChord)
      if (it == 0 && newton && qmax * astep <= T(0.0625))
        done = done || qmax * astep * astep <= T(0x1.0p-22) * fabs(tn);
    t = tn;
  }
  return t;
}

// KBC collision of one node in place: g <- g*. Between the passes g[] holds
// the shifted equilibrium, so every g^eq_i is evaluated once. EXACT selects
// the exact minimiser of the discrete H-function instead of the closed form.
template <int QN, bool EXACT = false, typename T>
__device__ __forceinline__ CellResult<T> kbc_collide(T (&g)[Q], const Relax<T>& rp) {
  CellResult<T> res;
  res.m = macroscopic<QN>(g);
  const Macro<T>& m = res.m;
  T fneq[Q];
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const T ge = geq<QN, i>(m);
    fneq[i] = g[i] - ge;
    g[i] = ge;
  });
  const Shear<T> s = shear_coefficients<QN>(fneq);
  T A = T(0), B = T(0), fmin = T(1);
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const T feq = T(weight<QN>(i)) + g[i];
    const T r = recip(feq);
    fmin = vmin(fmin, feq);
    if constexpr (nonzeros(i) == 1 || nonzeros(i) == 2) {
      const T ds = shear_part<i>(s);
      const T dh = fneq[i] - ds;
      A += ds * dh * r;
      B += dh * dh * r;
    } else {
      B += fneq[i] * fneq[i] * r;
    }
  });
  const bool resolved = B > equilibrium_threshold<T>(m);
  T gamma = T(2);
  if (resolved) gamma = rp.two_over_omega - rp.kappa * (A / B);
  T t = T(0.5) * rp.omega * gamma;
  if constexpr (EXACT) {
    // g* = bs - t dh (the same update as below, in the terms of the exact
    // minimiser, which are all it keeps through its iteration)
    T dh[Q], bs[Q];
    exact_terms<QN>(g, fneq, s, rp.eps, dh, bs);
    if (resolved) {
      t = exact_entropic_t<QN>(dh, bs, m, t);
      gamma = T(2) * t / rp.omega;
    }
    for_vel<QN>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      g[i] = bs[i] - t * dh[i];
    });
  } else {
    // g* = g - omega ds - t dh = (g^eq - ds) + (2 - omega) ds + (1 - t) dh.
    // The shear relaxation enters through eps = 2 - omega, which keeps the
    // viscosity (proportional to eps for omega near 2) at full relative
    // precision even in float.
    const T one_t = T(1) - t;
    for_vel<QN>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      if constexpr (nonzeros(i) == 1 || nonzeros(i) == 2) {
        const T ds = shear_part<i>(s);
        g[i] = (g[i] - ds) + rp.eps * ds + one_t * (fneq[i] - ds);
      } else {
        g[i] = g[i] + one_t * fneq[i];
      }
    });
  }
  res.gamma = gamma;
  res.bad = !(m.rho > T(0)) || !(m.usq15 < T(1.5)) || !(fmin > T(0));
  if constexpr (EXACT) res.bad = res.bad || !(t == t);
  return res;
}

// ---------------------------------------------------------------- addressing
struct Cell {
  uint32_t cell;
  uint32_t ox[3], oy[3], oz[3];  // neighbour coordinates along each axis: -1, 0, +1
};

__host__ __device__ __forceinline__ Cell make_cell(uint32_t cell, int l) {
  Cell c;
  c.cell = cell;
  const uint32_t msk = (1u << l) - 1u;
  const uint32_t x = cell & msk, y = (cell >> l) & msk, z = cell >> (2 * l);
  c.ox[0] = (x - 1u) & msk;
  c.ox[1] = x;
  c.ox[2] = (x + 1u) & msk;
  c.oy[0] = ((y - 1u) & msk) << l;
  c.oy[1] = y << l;
  c.oy[2] = ((y + 1u) & msk) << l;
  c.oz[0] = ((z - 1u) & msk) << (2 * l);
  c.oz[1] = z << (2 * l);
  c.oz[2] = ((z + 1u) & msk) << (2 * l);
  return c;
}

// index of the neighbour x + s * c_i
template <int i, int s>
__host__ __device__ __forceinline__ uint32_t neighbour(const Cell& c) {
  return c.oz[1 + s * cz(i)] + c.oy[1 + s * cy(i)] + c.ox[1 + s * cx(i)];
}

// AA slots of population i (D3Q27 numbering) of the node at c: the slot a
// step of the given parity reads it from before the collision, and the slot
// it writes the post-collision value to. A slot is a velocity (whose storage
// plane holds it) and a node. Even step: read slot i of the node, write slot
// opposite(i) of the node. Odd step: read slot opposite(i) of x - c_i, write
// slot i of x + c_i. The odd step's read undoes the even step's write of
// population i at x - c_i, so the pair streams by c_i twice over two steps,
// once per step.
struct Slot {
  int vel;
  uint32_t idx;
};
template <int i>
__host__ __device__ __forceinline__ Slot aa_read_slot(const Cell& c, bool odd) {
  return odd ? Slot{opposite(i), neighbour<i, -1>(c)} : Slot{i, c.cell};
}
template <int i>
__host__ __device__ __forceinline__ Slot aa_write_slot(const Cell& c, bool odd) {
  return odd ? Slot{i, neighbour<i, +1>(c)} : Slot{opposite(i), c.cell};
}

// element access with a 32-bit byte offset from a uniform plane base
template <typename T>
__host__ __device__ __forceinline__ T ld(const T* plane, uint32_t idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(plane) + idx * uint32_t(sizeof(T)));
}
template <typename T>
__host__ __device__ __forceinline__ void st(T* plane, uint32_t idx, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(plane) + idx * uint32_t(sizeof(T))) = v;
}

// The 27 planes of one sample through one buffer resource: the per-plane
// offset is a scalar (SGPR) operand and each lane supplies a 32-bit byte
// offset, so an access costs one VGPR of address. Used when the sample's
// populations occupy less than 4 GiB.
constexpr int kBufferFlags = 0x00020000;  // 32-bit raw data format (gfx9 family)

// NT: non-temporal loads and stores (each population is read once and written
// once per step, so nothing is gained by keeping it in the caches).
constexpr int kAuxNontemporal = 2;  // cache-policy operand of buffer instructions: nt

// Accesses name a velocity i (D3Q27 numbering); the plane is plane_of<QN>(i).
template <typename T, bool NT, int QN>
struct BufPlanes {
  static constexpr int aux = NT ? kAuxNontemporal : 0;
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t plane_bytes;
  __device__ __forceinline__ BufPlanes(T* base, uint32_t pstride)
      : rsrc(__builtin_amdgcn_make_buffer_rsrc(base, 0, int(uint32_t(QN) * pstride * uint32_t(sizeof(T))), kBufferFlags)),
        plane_bytes(pstride * uint32_t(sizeof(T))) {}
  __device__ __forceinline__ T load(int i, uint32_t idx) const {
    const int plane = plane_of<QN>(i);
    if constexpr (sizeof(T) == 4)
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rsrc, int(idx * 4u), int(plane * plane_bytes), aux));
    else
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rsrc, int(idx * 8u), int(plane * plane_bytes), aux));
  }
  __device__ __forceinline__ void store(int i, uint32_t idx, T v) const {
    const int plane = plane_of<QN>(i);
    if constexpr (sizeof(T) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rsrc, int(idx * 4u),
                                            int(plane * plane_bytes), aux);
    else
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(
                                                                   rsrc, 0, 0, 0)), v),
                                            rsrc, int(idx * 8u), int(plane * plane_bytes), aux);
  }
};

// The same access through plain pointers (any sample size).
template <typename T, bool NT, int QN>
struct PtrPlanes {
  T* base;
  uint32_t pstride;
  __device__ __forceinline__ PtrPlanes(T* b, uint32_t p) : base(b), pstride(p) {}
  __device__ __forceinline__ T load(int i, uint32_t idx) const {
    const size_t plane = size_t(plane_of<QN>(i));
    if constexpr (NT) return __builtin_nontemporal_load(base + plane * pstride + idx);
    else return ld(base + plane * pstride, idx);
  }
  __device__ __forceinline__ void store(int i, uint32_t idx, T v) const {
    const size_t plane = size_t(plane_of<QN>(i));
    if constexpr (NT) __builtin_nontemporal_store(v, base + plane * pstride + idx);
    else st(base + plane * pstride, idx, v);
  }
};

// populations of the post-stream state at a node, for either AA parity: the
// slots the next step reads them from
template <int QN, typename T>
__host__ __device__ __forceinline__ void load_state(const T* base, uint32_t pstride, const Cell& c, bool odd,
                                                    T (&g)[Q]) {
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const Slot s = aa_read_slot<i>(c, odd);
    g[i] = ld(base + size_t(plane_of<QN>(s.vel)) * pstride, s.idx);
  });
}

// the inverse mapping: write a post-stream state at a node
template <int QN, typename T>
__host__ __device__ __forceinline__ void write_state(T* base, uint32_t pstride, const Cell& c, bool odd,
                                                     const T (&g)[Q]) {
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const Slot s = aa_read_slot<i>(c, odd);
    st(base + size_t(plane_of<QN>(s.vel)) * pstride, s.idx, g[i]);
  });
}

// ---------------------------------------------------------------- x-shifts without partial cache lines
// On an odd step (and in the push and adjoint kernels) population i moves by
// c_i. Addressed directly, the 18 populations with c_x != 0 are read and
// written one 4-byte element off the 256-byte segment of their wave, so every
// such access of a wave touches three cache lines, two of them partly; on
// rows longer than one wave the neighbouring wave completes those lines later
// and, on large lattices, after they have left the cache. Instead every lane
// accesses its own x (y and z shifted as before) and the values move by one
// lane inside the wave (a DPP rotation of the whole wave); the lane at the
// wave's edge takes its value from the neighbouring wave of the same row,
// through LDS. A block must hold whole rows (64 < n <= block size; x is the
// fastest index, so a row is n/64 consecutive waves). For n = 64 the row is
// one wave and the direct addresses already stay inside the wave's segment.

// lane l receives the value of lane l - 1 (lane 0: lane 63)
__device__ __forceinline__ uint32_t rot_from_prev(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x13C /* wave_ror:1 */, 0xF, 0xF, false));
}
// lane l receives the value of lane l + 1 (lane 63: lane 0)
__device__ __forceinline__ uint32_t rot_from_next(uint32_t v) {
  return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x134 /* wave_rol:1 */, 0xF, 0xF, false));
}
template <bool PREV, typename T>
__device__ __forceinline__ T rotate_lanes(T v) {
  if constexpr (sizeof(T) == 4) {
    const uint32_t u = __builtin_bit_cast(uint32_t, v);
    return __builtin_bit_cast(T, PREV ? rot_from_prev(u) : rot_from_next(u));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = uint32_t(u), hi = uint32_t(u >> 32);
    const uint32_t rl = PREV ? rot_from_prev(lo) : rot_from_next(lo);
    const uint32_t rh = PREV ? rot_from_prev(hi) : rot_from_next(hi);
    return __builtin_bit_cast(T, (uint64_t(rh) << 32) | rl);
  }
}

// LDS for one exchange: per wave, the 9 values leaving through lane 63
// (towards +x) and the 9 leaving through lane 0 (towards -x)
template <typename T, int BLOCK>
using EdgeLds = T[BLOCK / 64][2][9];

// v[i] <- v[i] of node x - DIR * c_i,x of the same row (periodic), for every
// population i with c_i,x != 0. DIR = +1: values follow their velocity
// (streaming); DIR = -1: values are pulled from x + c_i (adjoint).
// Must be called by every thread of the block (it contains a barrier).
template <int QN, int DIR, int BLOCK, typename T>
__device__ __forceinline__ void row_shift(T (&v)[Q], EdgeLds<T, BLOCK>& edge, uint32_t n) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wpr = int(n >> 6), rw = w & (wpr - 1), base = w - rw;
  const int prev = base + ((rw + wpr - 1) & (wpr - 1)), next = base + ((rw + 1) & (wpr - 1));
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int d = cx(i) * DIR;
    if constexpr (d == 1) {
      if (lane == 63) edge[w][0][i % 9] = v[i];
    } else if constexpr (d == -1) {
      if (lane == 0) edge[w][1][i % 9] = v[i];
    }
  });
  __syncthreads();
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    constexpr int d = cx(i) * DIR;
    if constexpr (d == 1) {
      const T r = rotate_lanes<true>(v[i]);
      const T e = edge[prev][0][i % 9];
      v[i] = lane == 0 ? e : r;
    } else if constexpr (d == -1) {
      const T r = rotate_lanes<false>(v[i]);
      const T e = edge[next][1][i % 9];
      v[i] = lane == 63 ? e : r;
    }
  });
}

// index of x + s * (0, c_i,y, c_i,z): the node of the same x in the shifted row
template <int i, int s>
__host__ __device__ __forceinline__ uint32_t neighbour_yz(const Cell& c) {
  return c.oz[1 + s * cz(i)] + c.oy[1 + s * cy(i)] + c.ox[1];
}

__host__ __device__ __forceinline__ int remap_block(int b, int total, int xcd_remap) {
  // hardware dispatches workgroup b to XCD b % 8; give each XCD a contiguous run
  if (xcd_remap) {
    const int g8 = total & ~7;
    if (b < g8) b = (b & 7) * (g8 >> 3) + (b >> 3);
  }
  return b;
}

__host__ __device__ __forceinline__ int find_segment(const Seg* segs, int nseg, int b) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].first_block <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block reduction of the record quantities: 6 sums, 1 min, 1 max.
template <int BLOCK>
__device__ __forceinline__ void block_record(double (&v)[kRecord], double* out) {
  __shared__ double sh[BLOCK / 64][kRecord];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) v[k] = wave_sum(v[k]);
  v[6] = wave_min(v[6]);
  v[7] = wave_max(v[7]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < kRecord; ++k) sh[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double r[kRecord];
#pragma unroll
    for (int k = 0; k < kRecord; ++k) r[k] = sh[0][k];
    for (int w = 1; w < BLOCK / 64; ++w) {
#pragma unroll
      for (int k = 0; k < 6; ++k) r[k] += sh[w][k];
      r[6] = fmin(r[6], sh[w][6]);
      r[7] = fmax(r[7], sh[w][7]);
    }
#pragma unroll
    for (int k = 0; k < kRecord; ++k) out[k] = r[k];
  }
}

}  // namespace
}  // namespace mclbm
