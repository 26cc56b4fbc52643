// Oracle for the Monte Carlo KBC lattice Boltzmann hot path.
//
// TEST INFRASTRUCTURE ONLY. This is a plain, slow, double-precision CPU
// implementation of what the GPU path computes. It exists so that tests,
// the smoke check and the benchmark's CPU baseline can compare against an
// independent statement of the method. No product code may link or call it.
// It shares no source, header, table or helper with the GPU library.
//
// What it follows (paper section "Deterministic numerical methodology"):
//   * the D3Q27 velocity set (tensor product of the 1-D {-1,0,1} set with
//     weights 2/3, 1/6, 1/6), speed of sound c_s^2 = 1/3, or the paper's own
//     D3Q19 set (the 19 of those velocities with at most two non-zero
//     components, with the usual D3Q19 weights 1/3, 1/18, 1/36);
//   * the second-order truncated equilibrium, eq. (equilibrium);
//   * density and momentum as the zeroth and first moments;
//   * the multi-relaxation form J = -M^{-1} S M (f - f^eq), eqs.
//     (bgkCollisionOp), (momentInnerProd), (momentDefin), with M built from
//     raw monomial moments and the moments sorted into the kinematic, shear
//     and higher-order (hom) groups of Table 1;
//   * the KBC collision, eq. (kbcCollision), with the stabiliser gamma from
//     the closed form eq. (entropyControl) and the entropic inner product
//     weighted by 1/f^eq;
//   * optionally gamma from the exact minimisation of the discrete
//     H-function, eq. (kbc_entropy), by bisection on its derivative;
//   * periodic streaming, eq. (lbIteration), done as a two-lattice pull.
//
// Moment basis (the paper defers the tensors of Table 1 to an earlier work):
// the raw moments M_pqr, p,q,r in {0,1,2}, that do not vanish identically on
// the velocity set (all 27 for D3Q27; for D3Q19 the 19 with at most two
// non-zero exponents); the three diagonal second moments are replaced by the
// trace T and the differences Nxz = M200 - M002, Nyz = M020 - M002.
// Kinematic group: M000, M100, M010, M001. Shear group: Nxz, Nyz, M110,
// M101, M011. Hom group: T and the remaining raw moments of order >= 3
// (17 of order 3 to 6 for D3Q27; for D3Q19 the 6 of order 3 and the 3 of
// order 4, the Q and A tensors of Table 1).
//
// When <dh|dh> <= 1e-30 the closed form is undefined and the exact
// minimiser is set by rounding noise alone; gamma = 2 (BGK) is used then by
// both. The hom part is zero in that case up to rounding.
//
// Scalar type: double, or std::complex<double> for complex-step derivatives
// (every operation below is analytic in the populations; the threshold test
// looks at the real part only; the exact stabiliser's root is carried into
// complex arithmetic by Newton steps, see collide).
//
// State layout at this interface: f[cell][i], cell = (z*n + y)*n + x. D3Q27:
// i = 9*(cx+1) + 3*(cy+1) + (cz+1). D3Q19: the same order with the eight
// corner velocities left out (so the opposite of i is q-1-i in both).

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;

inline double re(double v) { return v; }
inline double re(const cplx& v) { return v.real(); }

template <int Q>
struct VelocitySet {
  int c[Q][3];
  double w[Q];
  VelocitySet() {
    const double w1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};  // 1-D weights of -1, 0, +1
    // D3Q19 weights by number of non-zero components (rest, axis, diagonal)
    const double w19[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
    int k = 0;
    for (int i = 0; i < 27; ++i) {
      int a = i / 9, b = (i / 3) % 3, d = i % 3;
      int nz = (a != 1) + (b != 1) + (d != 1);
      if (Q == 19 && nz == 3) continue;
      c[k][0] = a - 1;
      c[k][1] = b - 1;
      c[k][2] = d - 1;
      w[k] = (Q == 27) ? w1[a] * w1[b] * w1[d] : w19[nz];
      ++k;
    }
  }
};

template <int Q>
const VelocitySet<Q>& vs() {
  static const VelocitySet<Q> v;
  return v;
}

int ipow(int base, int e) {
  int r = 1;
  for (int k = 0; k < e; ++k) r *= base;
  return r;
}

// Moment matrix in the kinematic / shear / hom basis and its inverse.
template <int Q>
struct MomentBasis {
  double M[Q][Q];
  double Minv[Q][Q];
  int group[Q];  // 0 kinematic, 1 shear, 2 hom
  bool complete = false;

  MomentBasis() {
    const VelocitySet<Q>& v = vs<Q>();
    // raw monomial rows, indexed by exponents (p, q, r)
    auto raw = [&](int p, int q, int r, int i) {
      return double(ipow(v.c[i][0], p) * ipow(v.c[i][1], q) * ipow(v.c[i][2], r));
    };
    int row = 0;
    auto put_raw = [&](int p, int q, int r, int g) {
      if (row < Q) {
        for (int i = 0; i < Q; ++i) M[row][i] = raw(p, q, r, i);
        group[row] = g;
      }
      ++row;
    };
    // kinematic
    put_raw(0, 0, 0, 0);
    put_raw(1, 0, 0, 0);
    put_raw(0, 1, 0, 0);
    put_raw(0, 0, 1, 0);
    // shear: normal-stress differences and off-diagonal stresses
    for (int i = 0; i < Q; ++i) M[row][i] = raw(2, 0, 0, i) - raw(0, 0, 2, i);
    group[row++] = 1;
    for (int i = 0; i < Q; ++i) M[row][i] = raw(0, 2, 0, i) - raw(0, 0, 2, i);
    group[row++] = 1;
    put_raw(1, 1, 0, 1);
    put_raw(1, 0, 1, 1);
    put_raw(0, 1, 1, 1);
    // hom: trace of the second moment, then every raw moment of order >= 3
    // that does not vanish on the whole velocity set
    for (int i = 0; i < Q; ++i) M[row][i] = raw(2, 0, 0, i) + raw(0, 2, 0, i) + raw(0, 0, 2, i);
    group[row++] = 2;
    for (int p = 0; p <= 2; ++p)
      for (int q = 0; q <= 2; ++q)
        for (int r = 0; r <= 2; ++r) {
          if (p + q + r < 3) continue;
          bool nonzero = false;
          for (int i = 0; i < Q; ++i) nonzero = nonzero || raw(p, q, r, i) != 0.0;
          if (nonzero) put_raw(p, q, r, 2);
        }
    complete = row == Q;
    if (complete) invert();
  }

  // Gauss-Jordan elimination with partial pivoting.
  void invert() {
    double a[Q][2 * Q];
    for (int r = 0; r < Q; ++r)
      for (int k = 0; k < 2 * Q; ++k) a[r][k] = (k < Q) ? M[r][k] : (k - Q == r ? 1.0 : 0.0);
    for (int col = 0; col < Q; ++col) {
      int piv = col;
      for (int r = col + 1; r < Q; ++r)
        if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
      if (piv != col)
        for (int k = 0; k < 2 * Q; ++k) std::swap(a[piv][k], a[col][k]);
      double d = a[col][col];
      for (int k = 0; k < 2 * Q; ++k) a[col][k] /= d;
      for (int r = 0; r < Q; ++r) {
        if (r == col) continue;
        double fct = a[r][col];
        if (fct == 0.0) continue;
        for (int k = 0; k < 2 * Q; ++k) a[r][k] -= fct * a[col][k];
      }
    }
    for (int r = 0; r < Q; ++r)
      for (int k = 0; k < Q; ++k) Minv[r][k] = a[r][Q + k];
  }
};

template <int Q>
const MomentBasis<Q>& basis() {
  static const MomentBasis<Q> b;
  return b;
}

// eq. (equilibrium) with c_s^2 = 1/3
template <int Q, class T>
void equilibrium(const T& rho, const T u[3], T feq[Q]) {
  const VelocitySet<Q>& v = vs<Q>();
  T usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < Q; ++i) {
    T cu = double(v.c[i][0]) * u[0] + double(v.c[i][1]) * u[1] + double(v.c[i][2]) * u[2];
    feq[i] = rho * v.w[i] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
  }
}

template <int Q, class T>
void density_velocity(const T f[Q], T& rho, T u[3]) {
  const VelocitySet<Q>& v = vs<Q>();
  rho = 0.0;
  T j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; ++i) {
    rho += f[i];
    for (int a = 0; a < 3; ++a) j[a] += double(v.c[i][a]) * f[i];
  }
  for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;
}

// Exact entropic stabiliser, eq. (kbc_entropy): argmin over gamma' of
// H(f*) = sum f*_i ln(f*_i / w_i), f*(gamma') = f - omega ds - (omega gamma'/2) dh.
// H is convex in gamma'; its derivative is -(omega/2) sum dh_i (ln(f*_i/w_i) + 1).
// Bisection on the derivative inside the interval where every f*_i > 0.
template <int Q>
double exact_entropic_gamma(const double f[Q], const double ds[Q], const double dh[Q], double omega) {
  const VelocitySet<Q>& v = vs<Q>();
  double base[Q];
  for (int i = 0; i < Q; ++i) base[i] = f[i] - omega * ds[i];
  // admissible interval of t = omega*gamma/2: base_i - t dh_i > 0 for all i
  double tlo = -1e300, thi = 1e300;
  for (int i = 0; i < Q; ++i) {
    if (dh[i] > 0) thi = std::fmin(thi, base[i] / dh[i]);
    if (dh[i] < 0) tlo = std::fmax(tlo, base[i] / dh[i]);
  }
  auto dH = [&](double t) {
    double s = 0.0;
    for (int i = 0; i < Q; ++i) {
      double fs = base[i] - t * dh[i];
      s += -dh[i] * (std::log(fs / v.w[i]) + 1.0);
    }
    return s;
  };
  // dH tends to -inf at tlo and +inf at thi, so a sign change exists;
  // walk out from the BGK value t = omega until it is bracketed.
  double lo = omega, hi = omega;
  double stepv = 1e-6;
  if (dH(omega) > 0.0) {
    for (int it = 0; it < 2000; ++it) {
      double cand = omega - stepv;
      if (cand <= tlo) cand = 0.5 * (lo + tlo);
      lo = cand;
      if (dH(lo) <= 0.0) break;
      stepv *= 2.0;
    }
  } else {
    for (int it = 0; it < 2000; ++it) {
      double cand = omega + stepv;
      if (cand >= thi) cand = 0.5 * (hi + thi);
      hi = cand;
      if (dH(hi) >= 0.0) break;
      stepv *= 2.0;
    }
  }
  for (int it = 0; it < 400; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (dH(mid) > 0.0) hi = mid; else lo = mid;
  }
  return 2.0 * (0.5 * (lo + hi)) / omega;
}

// One KBC collision at one node.
// mode 0: closed-form gamma (eq. entropyControl)
// mode 1: gamma forced to 2 (BGK)
// mode 2: exact entropic gamma (complex scalars: see the complex step below)
template <int Q, class T>
void collide(const T f[Q], double omega, int mode, T fstar[Q], T* gamma_out, T ds_out[Q], T dh_out[Q]) {
  const MomentBasis<Q>& mb = basis<Q>();
  T rho, u[3], feq[Q], fneq[Q];
  density_velocity<Q>(f, rho, u);
  equilibrium<Q>(rho, u, feq);
  for (int i = 0; i < Q; ++i) fneq[i] = f[i] - feq[i];
  // moments of the non-equilibrium part in the grouped basis
  T m[Q];
  for (int r = 0; r < Q; ++r) {
    m[r] = 0.0;
    for (int i = 0; i < Q; ++i) m[r] += mb.M[r][i] * fneq[i];
  }
  // back to populations, one group at a time
  T ds[Q], dh[Q];
  for (int i = 0; i < Q; ++i) {
    ds[i] = 0.0;
    dh[i] = 0.0;
    for (int r = 0; r < Q; ++r) {
      if (mb.group[r] == 1) ds[i] += mb.Minv[i][r] * m[r];
      if (mb.group[r] == 2) dh[i] += mb.Minv[i][r] * m[r];
    }
  }
  T gamma = 2.0;
  if (mode == 0) {
    T sh = 0.0, hh = 0.0;
    for (int i = 0; i < Q; ++i) {
      sh += ds[i] * dh[i] / feq[i];
      hh += dh[i] * dh[i] / feq[i];
    }
    if (re(hh) > 1e-30) gamma = 2.0 / omega - (2.0 - 2.0 / omega) * sh / hh;
  } else if (mode == 2) {
    // the same threshold as the closed form: with <dh|dh> <= 1e-30 the
    // H-function does not depend on gamma beyond rounding, and gamma = 2
    double hh = 0.0;
    for (int i = 0; i < Q; ++i) hh += re(dh[i]) * re(dh[i]) / re(feq[i]);
    if (hh > 1e-30) {
      if constexpr (std::is_same<T, double>::value) {
        gamma = exact_entropic_gamma<Q>(f, ds, dh, omega);
      } else {
        // Complex step: the minimiser of the real parts by the same bisection,
        // then Newton steps on the stationarity condition dH/dt = 0 in complex
        // arithmetic. At the real root each step leaves the real part in
        // place and puts the first-order change of the root, -(dF/df . dv) /
        // (dF/dt) (implicit function theorem), into the imaginary part.
        const VelocitySet<Q>& v = vs<Q>();
        double fr[Q], dsr[Q], dhr[Q];
        for (int i = 0; i < Q; ++i) {
          fr[i] = re(f[i]);
          dsr[i] = re(ds[i]);
          dhr[i] = re(dh[i]);
        }
        T t = 0.5 * omega * exact_entropic_gamma<Q>(fr, dsr, dhr, omega);
        for (int it = 0; it < 3; ++it) {
          T dH = 0.0, d2H = 0.0;
          for (int i = 0; i < Q; ++i) {
            const T fs = f[i] - omega * ds[i] - t * dh[i];
            dH -= dh[i] * (std::log(fs / v.w[i]) + 1.0);
            d2H += dh[i] * dh[i] / fs;
          }
          t = t - dH / d2H;
        }
        gamma = 2.0 * t / omega;
      }
    }
  }
  // relaxation rates per group: kinematic 0, shear omega, hom omega*gamma/2
  // f* = f - M^{-1} S M (f - f^eq)
  T mrelaxed[Q];
  for (int r = 0; r < Q; ++r) {
    T s = 0.0;
    if (mb.group[r] == 1) s = omega;
    if (mb.group[r] == 2) s = omega * gamma / 2.0;
    mrelaxed[r] = s * m[r];
  }
  for (int i = 0; i < Q; ++i) {
    T acc = 0.0;
    for (int r = 0; r < Q; ++r) acc += mb.Minv[i][r] * mrelaxed[r];
    fstar[i] = f[i] - acc;
  }
  if (gamma_out) *gamma_out = gamma;
  if (ds_out)
    for (int i = 0; i < Q; ++i) ds_out[i] = ds[i];
  if (dh_out)
    for (int i = 0; i < Q; ++i) dh_out[i] = dh[i];
}

// One time step: collide every node, then pull-stream periodically.
// gamma_cell (optional) receives the gamma used at each node.
template <int Q, class T>
void step(int n, double omega, int mode, const T* f, T* fnew, T* post, double* gamma_cell) {
  const VelocitySet<Q>& v = vs<Q>();
  const int64_t ncell = int64_t(n) * n * n;
#pragma omp parallel for schedule(static)
  for (int64_t cell = 0; cell < ncell; ++cell) {
    T g;
    collide<Q>(f + cell * Q, omega, mode, post + cell * Q, &g, (T*)nullptr, (T*)nullptr);
    if (gamma_cell) gamma_cell[cell] = re(g);
  }
#pragma omp parallel for schedule(static)
  for (int z = 0; z < n; ++z)
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        int64_t cell = (int64_t(z) * n + y) * n + x;
        for (int i = 0; i < Q; ++i) {
          int xs = (x - v.c[i][0] + n) % n;
          int ys = (y - v.c[i][1] + n) % n;
          int zs = (z - v.c[i][2] + n) % n;
          int64_t src = (int64_t(zs) * n + ys) * n + xs;
          fnew[cell * Q + i] = post[src * Q + i];
        }
      }
}

template <int Q, class T>
void run(int n, int steps, double omega, int mode, T* f, double* gamma_stats) {
  const int64_t len = int64_t(n) * n * n * Q;
  std::vector<T> tmp(len), post(len);
  std::vector<double> gcell(gamma_stats ? int64_t(n) * n * n : 0);
  for (int s = 0; s < steps; ++s) {
    step<Q, T>(n, omega, mode, f, tmp.data(), post.data(), gamma_stats ? gcell.data() : nullptr);
    std::memcpy(f, tmp.data(), sizeof(T) * len);
    if (gamma_stats) {
      double gmin = 1e300, gmax = -1e300, gsum = 0.0;
      for (double g : gcell) {
        gmin = std::fmin(gmin, g);
        gmax = std::fmax(gmax, g);
        gsum += g;
      }
      gamma_stats[3 * s + 0] = gmin;
      gamma_stats[3 * s + 1] = gmax;
      gamma_stats[3 * s + 2] = gsum / double(gcell.size());
    }
  }
}

// D3Q27 or D3Q19 by the number of velocities q (any other q: no effect, 0)
template <class F>
int32_t with_lattice(int32_t q, F&& f) {
  if (q == 27) {
    f(std::integral_constant<int, 27>{});
    return 1;
  }
  if (q == 19) {
    f(std::integral_constant<int, 19>{});
    return 1;
  }
  return 0;
}

}  // namespace

extern "C" {

// Velocity set: c[q][3] integers and w[q]. Returns 0 for an unknown q.
int32_t oracle_velocity_set(int32_t q, int32_t* c, double* w) {
  return with_lattice(q, [&](auto qc) {
    constexpr int Q = decltype(qc)::value;
    const VelocitySet<Q>& v = vs<Q>();
    for (int i = 0; i < Q; ++i) {
      for (int a = 0; a < 3; ++a) c[3 * i + a] = v.c[i][a];
      w[i] = v.w[i];
    }
  });
}

// Moment matrix (row-major q x q), its inverse and the group of each row.
int32_t oracle_moment_basis(int32_t q, double* M, double* Minv, int32_t* group) {
  return with_lattice(q, [&](auto qc) {
    constexpr int Q = decltype(qc)::value;
    const MomentBasis<Q>& b = basis<Q>();
    for (int r = 0; r < Q; ++r) {
      group[r] = b.group[r];
      for (int k = 0; k < Q; ++k) {
        M[r * Q + k] = b.M[r][k];
        Minv[r * Q + k] = b.Minv[r][k];
      }
    }
  });
}

int32_t oracle_equilibrium(int32_t q, double rho, const double* u, double* feq) {
  return with_lattice(q, [&](auto qc) { equilibrium<decltype(qc)::value, double>(rho, u, feq); });
}

int32_t oracle_collide(int32_t q, const double* f, double omega, int32_t mode, double* fstar, double* gamma,
                       double* ds, double* dh) {
  return with_lattice(q, [&](auto qc) { collide<decltype(qc)::value, double>(f, omega, mode, fstar, gamma, ds, dh); });
}

int32_t oracle_collide_z(int32_t q, const double* f_ri, double omega, int32_t mode, double* fstar_ri,
                         double* gamma_ri) {
  return with_lattice(q, [&](auto qc) {
    collide<decltype(qc)::value, cplx>(reinterpret_cast<const cplx*>(f_ri), omega, mode,
                                       reinterpret_cast<cplx*>(fstar_ri), reinterpret_cast<cplx*>(gamma_ri),
                                       nullptr, nullptr);
  });
}

// Advance f[n^3][q] by `steps` steps in place. gamma_stats (optional):
// steps x (min, max, mean) of the gamma used at each step.
int32_t oracle_run(int32_t q, int32_t n, int32_t steps, double omega, int32_t mode, double* f, double* gamma_stats,
                   int32_t threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
  return with_lattice(q, [&](auto qc) { run<decltype(qc)::value, double>(n, steps, omega, mode, f, gamma_stats); });
}

// Same in complex arithmetic (interleaved re/im) for complex-step derivatives:
// mode 0 (closed-form gamma) or 2 (exact gamma, see collide).
int32_t oracle_run_z(int32_t q, int32_t n, int32_t steps, double omega, int32_t mode, double* f_ri,
                     int32_t threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
  if (mode != 0 && mode != 2) return 0;
  return with_lattice(q, [&](auto qc) {
    run<decltype(qc)::value, cplx>(n, steps, omega, mode, reinterpret_cast<cplx*>(f_ri), nullptr);
  });
}

// Equilibrium populations f = f^eq(1, u) for every node; u is [3][ncell].
int32_t oracle_init_field(int32_t q, int64_t ncell, const double* u, double* f) {
  return with_lattice(q, [&](auto qc) {
    constexpr int Q = decltype(qc)::value;
    for (int64_t cell = 0; cell < ncell; ++cell) {
      double uc[3] = {u[cell], u[ncell + cell], u[2 * ncell + cell]};
      equilibrium<Q, double>(1.0, uc, f + cell * Q);
    }
  });
}

int32_t oracle_init_field_z(int32_t q, int64_t ncell, const double* u_ri, double* f_ri) {
  const cplx* u = reinterpret_cast<const cplx*>(u_ri);
  cplx* f = reinterpret_cast<cplx*>(f_ri);
  return with_lattice(q, [&](auto qc) {
    constexpr int Q = decltype(qc)::value;
    for (int64_t cell = 0; cell < ncell; ++cell) {
      cplx uc[3] = {u[cell], u[ncell + cell], u[2 * ncell + cell]};
      equilibrium<Q, cplx>(cplx(1.0), uc, f + cell * Q);
    }
  });
}

int32_t oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
