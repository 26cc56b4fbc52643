// HIP kernels (gfx950) of the library other than collide-and-stream:
// reductions, initial data, read-out and state access, the adjoint sweep and
// the plain copy kernel used as the bandwidth reference.
#include "lbm_device.h"

namespace mclbm {
namespace {

__global__ void __launch_bounds__(256)
    record_finalize_kernel(const double* partials, const Seg* segs, const DevSample* samples, double* out) {
  const Seg sg = segs[blockIdx.x];
  double v[kRecord] = {0, 0, 0, 0, 0, 0, 1e300, -1e300};
  for (int k = threadIdx.x; k < sg.nblocks; k += 256) {
    const double* p = partials + size_t(sg.first_block + k) * kRecord;
#pragma unroll
    for (int q = 0; q < 6; ++q) v[q] += p[q];
    v[6] = fmin(v[6], p[6]);
    v[7] = fmax(v[7], p[7]);
  }
  double res[kRecord];
  block_record<256>(v, res);
  if (threadIdx.x == 0) {
    const DevSample& sp = samples[sg.sample];
    const double ncell = double(uint64_t(1) << (3 * sp.log2n));
    double* o = out + size_t(sg.sample) * kRecord;
    o[0] = ncell + res[0];
    o[1] = res[1];
    o[2] = res[2];
    o[3] = res[3];
    o[4] = res[4] / ncell;
    o[5] = res[6];
    o[6] = res[7];
    o[7] = res[5] / ncell;
  }
}

// ---------------------------------------------------------------- initial data
// u0(x) = u0 [TGV(x) + amp * s(x)] with s from the (projected) coefficients yc[24].
struct Basis {
  double a[3][2];  // a[axis][0] = sin(2 x_axis), a[axis][1] = cos(2 x_axis)
};

__device__ __forceinline__ void initial_velocity(uint32_t cell, int l, double u0, double amp, const double* yc,
                                                 double (&u)[3], Basis& bs) {
  const uint32_t msk = (1u << l) - 1u;
  const double n = double(1u << l);
  const uint32_t x = cell & msk, y = (cell >> l) & msk, z = cell >> (2 * l);
  // x_k = 2 pi k / n: sin(x_k) = sinpi(2k/n), sin(2 x_k) = sinpi(4k/n)
  const double s1x = sinpi(2.0 * x / n), c1x = cospi(2.0 * x / n);
  const double s1y = sinpi(2.0 * y / n), c1y = cospi(2.0 * y / n);
  const double c1z = cospi(2.0 * z / n);
  bs.a[0][0] = sinpi(4.0 * x / n);
  bs.a[0][1] = cospi(4.0 * x / n);
  bs.a[1][0] = sinpi(4.0 * y / n);
  bs.a[1][1] = cospi(4.0 * y / n);
  bs.a[2][0] = sinpi(4.0 * z / n);
  bs.a[2][1] = cospi(4.0 * z / n);
  double s[3] = {0.0, 0.0, 0.0};
  for (int al = 0; al < 3; ++al)
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 2; ++k)
          s[al] += yc[8 * al + 4 * i + 2 * j + k] * bs.a[0][i] * bs.a[1][j] * bs.a[2][k];
  u[0] = u0 * (s1x * c1y * c1z + amp * 0.125 * s[0]);
  u[1] = u0 * (-c1x * s1y * c1z + amp * 0.125 * s[1]);
  u[2] = u0 * (amp * 0.125 * s[2]);
}

template <int QN, typename T>
__global__ void __launch_bounds__(256)
    init_kernel(T* pop, const DevSample* samples, const Seg* segs, int nseg, const double* ycoef) {
  const int b = blockIdx.x;
  const Seg sg = segs[find_segment(segs, nseg, b)];
  const DevSample& sp = samples[sg.sample];
  const int l = sp.log2n;
  const uint32_t cell = uint32_t(b - sg.first_block) * 256u + threadIdx.x;
  double u[3];
  Basis bs;
  initial_velocity(cell, l, sp.u0, sp.amp, ycoef + size_t(sg.sample) * 24, u, bs);
  const double usq15 = 1.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  T* base = pop + sp.offset;
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const double cu = double(cx(i)) * u[0] + double(cy(i)) * u[1] + double(cz(i)) * u[2];
    const double gi = weight<QN>(i) * (3.0 * cu + 4.5 * cu * cu - usq15);
    st(base + size_t(plane_of<QN>(i)) * sp.pstride, cell, T(gi));
  });
}

// ---------------------------------------------------------------- read-out and state access
template <int QN, typename T>
__global__ void __launch_bounds__(256)
    moments_kernel(const T* pop, const DevSample* samples, int sample, int parity, double* rho, double* u) {
  const DevSample& sp = samples[sample];
  const int l = sp.log2n;
  const uint32_t ncell = 1u << (3 * l);
  const Cell c = make_cell(blockIdx.x * 256u + threadIdx.x, l);
  T g[Q];
  load_state<QN>(pop + sp.offset, sp.pstride, c, parity & 1, g);
  double d = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const double v = double(g[i]);
    d += v;
    if constexpr (cx(i) != 0) jx += cx(i) * v;
    if constexpr (cy(i) != 0) jy += cy(i) * v;
    if constexpr (cz(i) != 0) jz += cz(i) * v;
  });
  const double r = 1.0 + d;
  if (rho) rho[c.cell] = r;
  if (u) {
    u[c.cell] = jx / r;
    u[size_t(ncell) + c.cell] = jy / r;
    u[2 * size_t(ncell) + c.cell] = jz / r;
  }
}

template <int QN, typename T>
__global__ void __launch_bounds__(256)
    get_state_kernel(const T* pop, const DevSample* samples, int sample, int parity, double* f) {
  const DevSample& sp = samples[sample];
  const int l = sp.log2n;
  const uint32_t ncell = 1u << (3 * l);
  const Cell c = make_cell(blockIdx.x * 256u + threadIdx.x, l);
  T g[Q];
  load_state<QN>(pop + sp.offset, sp.pstride, c, parity & 1, g);
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    f[size_t(plane_of<QN>(i)) * ncell + c.cell] = weight<QN>(i) + double(g[i]);
  });
}

template <int QN, typename T>
__global__ void __launch_bounds__(256)
    set_state_kernel(T* pop, const DevSample* samples, int sample, int parity, const double* f) {
  const DevSample& sp = samples[sample];
  const int l = sp.log2n;
  const uint32_t ncell = 1u << (3 * l);
  const Cell c = make_cell(blockIdx.x * 256u + threadIdx.x, l);
  T g[Q];
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    g[i] = T(f[size_t(plane_of<QN>(i)) * ncell + c.cell] - weight<QN>(i));
  });
  write_state<QN>(pop + sp.offset, sp.pstride, c, parity & 1, g);
}

// Populations (unshifted, double) of selected cells of one sample: f[k][27].
template <int QN, typename T>
__global__ void __launch_bounds__(64)
    gather_cells_kernel(const T* pop, const DevSample* samples, int sample, int parity, const int64_t* cells,
                        int count, double* f) {
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k >= count) return;
  const DevSample& sp = samples[sample];
  const int l = sp.log2n;
  const Cell c = make_cell(uint32_t(cells[k]), l);
  T g[Q];
  load_state<QN>(pop + sp.offset, sp.pstride, c, parity & 1, g);
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    f[size_t(k) * QN + plane_of<QN>(i)] = weight<QN>(i) + double(g[i]);
  });
}

template <int QN, typename T>
__global__ void poison_kernel(T* pop, const DevSample* samples, int sample, int parity, uint32_t cell, int k) {
  const DevSample& sp = samples[sample];
  const int l = sp.log2n;
  const Cell c = make_cell(cell, l);
  T* base = pop + sp.offset;
  const T nan = T(__builtin_nan(""));
  const int i = velocity_of_plane<QN>(k);
  // slot of population i of this node (see load_state)
  if (!(parity & 1)) {
    base[size_t(k) * sp.pstride + cell] = nan;
  } else {
    const uint32_t nb = c.oz[1 - cz(i)] + c.oy[1 - cy(i)] + c.ox[1 - cx(i)];
    base[size_t(plane_of<QN>(opposite(i))) * sp.pstride + nb] = nan;
  }
}

template <int QN, typename T>
__global__ void __launch_bounds__(256)
    canonical_copy_kernel(const T* pop, T* dst, const DevSample* samples, const Seg* segs, int nseg) {
  const int b = blockIdx.x;
  const Seg sg = segs[find_segment(segs, nseg, b)];
  const DevSample& sp = samples[sg.sample];
  const int l = sp.log2n;
  const Cell c = make_cell(uint32_t(b - sg.first_block) * 256u + threadIdx.x, l);
  T g[Q];
  load_state<QN>(pop + sp.offset, sp.pstride, c, sg.parity & 1, g);
  write_state<QN>(dst + sp.offset, sp.pstride, c, false, g);
}

// Adjoint vectors lam[q][n^3] (double, the population order of get_state)
// into or out of the natural layout of the storage type. No shift: an
// adjoint is a derivative, which the constant weights do not enter.
template <int QN, typename T>
__global__ void __launch_bounds__(256) put_adjoint_kernel(T* dst, const DevSample* samples, int sample,
                                                          const double* lam) {
  const DevSample& sp = samples[sample];
  const uint32_t ncell = 1u << (3 * sp.log2n);
  const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
  for_vel<QN>([&](auto ic) {
    constexpr int k = plane_of<QN>(decltype(ic)::value);
    dst[sp.offset + size_t(k) * sp.pstride + cell] = T(lam[size_t(k) * ncell + cell]);
  });
}

template <int QN, typename T>
__global__ void __launch_bounds__(256) get_adjoint_kernel(const T* src, const DevSample* samples, int sample,
                                                          double* lam) {
  const DevSample& sp = samples[sample];
  const uint32_t ncell = 1u << (3 * sp.log2n);
  const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
  for_vel<QN>([&](auto ic) {
    constexpr int k = plane_of<QN>(decltype(ic)::value);
    lam[size_t(k) * ncell + cell] = double(src[sp.offset + size_t(k) * sp.pstride + cell]);
  });
}

// ---------------------------------------------------------------- adjoint
// Seed: J = (1/M) sum_m KE_m with KE = (1/n^3) sum_x |u|^2 / 2, u = j / rho:
// dJ/dg_i(x) = (1 / (M n^3)) (c_i . u - |u|^2) / rho.
template <int QN, typename T>
__global__ void __launch_bounds__(256) adjoint_seed_kernel(const T* pop, T* lam, const DevSample* samples,
                                                           const Seg* segs, int nseg, double inv_m) {
  const int b = blockIdx.x;
  const Seg sg = segs[find_segment(segs, nseg, b)];
  const DevSample& sp = samples[sg.sample];
  const int l = sp.log2n;
  const uint32_t ncell = 1u << (3 * l);
  const Cell c = make_cell(uint32_t(b - sg.first_block) * 256u + threadIdx.x, l);
  T g[Q];
  load_state<QN>(pop + sp.offset, sp.pstride, c, sg.parity & 1, g);
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
  const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
  const double usq = ux * ux + uy * uy + uz * uz;
  const double coef = inv_m / double(ncell) / rho;
  T* lb = lam + sp.offset;
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const double cu = double(cx(i)) * ux + double(cy(i)) * uy + double(cz(i)) * uz;
    st(lb + size_t(plane_of<QN>(i)) * sp.pstride, c.cell, T(coef * (cu - usq)));
  });
}

// One reverse step: lambda_n(x) = (d collide / d g_n(x))^T [lambda_{n+1, i}(x + c_i)]_i,
// the transpose of "collide at x, then move population i to x + c_i".
// EXACT: the collision with the exact stabiliser of eq. (kbc_entropy), whose
// t = omega gamma / 2 is the root of F(t) = sum_i dh_i ln(f*_i / w_i) with
// f*_i = w_i + g_i - omega ds_i - t dh_i; by the implicit function theorem
// dt = (dF at fixed t) / D, D = sum_i dh_i^2 / f*_i, so the adjoint of t
// reaches F's inputs (dh, ds and g directly) with weight tbar / D.
template <int QN, typename T, bool BUF, bool EXACT>
__global__ void __launch_bounds__(256) adjoint_step_kernel(const T* state, const T* lam_in, T* lam_out,
                                                           const DevSample* samples, const Seg* segs, int nseg) {
  const int b = blockIdx.x;
  const Seg sg = segs[find_segment(segs, nseg, b)];
  const DevSample& sp = samples[sg.sample];
  const int l = sp.log2n;
  const Cell c = make_cell(uint32_t(b - sg.first_block) * 256u + threadIdx.x, l);
  const Relax<T> rp = relax_of<T>(sp);
  // every array is streamed once per reverse step: non-temporal accesses
  using Planes = typename std::conditional<BUF, BufPlanes<T, true, QN>, PtrPlanes<T, true, QN>>::type;
  const Planes st_in(const_cast<T*>(state) + sp.offset, sp.pstride);
  const Planes lam_src(const_cast<T*>(lam_in) + sp.offset, sp.pstride);
  const Planes lam_dst(lam_out + sp.offset, sp.pstride);

  // lambda is pulled from x + c_i; rows longer than a wave (and held whole by
  // the block) are read at the node's own x and shifted by lane exchange
  const uint32_t n = 1u << l;
  const bool rows = n > 64u && n <= 256u;
  __shared__ EdgeLds<T, 256> edge;
  T g[Q], nu[Q];
  if (rows) {
    for_vel<QN>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      g[i] = st_in.load(i, c.cell);
      nu[i] = lam_src.load(i, neighbour_yz<i, +1>(c));
    });
    row_shift<QN, -1, 256>(nu, edge, n);
  } else {
    for_vel<QN>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      g[i] = st_in.load(i, c.cell);
      nu[i] = lam_src.load(i, neighbour<i, +1>(c));
    });
  }

  // forward intermediates, as in kbc_collide
  const Macro<T> m = macroscopic<QN>(g);
  T fneq[Q];
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    fneq[i] = g[i] - geq<QN, i>(m);
  });
  const Shear<T> s = shear_coefficients<QN>(fneq);
  T A = T(0), B = T(0);
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const T r = recip(T(weight<QN>(i)) + geq<QN, i>(m));
    if constexpr (nonzeros(i) == 1 || nonzeros(i) == 2) {
      const T ds = shear_part<i>(s);
      const T dh = fneq[i] - ds;
      A += ds * dh * r;
      B += dh * dh * r;
    } else {
      B += fneq[i] * fneq[i] * r;
    }
  });
  const bool active = B > equilibrium_threshold<T>(m);  // as in the forward collision
  T gamma = T(2);
  if (active) gamma = rp.two_over_omega - rp.kappa * (A / B);
  T t = T(0.5) * rp.omega * gamma;
  if constexpr (EXACT) {
    // the forward collision's t, from the same start and with the same steps
    if (active) {
      T ge[Q], dh[Q], bs[Q];
      for_vel<QN>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        ge[i] = geq<QN, i>(m);
      });
      exact_terms<QN>(ge, fneq, s, rp.eps, dh, bs);
      t = exact_entropic_t<QN>(dh, bs, m, t);
    }
  }

  // reverse sweep (the direct path of g* = g - omega ds - t dh hands nu to g
  // unchanged; tbar is the adjoint of t)
  T tbar = T(0);
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (nonzeros(i) == 1 || nonzeros(i) == 2) tbar -= nu[i] * (fneq[i] - shear_part<i>(s));
    else tbar -= nu[i] * fneq[i];
  });
  T Abar = T(0), Bbar = T(0), Fbar = T(0);
  if (active) {
    if constexpr (EXACT) {
      T d = T(0);
      for_vel<QN>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        T ds = T(0);
        if constexpr (nonzeros(i) == 1 || nonzeros(i) == 2) ds = shear_part<i>(s);
        const T dh = fneq[i] - ds;
        const T gs = (((geq<QN, i>(m) - ds) + rp.eps * ds) + dh) - t * dh;  // f*_i - w_i
        d += dh * dh * recip(T(weight<QN>(i)) + gs);
      });
      Fbar = tbar / d;
    } else {
      const T gbar = T(0.5) * rp.omega * tbar;
      Abar = -rp.kappa * gbar / B;
      Bbar = rp.kappa * gbar * (A / B) / B;  // B * B would underflow in float
    }
  }
  // adjoints of fneq (through dh and the weights) and of the shear coefficients
  T fbar[Q], geqbar[Q];
  T dsxb = T(0), dsyb = T(0), dszb = T(0), exyb = T(0), exzb = T(0), eyzb = T(0);
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    T dsb, dhb;
    if constexpr (EXACT) {
      // dF = sum_i [ln(f*_i / w_i) - t dh_i / f*_i] d(dh_i) - omega dh_i / f*_i d(ds_i)
      //      + dh_i / f*_i d(g_i), with g_i = g^eq_i + fneq_i
      T ds = T(0);
      if constexpr (nonzeros(i) == 1 || nonzeros(i) == 2) ds = shear_part<i>(s);
      const T dh = fneq[i] - ds;
      T x = T(0), lg = T(0);
      if (active) {
        constexpr double w = weight<QN>(i);
        const T gs = geq<QN, i>(m) + (fneq[i] - rp.omega * ds) - t * dh;
        x = Fbar * dh * recip(T(w) + gs);
        lg = Fbar * log1p_acc(gs * T(1.0 / w));
      }
      if constexpr (nonzeros(i) == 1 || nonzeros(i) == 2) dsb = -rp.omega * nu[i] - rp.omega * x;
      else dsb = T(0);
      dhb = -t * nu[i] + lg - t * x;
      geqbar[i] = x;
      fbar[i] = dhb + x;
    } else {
      const T r = recip(T(weight<QN>(i)) + geq<QN, i>(m));
      T rbar;
      T ds = T(0), dh;
      if constexpr (nonzeros(i) == 1 || nonzeros(i) == 2) {
        ds = shear_part<i>(s);
        dh = fneq[i] - ds;
        dsb = -rp.omega * nu[i] + Abar * dh * r;
        dhb = -t * nu[i] + Abar * ds * r + T(2) * Bbar * dh * r;
        rbar = Abar * ds * dh + Bbar * dh * dh;
      } else {
        dh = fneq[i];
        dsb = T(0);
        dhb = -t * nu[i] + T(2) * Bbar * dh * r;
        rbar = Bbar * dh * dh;
      }
      geqbar[i] = -rbar * r * r;  // through f^eq = w + g^eq
      fbar[i] = dhb;              // dh = fneq - ds
    }
    dsb -= dhb;
    if constexpr (nonzeros(i) == 1) {
      if constexpr (cx(i) != 0) dsxb += dsb;
      else if constexpr (cy(i) != 0) dsyb += dsb;
      else dszb += dsb;
    } else if constexpr (nonzeros(i) == 2) {
      if constexpr (cz(i) == 0) exyb += signed_term<cx(i) * cy(i)>(dsb);
      else if constexpr (cy(i) == 0) exzb += signed_term<cx(i) * cz(i)>(dsb);
      else eyzb += signed_term<cy(i) * cz(i)>(dsb);
    }
  });
  // dsz = -(dsx + dsy); dsx = (2 Nxz - Nyz)/6; dsy = (2 Nyz - Nxz)/6
  const T dsxt = dsxb - dszb, dsyt = dsyb - dszb;
  const T sixth = T(1) / T(6);
  const T nxzb = (T(2) * dsxt - dsyt) * sixth;
  const T nyzb = (T(2) * dsyt - dsxt) * sixth;
  const T pxxb = nxzb, pyyb = nyzb, pzzb = -(nxzb + nyzb);
  const T pxyb = T(0.25) * exyb, pxzb = T(0.25) * exzb, pyzb = T(0.25) * eyzb;
  // second moments of fneq
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    T acc = fbar[i];
    if constexpr (cx(i) != 0) acc += pxxb;
    if constexpr (cy(i) != 0) acc += pyyb;
    if constexpr (cz(i) != 0) acc += pzzb;
    if constexpr (cx(i) * cy(i) != 0) acc += signed_term<cx(i) * cy(i)>(pxyb);
    if constexpr (cx(i) * cz(i) != 0) acc += signed_term<cx(i) * cz(i)>(pxzb);
    if constexpr (cy(i) * cz(i) != 0) acc += signed_term<cy(i) * cz(i)>(pyzb);
    fbar[i] = acc;
    geqbar[i] -= acc;  // fneq = g - geq
  });
  // g^eq_i = w_i [drho + 3 c.j + inv (4.5 (c.j)^2 - 1.5 |j|^2)], inv = 1 / (1 + drho)
  T S = T(0), jxb = T(0), jyb = T(0), jzb = T(0), invb = T(0);
  const T jsq15 = T(1.5) * (m.jx * m.jx + m.jy * m.jy + m.jz * m.jz);
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const T si = T(weight<QN>(i)) * geqbar[i];
    S += si;
    if constexpr (nonzeros(i) == 0) {
      invb -= si * jsq15;
    } else {
      const T cj = cdot<i>(m.jx, m.jy, m.jz);
      invb += si * (T(4.5) * cj * cj - jsq15);
      const T coef = si * (T(3) + T(9) * m.inv * cj);
      if constexpr (cx(i) != 0) jxb += signed_term<cx(i)>(coef);
      if constexpr (cy(i) != 0) jyb += signed_term<cy(i)>(coef);
      if constexpr (cz(i) != 0) jzb += signed_term<cz(i)>(coef);
    }
  });
  jxb -= T(3) * m.inv * S * m.jx;
  jyb -= T(3) * m.inv * S * m.jy;
  jzb -= T(3) * m.inv * S * m.jz;
  const T drhob = S - m.inv * m.inv * invb;
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    T v = nu[i] + fbar[i] + drhob;
    if constexpr (cx(i) != 0) v += signed_term<cx(i)>(jxb);
    if constexpr (cy(i) != 0) v += signed_term<cy(i)>(jyb);
    if constexpr (cz(i) != 0) v += signed_term<cz(i)>(jzb);
    lam_dst.store(i, c.cell, v);
  });
}

// dJ/du0(x) = sum_i lambda_0,i w_i [3 c_i + 9 (c_i.u0) c_i - 3 u0]; projected on the
// 24 basis products with factor amp * u0 / 8 (before the projection matrix).
template <int QN, typename T>
__global__ void __launch_bounds__(256) init_adjoint_kernel(const T* lam, const DevSample* samples, const Seg* segs,
                                                           int nseg, const double* ycoef, double* partials) {
  const int b = blockIdx.x;
  const Seg sg = segs[find_segment(segs, nseg, b)];
  const DevSample& sp = samples[sg.sample];
  const int l = sp.log2n;
  const uint32_t cell = uint32_t(b - sg.first_block) * 256u + threadIdx.x;
  double u[3];
  Basis bs;
  initial_velocity(cell, l, sp.u0, sp.amp, ycoef + size_t(sg.sample) * 24, u, bs);
  const T* lb = lam + sp.offset;
  double ub[3] = {0.0, 0.0, 0.0};
  for_vel<QN>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const double li = double(ld(lb + size_t(plane_of<QN>(i)) * sp.pstride, cell)) * weight<QN>(i);
    const double cu = double(cx(i)) * u[0] + double(cy(i)) * u[1] + double(cz(i)) * u[2];
    ub[0] += li * (3.0 * cx(i) + 9.0 * cu * cx(i) - 3.0 * u[0]);
    ub[1] += li * (3.0 * cy(i) + 9.0 * cu * cy(i) - 3.0 * u[1]);
    ub[2] += li * (3.0 * cz(i) + 9.0 * cu * cz(i) - 3.0 * u[2]);
  });
  const double scale = sp.amp * sp.u0 * 0.125;
  __shared__ double sh[4][24];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int p = 0; p < 24; ++p) {
    const int al = p >> 3, i = (p >> 2) & 1, j = (p >> 1) & 1, k = p & 1;
    double v = scale * ub[al] * bs.a[0][i] * bs.a[1][j] * bs.a[2][k];
    v = wave_sum(v);
    if (lane == 0) sh[wave][p] = v;
  }
  __syncthreads();
  if (threadIdx.x < 24) {
    const int p = threadIdx.x;
    partials[size_t(b) * 24 + p] = ((sh[0][p] + sh[1][p]) + sh[2][p]) + sh[3][p];
  }
}

__global__ void __launch_bounds__(256) init_adjoint_finalize_kernel(const double* partials, const Seg* segs,
                                                                    const DevSample* samples, const double* pmat,
                                                                    double* dJdY) {
  const Seg sg = segs[blockIdx.x];
  __shared__ double red[256];
  __shared__ double dprime[24];
  for (int p = 0; p < 24; ++p) {
    double acc = 0.0;
    for (int k = threadIdx.x; k < sg.nblocks; k += 256) acc += partials[size_t(sg.first_block + k) * 24 + p];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) dprime[p] = red[0];
    __syncthreads();
  }
  if (threadIdx.x < 24) {
    const int q = threadIdx.x;
    double v = dprime[q];
    if (samples[sg.sample].project) {
      // Y' = P Y, so dJ/dY = P^T dJ/dY'
      v = 0.0;
      for (int p = 0; p < 24; ++p) v += pmat[p * 24 + q] * dprime[p];
    }
    dJdY[size_t(sg.sample) * 24 + q] = v;
  }
}

__global__ void extract_kernel(const double* records, int m, int field, double* out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < m) out[s] = records[size_t(s) * kRecord + field];
}

// Energy per unit volume of sample s at record k, in lattice units: the
// kinetic energy of a record of the step kernel (field 4, the mean of |u|^2/2
// over the nodes), or the shell spectrum of eq. (energySpecDisc) summed over
// kappa = 0..n/2 in fixed order.
struct RecordEnergy {
  const double* rec;
  int m;
  __device__ double operator()(int k, int s) const { return rec[(size_t(k) * m + s) * kRecord + 4]; }
};
struct SpectrumEnergy {
  const double* ek;
  int count, len;
  __device__ double operator()(int k, int s) const {
    const double* e = ek + (size_t(k) * count + s) * len;
    double sum = 0.0;
    for (int j = 0; j < len; ++j) sum += e[j];
    return sum;
  }
};

// Dissipation rate per sample and record, d = -dE/dt in physical units (E /
// u0^2 against t = steps * (2 pi / n) * u0): centred differences inside the
// series, one-sided at its ends; and eta = (eps^3 / mean_s d)^(1/4). One
// thread per record.
template <class Energy>
__global__ void dissipation_kernel(Energy energy, const DissSample* smp, int m, int nrec, int64_t first_tick,
                                   int record_every, double eps, double* diss, double* eta) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nrec) return;
  const int k0 = k > 0 ? k - 1 : 0, k1 = k + 1 < nrec ? k + 1 : nrec - 1;
  double mean = 0.0;
  for (int s = 0; s < m; ++s) {
    const DissSample& d = smp[s];
    const double e0 = energy(k0, s) * d.inv_u0sq;
    const double e1 = energy(k1, s) * d.inv_u0sq;
    const double t0 = double((first_tick + int64_t(k0) * record_every) / d.stride) * d.dt;
    const double t1 = double((first_tick + int64_t(k1) * record_every) / d.stride) * d.dt;
    const double v = -(e1 - e0) / (t1 - t0);
    diss[size_t(k) * m + s] = v;
    mean += v;
  }
  if (eta) eta[k] = sqrt(sqrt(eps * eps * eps / (mean / m)));
}

// One 16-byte element per thread with non-temporal loads and stores (the
// fastest plain copy measured on gfx950: 6.5-6.6 TB/s on 4 GiB, against
// 6.1-6.2 TB/s with ordinary accesses and 5.1-5.3 TB/s with grid-stride
// loops).
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) stream_copy_kernel(const f32x4* __restrict__ src, f32x4* __restrict__ dst,
                                                          size_t n4) {
  const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n4) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// f(lattice, value of the storage type) for a run-time lattice and precision
template <typename F>
hipError_t dispatch(int q, int precision, F&& f) {
  using Q27 = std::integral_constant<int, 27>;
  using Q19 = std::integral_constant<int, 19>;
  if (q == 27) return precision == 0 ? f(Q27{}, double{}) : f(Q27{}, float{});
  if (q == 19) return precision == 0 ? f(Q19{}, double{}) : f(Q19{}, float{});
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_step(int q, int precision, StepKind kind, const StepLaunch& L, hipStream_t s) {
  if (q == 27) return precision == 0 ? launch_step_d3q27_f64(kind, L, s) : launch_step_d3q27_f32(kind, L, s);
  if (q == 19) return precision == 0 ? launch_step_d3q19_f64(kind, L, s) : launch_step_d3q19_f32(kind, L, s);
  return hipErrorInvalidValue;
}

hipError_t launch_record_finalize(const double* partials, const Seg* segs, int32_t nseg, const DevSample* samples,
                                  double* out, hipStream_t s) {
  hipLaunchKernelGGL(record_finalize_kernel, dim3(nseg), dim3(256), 0, s, partials, segs, samples, out);
  return hipGetLastError();
}

hipError_t launch_init(int q, int precision, void* pop, const DevSample* samples, const Seg* segs, int32_t nseg,
                       int32_t total_blocks, const double* ycoef, hipStream_t s) {
  return dispatch(q, precision, [&](auto qc, auto tc) {
    using T = decltype(tc);
    hipLaunchKernelGGL((init_kernel<decltype(qc)::value, T>), dim3(total_blocks), dim3(256), 0, s,
                       static_cast<T*>(pop), samples, segs, nseg, ycoef);
    return hipGetLastError();
  });
}

hipError_t launch_moments(int q, int precision, const void* pop, const DevSample* samples, int32_t sample, int32_t n,
                          int32_t parity, double* rho, double* u, hipStream_t s) {
  const unsigned blocks = unsigned((uint64_t(n) * n * n) / 256);
  return dispatch(q, precision, [&](auto qc, auto tc) {
    using T = decltype(tc);
    hipLaunchKernelGGL((moments_kernel<decltype(qc)::value, T>), dim3(blocks), dim3(256), 0, s,
                       static_cast<const T*>(pop), samples, sample, parity, rho, u);
    return hipGetLastError();
  });
}

hipError_t launch_get_state(int q, int precision, const void* pop, const DevSample* samples, int32_t sample,
                            int32_t n, int32_t parity, double* f, hipStream_t s) {
  const unsigned blocks = unsigned((uint64_t(n) * n * n) / 256);
  return dispatch(q, precision, [&](auto qc, auto tc) {
    using T = decltype(tc);
    hipLaunchKernelGGL((get_state_kernel<decltype(qc)::value, T>), dim3(blocks), dim3(256), 0, s,
                       static_cast<const T*>(pop), samples, sample, parity, f);
    return hipGetLastError();
  });
}

hipError_t launch_set_state(int q, int precision, void* pop, const DevSample* samples, int32_t sample, int32_t n,
                            int32_t parity, const double* f, hipStream_t s) {
  const unsigned blocks = unsigned((uint64_t(n) * n * n) / 256);
  return dispatch(q, precision, [&](auto qc, auto tc) {
    using T = decltype(tc);
    hipLaunchKernelGGL((set_state_kernel<decltype(qc)::value, T>), dim3(blocks), dim3(256), 0, s,
                       static_cast<T*>(pop), samples, sample, parity, f);
    return hipGetLastError();
  });
}

hipError_t launch_gather_cells(int q, int precision, const void* pop, const DevSample* samples, int32_t sample,
                               int32_t parity, const int64_t* cells, int32_t count, double* f, hipStream_t s) {
  const unsigned blocks = unsigned((count + 63) / 64);
  return dispatch(q, precision, [&](auto qc, auto tc) {
    using T = decltype(tc);
    hipLaunchKernelGGL((gather_cells_kernel<decltype(qc)::value, T>), dim3(blocks), dim3(64), 0, s,
                       static_cast<const T*>(pop), samples, sample, parity, cells, count, f);
    return hipGetLastError();
  });
}

hipError_t launch_poison(int q, int precision, void* pop, const DevSample* samples, int32_t sample, int32_t parity,
                         int64_t cell, int32_t k, hipStream_t s) {
  return dispatch(q, precision, [&](auto qc, auto tc) {
    using T = decltype(tc);
    hipLaunchKernelGGL((poison_kernel<decltype(qc)::value, T>), dim3(1), dim3(1), 0, s, static_cast<T*>(pop),
                       samples, sample, parity, uint32_t(cell), k);
    return hipGetLastError();
  });
}

hipError_t launch_canonical_copy(int q, int precision, const void* pop, void* dst, const DevSample* samples,
                                 const Seg* segs, int32_t nseg, int32_t total_blocks, hipStream_t s) {
  return dispatch(q, precision, [&](auto qc, auto tc) {
    using T = decltype(tc);
    hipLaunchKernelGGL((canonical_copy_kernel<decltype(qc)::value, T>), dim3(total_blocks), dim3(256), 0, s,
                       static_cast<const T*>(pop), static_cast<T*>(dst), samples, segs, nseg);
    return hipGetLastError();
  });
}

hipError_t launch_put_adjoint(int q, int precision, void* dst, const DevSample* samples, int32_t sample, int32_t n,
                              const double* lam, hipStream_t s) {
  const unsigned blocks = unsigned((uint64_t(n) * n * n) / 256);
  return dispatch(q, precision, [&](auto qc, auto tc) {
    using T = decltype(tc);
    hipLaunchKernelGGL((put_adjoint_kernel<decltype(qc)::value, T>), dim3(blocks), dim3(256), 0, s,
                       static_cast<T*>(dst), samples, sample, lam);
    return hipGetLastError();
  });
}

hipError_t launch_get_adjoint(int q, int precision, const void* src, const DevSample* samples, int32_t sample,
                              int32_t n, double* lam, hipStream_t s) {
  const unsigned blocks = unsigned((uint64_t(n) * n * n) / 256);
  return dispatch(q, precision, [&](auto qc, auto tc) {
    using T = decltype(tc);
    hipLaunchKernelGGL((get_adjoint_kernel<decltype(qc)::value, T>), dim3(blocks), dim3(256), 0, s,
                       static_cast<const T*>(src), samples, sample, lam);
    return hipGetLastError();
  });
}

hipError_t launch_adjoint_seed(int q, int precision, const void* pop, void* lam, const DevSample* samples,
                               const Seg* segs, int32_t nseg, int32_t total_blocks, double inv_m, hipStream_t s) {
  return dispatch(q, precision, [&](auto qc, auto tc) {
    using T = decltype(tc);
    hipLaunchKernelGGL((adjoint_seed_kernel<decltype(qc)::value, T>), dim3(total_blocks), dim3(256), 0, s,
                       static_cast<const T*>(pop), static_cast<T*>(lam), samples, segs, nseg, inv_m);
    return hipGetLastError();
  });
}

hipError_t launch_adjoint_step(int q, int precision, const void* state, const void* lam_in, void* lam_out,
                               const DevSample* samples, const Seg* segs, int32_t nseg, int32_t total_blocks,
                               int32_t buffer_ok, int32_t exact_gamma, hipStream_t s) {
  return dispatch(q, precision, [&](auto qc, auto tc) {
    constexpr int QN = decltype(qc)::value;
    using T = decltype(tc);
    const T* a = static_cast<const T*>(state);
    const T* b = static_cast<const T*>(lam_in);
    T* o = static_cast<T*>(lam_out);
    const dim3 grid(total_blocks), blk(256);
    if (exact_gamma) {
      // FP64 only (the host refuses FP32): see mclbm_backward
      if constexpr (!std::is_same<T, double>::value) return hipErrorInvalidValue;
      else if (buffer_ok)
        hipLaunchKernelGGL((adjoint_step_kernel<QN, T, true, true>), grid, blk, 0, s, a, b, o, samples, segs, nseg);
      else
        hipLaunchKernelGGL((adjoint_step_kernel<QN, T, false, true>), grid, blk, 0, s, a, b, o, samples, segs, nseg);
    } else if (buffer_ok) {
      hipLaunchKernelGGL((adjoint_step_kernel<QN, T, true, false>), grid, blk, 0, s, a, b, o, samples, segs, nseg);
    } else {
      hipLaunchKernelGGL((adjoint_step_kernel<QN, T, false, false>), grid, blk, 0, s, a, b, o, samples, segs, nseg);
    }
    return hipGetLastError();
  });
}

hipError_t launch_init_adjoint(int q, int precision, const void* lam, const DevSample* samples, const Seg* segs,
                               int32_t nseg, int32_t total_blocks, const double* ycoef, double* partials,
                               hipStream_t s) {
  return dispatch(q, precision, [&](auto qc, auto tc) {
    using T = decltype(tc);
    hipLaunchKernelGGL((init_adjoint_kernel<decltype(qc)::value, T>), dim3(total_blocks), dim3(256), 0, s,
                       static_cast<const T*>(lam), samples, segs, nseg, ycoef, partials);
    return hipGetLastError();
  });
}

hipError_t launch_init_adjoint_finalize(const double* partials, const Seg* segs, int32_t nseg,
                                        const DevSample* samples, const double* pmat, double* dJdY,
                                        hipStream_t s) {
  hipLaunchKernelGGL(init_adjoint_finalize_kernel, dim3(nseg), dim3(256), 0, s, partials, segs, samples, pmat, dJdY);
  return hipGetLastError();
}

hipError_t launch_extract(const double* records, int32_t m, int32_t field, double* out, hipStream_t s) {
  hipLaunchKernelGGL(extract_kernel, dim3((m + 255) / 256), dim3(256), 0, s, records, m, field, out);
  return hipGetLastError();
}

hipError_t launch_dissipation(const double* records, const DissSample* smp, int32_t m, int32_t nrec,
                              int64_t first_tick, int32_t record_every, double eps, double* diss, double* eta,
                              hipStream_t s) {
  hipLaunchKernelGGL(dissipation_kernel<RecordEnergy>, dim3((nrec + 63) / 64), dim3(64), 0, s,
                     RecordEnergy{records, m}, smp, m, nrec, first_tick, record_every, eps, diss, eta);
  return hipGetLastError();
}

hipError_t launch_dissipation_spectra(const double* ek, int32_t n, const DissSample* smp, int32_t count,
                                      int32_t nrec, int64_t first_tick, int32_t record_every, double eps,
                                      double* diss, double* eta, hipStream_t s) {
  hipLaunchKernelGGL(dissipation_kernel<SpectrumEnergy>, dim3((nrec + 63) / 64), dim3(64), 0, s,
                     SpectrumEnergy{ek, count, n / 2 + 1}, smp, count, nrec, first_tick, record_every, eps, diss,
                     eta);
  return hipGetLastError();
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const size_t n4 = bytes / 16;
  const size_t blocks = (n4 + 255) / 256;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(stream_copy_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<const f32x4*>(src),
                     static_cast<f32x4*>(dst), n4);
  return hipGetLastError();
}

}  // namespace mclbm
