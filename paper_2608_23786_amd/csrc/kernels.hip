// HIP kernels (gfx950) of the Monte Carlo KBC lattice Boltzmann library.
//
// State layout: per sample, 27 population planes of n^3 values (SoA),
// plane i holds velocity i, cells C-ordered [z][y][x]. Values are shifted:
// g_i = f_i - w_i (stored in float or double). The state is updated in place
// with the AA pattern: on an even step a node reads its own 27 slots and
// writes the post-collision populations back into the opposite slots of the
// same node; on an odd step it reads population i from slot 26-i of node
// x - c_i and writes the post-collision population i into slot i of node
// x + c_i. Every slot is read and written by exactly one thread per step, so
// the update is race free, and one step moves 27 loads + 27 stores per node.
//
// Collision (eqs. (equilibrium), (kbcCollision), (entropyControl), Table 1):
//   rho = 1 + sum g, j = sum c g, u = j / rho,
//   g^eq_i = w_i [drho + 3 c_i.j + rho (4.5 (c_i.u)^2 - 1.5 |u|^2)],
//   f^neq = g - g^eq,
//   shear part ds: the population vector with the traceless normal-stress
//   differences Nxz, Nyz and the off-diagonal stresses of f^neq and no other
//   raw moment: faces (+-1,0,0): (2Nxz - Nyz)/6, (0,+-1,0): (2Nyz - Nxz)/6,
//   (0,0,+-1): -(Nxz + Nyz)/6; edges: cx cy Pxy/4 + cx cz Pxz/4 + cy cz Pyz/4;
//   rest and corners: 0.  Higher-order part dh = f^neq - ds.
//   gamma = 2/omega - (2 - 2/omega) <ds|dh>/<dh|dh>, <X|Y> = sum X_i Y_i / f^eq_i
//   (gamma = 2 when <dh|dh> <= 1e-30),
//   g* = g - omega ds - (omega gamma / 2) dh.
// Everything is computed in the storage precision from the shifted values,
// so the weights w_i never enter a subtraction of nearly equal numbers.

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "kernels.h"
#include "lattice.h"

namespace mclbm {
namespace {

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
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
struct Macro {
  T drho, jx, jy, jz, rho, inv, ux, uy, uz, usq15;
};

template <typename T>
__device__ __forceinline__ Macro<T> macroscopic(const T (&g)[Q]) {
  T d = g[0], x = T(0), y = T(0), z = T(0);
  static_for<1, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    d += g[i];
  });
  // momentum: +direction partial sums minus -direction partial sums
  T xp = T(0), xm = T(0), yp = T(0), ym = T(0), zp = T(0), zm = T(0);
  static_for<0, Q>([&](auto ic) {
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

// shifted equilibrium g^eq_i = f^eq_i - w_i
template <int i, typename T>
__device__ __forceinline__ T geq(const Macro<T>& m) {
  const T w = T(weight(i));
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
      constexpr double w3 = 3.0 * weight(i);
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
template <typename T>
__device__ __forceinline__ Shear<T> shear_coefficients(const T (&fneq)[Q]) {
  T pxx = T(0), pyy = T(0), pzz = T(0), pxy = T(0), pxz = T(0), pyz = T(0);
  static_for<0, Q>([&](auto ic) {
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

// KBC collision of one node in place: g <- g*. Between the passes g[] holds
// the shifted equilibrium, so every g^eq_i is evaluated once.
template <typename T>
__device__ __forceinline__ CellResult<T> kbc_collide(T (&g)[Q], const Relax<T>& rp) {
  CellResult<T> res;
  res.m = macroscopic(g);
  const Macro<T>& m = res.m;
  T fneq[Q];
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const T ge = geq<i>(m);
    fneq[i] = g[i] - ge;
    g[i] = ge;
  });
  const Shear<T> s = shear_coefficients(fneq);
  T A = T(0), B = T(0), fmin = T(1);
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const T feq = T(weight(i)) + g[i];
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
  T gamma = T(2);
  if (B > T(1e-30)) gamma = rp.two_over_omega - rp.kappa * (A / B);
  const T t = T(0.5) * rp.omega * gamma;
  // g* = g - omega ds - t dh = (g^eq - ds) + (2 - omega) ds + (1 - t) dh.
  // The shear relaxation enters through eps = 2 - omega, which keeps the
  // viscosity (proportional to eps for omega near 2) at full relative
  // precision even in float.
  const T one_t = T(1) - t;
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (nonzeros(i) == 1 || nonzeros(i) == 2) {
      const T ds = shear_part<i>(s);
      g[i] = (g[i] - ds) + rp.eps * ds + one_t * (fneq[i] - ds);
    } else {
      g[i] = g[i] + one_t * fneq[i];
    }
  });
  res.gamma = gamma;
  res.bad = !(m.rho > T(0)) || !(m.usq15 < T(1.5)) || !(fmin > T(0));
  return res;
}

// ---------------------------------------------------------------- addressing
struct Cell {
  uint32_t cell;
  uint32_t ox[3], oy[3], oz[3];  // neighbour coordinates along each axis: -1, 0, +1
};

__device__ __forceinline__ Cell make_cell(uint32_t cell, int l) {
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
__device__ __forceinline__ uint32_t neighbour(const Cell& c) {
  return c.oz[1 + s * cz(i)] + c.oy[1 + s * cy(i)] + c.ox[1 + s * cx(i)];
}

// element access with a 32-bit byte offset from a uniform plane base
template <typename T>
__device__ __forceinline__ T ld(const T* plane, uint32_t idx) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(plane) + idx * uint32_t(sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void st(T* plane, uint32_t idx, T v) {
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

template <typename T, bool NT>
struct BufPlanes {
  static constexpr int aux = NT ? kAuxNontemporal : 0;
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t plane_bytes;
  __device__ __forceinline__ BufPlanes(T* base, uint32_t pstride)
      : rsrc(__builtin_amdgcn_make_buffer_rsrc(base, 0, int(uint32_t(Q) * pstride * uint32_t(sizeof(T))), kBufferFlags)),
        plane_bytes(pstride * uint32_t(sizeof(T))) {}
  __device__ __forceinline__ T load(int plane, uint32_t idx) const {
    if constexpr (sizeof(T) == 4)
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rsrc, int(idx * 4u), int(plane * plane_bytes), aux));
    else
      return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rsrc, int(idx * 8u), int(plane * plane_bytes), aux));
  }
  __device__ __forceinline__ void store(int plane, uint32_t idx, T v) const {
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
template <typename T, bool NT>
struct PtrPlanes {
  T* base;
  uint32_t pstride;
  __device__ __forceinline__ PtrPlanes(T* b, uint32_t p) : base(b), pstride(p) {}
  __device__ __forceinline__ T load(int plane, uint32_t idx) const {
    if constexpr (NT) return __builtin_nontemporal_load(base + size_t(plane) * pstride + idx);
    else return ld(base + size_t(plane) * pstride, idx);
  }
  __device__ __forceinline__ void store(int plane, uint32_t idx, T v) const {
    if constexpr (NT) __builtin_nontemporal_store(v, base + size_t(plane) * pstride + idx);
    else st(base + size_t(plane) * pstride, idx, v);
  }
};

// populations of the post-stream state at a node, for either AA parity
template <typename T>
__device__ __forceinline__ void load_state(const T* base, uint32_t pstride, const Cell& c, bool odd, T (&g)[Q]) {
  if (!odd) {
    static_for<0, Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      g[i] = ld(base + size_t(i) * pstride, c.cell);
    });
  } else {
    static_for<0, Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      g[i] = ld(base + size_t(opposite(i)) * pstride, neighbour<i, -1>(c));
    });
  }
}

// the inverse mapping: write a post-stream state at a node
template <typename T>
__device__ __forceinline__ void write_state(T* base, uint32_t pstride, const Cell& c, bool odd, const T (&g)[Q]) {
  if (!odd) {
    static_for<0, Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      st(base + size_t(i) * pstride, c.cell, g[i]);
    });
  } else {
    static_for<0, Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      st(base + size_t(opposite(i)) * pstride, neighbour<i, -1>(c), g[i]);
    });
  }
}

__device__ __forceinline__ int remap_block(int b, int total, int xcd_remap) {
  // hardware dispatches workgroup b to XCD b % 8; give each XCD a contiguous run
  if (xcd_remap) {
    const int g8 = total & ~7;
    if (b < g8) b = (b & 7) * (g8 >> 3) + (b >> 3);
  }
  return b;
}

__device__ __forceinline__ int find_segment(const Seg* segs, int nseg, int b) {
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

// ---------------------------------------------------------------- collide and stream
template <typename T>
struct StepArgs {
  T* pop;
  T* dst;
  const DevSample* samples;
  const Seg* segs;
  int32_t nseg;
  int32_t total_blocks;
  int32_t xcd_remap;
  int32_t* flags;
  double* partials;
};

template <typename T, int BLOCK, StepKind KIND, bool BUF, bool NT>
__global__ void __launch_bounds__(BLOCK) kbc_step_kernel(StepArgs<T> a) {
  const int b = remap_block(blockIdx.x, a.total_blocks, a.xcd_remap);
  const Seg sg = a.segs[find_segment(a.segs, a.nseg, b)];
  const DevSample& sp = a.samples[sg.sample];
  const int l = sp.log2n;
  const Cell c = make_cell(uint32_t(b - sg.first_block) * BLOCK + threadIdx.x, l);
  using Planes = typename std::conditional<BUF, BufPlanes<T, NT>, PtrPlanes<T, NT>>::type;
  const Planes src(a.pop + sp.offset, sp.pstride);
  const bool odd = (KIND != kPush) && (sg.parity & 1);

  T g[Q];
  if (!odd) {
    static_for<0, Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      g[i] = src.load(i, c.cell);
    });
  } else {
    static_for<0, Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      g[i] = src.load(opposite(i), neighbour<i, -1>(c));
    });
  }
  const CellResult<T> res = kbc_collide(g, relax_of<T>(sp));
  if (res.bad) a.flags[sg.sample] = 1;

  if constexpr (KIND == kStep || KIND == kStepRecord) {
    if (!odd) {
      static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        src.store(opposite(i), c.cell, g[i]);
      });
    } else {
      static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        src.store(i, neighbour<i, +1>(c), g[i]);
      });
    }
  } else if constexpr (KIND == kPush) {
    const Planes dst(a.dst + sp.offset, sp.pstride);
    static_for<0, Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      dst.store(i, neighbour<i, +1>(c), g[i]);
    });
  }

  if constexpr (KIND == kStepRecord || KIND == kReduceOnly) {
    const Macro<T>& m = res.m;
    const double drho = double(m.drho);
    const double jx = double(m.jx), jy = double(m.jy), jz = double(m.jz);
    const double rho = 1.0 + drho;
    const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
    double v[kRecord] = {drho, jx, jy, jz, 0.5 * (ux * ux + uy * uy + uz * uz), double(res.gamma),
                         double(res.gamma), double(res.gamma)};
    block_record<BLOCK>(v, a.partials + size_t(b) * kRecord);
  }
}

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

template <typename T>
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
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const double cu = double(cx(i)) * u[0] + double(cy(i)) * u[1] + double(cz(i)) * u[2];
    const double gi = weight(i) * (3.0 * cu + 4.5 * cu * cu - usq15);
    st(base + size_t(i) * sp.pstride, cell, T(gi));
  });
}

// ---------------------------------------------------------------- read-out and state access
template <typename T>
__global__ void __launch_bounds__(256)
    moments_kernel(const T* pop, const DevSample* samples, int sample, int parity, double* rho, double* u) {
  const DevSample& sp = samples[sample];
  const int l = sp.log2n;
  const uint32_t ncell = 1u << (3 * l);
  const Cell c = make_cell(blockIdx.x * 256u + threadIdx.x, l);
  T g[Q];
  load_state(pop + sp.offset, sp.pstride, c, parity & 1, g);
  double d = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  static_for<0, Q>([&](auto ic) {
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

template <typename T>
__global__ void __launch_bounds__(256)
    get_state_kernel(const T* pop, const DevSample* samples, int sample, int parity, double* f) {
  const DevSample& sp = samples[sample];
  const int l = sp.log2n;
  const uint32_t ncell = 1u << (3 * l);
  const Cell c = make_cell(blockIdx.x * 256u + threadIdx.x, l);
  T g[Q];
  load_state(pop + sp.offset, sp.pstride, c, parity & 1, g);
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    f[size_t(i) * ncell + c.cell] = weight(i) + double(g[i]);
  });
}

template <typename T>
__global__ void __launch_bounds__(256)
    set_state_kernel(T* pop, const DevSample* samples, int sample, int parity, const double* f) {
  const DevSample& sp = samples[sample];
  const int l = sp.log2n;
  const uint32_t ncell = 1u << (3 * l);
  const Cell c = make_cell(blockIdx.x * 256u + threadIdx.x, l);
  T g[Q];
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    g[i] = T(f[size_t(i) * ncell + c.cell] - weight(i));
  });
  write_state(pop + sp.offset, sp.pstride, c, parity & 1, g);
}

// Populations (unshifted, double) of selected cells of one sample: f[k][27].
template <typename T>
__global__ void __launch_bounds__(64)
    gather_cells_kernel(const T* pop, const DevSample* samples, int sample, int parity, const int64_t* cells,
                        int count, double* f) {
  const int k = blockIdx.x * 64 + threadIdx.x;
  if (k >= count) return;
  const DevSample& sp = samples[sample];
  const int l = sp.log2n;
  const Cell c = make_cell(uint32_t(cells[k]), l);
  T g[Q];
  load_state(pop + sp.offset, sp.pstride, c, parity & 1, g);
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    f[size_t(k) * Q + i] = weight(i) + double(g[i]);
  });
}

template <typename T>
__global__ void poison_kernel(T* pop, const DevSample* samples, int sample, int parity, uint32_t cell, int i) {
  const DevSample& sp = samples[sample];
  const int l = sp.log2n;
  const Cell c = make_cell(cell, l);
  T* base = pop + sp.offset;
  const T nan = T(__builtin_nan(""));
  // slot of population i of this node (see load_state)
  if (!(parity & 1)) {
    base[size_t(i) * sp.pstride + cell] = nan;
  } else {
    const uint32_t nb = c.oz[1 - cz(i)] + c.oy[1 - cy(i)] + c.ox[1 - cx(i)];
    base[size_t(opposite(i)) * sp.pstride + nb] = nan;
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
    canonical_copy_kernel(const T* pop, T* dst, const DevSample* samples, const Seg* segs, int nseg) {
  const int b = blockIdx.x;
  const Seg sg = segs[find_segment(segs, nseg, b)];
  const DevSample& sp = samples[sg.sample];
  const int l = sp.log2n;
  const Cell c = make_cell(uint32_t(b - sg.first_block) * 256u + threadIdx.x, l);
  T g[Q];
  load_state(pop + sp.offset, sp.pstride, c, sg.parity & 1, g);
  write_state(dst + sp.offset, sp.pstride, c, false, g);
}

// ---------------------------------------------------------------- adjoint
// Seed: J = (1/M) sum_m KE_m with KE = (1/n^3) sum_x |u|^2 / 2, u = j / rho:
// dJ/dg_i(x) = (1 / (M n^3)) (c_i . u - |u|^2) / rho.
template <typename T>
__global__ void __launch_bounds__(256) adjoint_seed_kernel(const T* pop, T* lam, const DevSample* samples,
                                                           const Seg* segs, int nseg, double inv_m) {
  const int b = blockIdx.x;
  const Seg sg = segs[find_segment(segs, nseg, b)];
  const DevSample& sp = samples[sg.sample];
  const int l = sp.log2n;
  const uint32_t ncell = 1u << (3 * l);
  const Cell c = make_cell(uint32_t(b - sg.first_block) * 256u + threadIdx.x, l);
  T g[Q];
  load_state(pop + sp.offset, sp.pstride, c, sg.parity & 1, g);
  double d = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
  static_for<0, Q>([&](auto ic) {
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
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const double cu = double(cx(i)) * ux + double(cy(i)) * uy + double(cz(i)) * uz;
    st(lb + size_t(i) * sp.pstride, c.cell, T(coef * (cu - usq)));
  });
}

// One reverse step: lambda_n(x) = (d collide / d g_n(x))^T [lambda_{n+1, i}(x + c_i)]_i,
// the transpose of "collide at x, then move population i to x + c_i".
template <typename T, bool BUF>
__global__ void __launch_bounds__(256) adjoint_step_kernel(const T* state, const T* lam_in, T* lam_out,
                                                           const DevSample* samples, const Seg* segs, int nseg) {
  const int b = blockIdx.x;
  const Seg sg = segs[find_segment(segs, nseg, b)];
  const DevSample& sp = samples[sg.sample];
  const int l = sp.log2n;
  const Cell c = make_cell(uint32_t(b - sg.first_block) * 256u + threadIdx.x, l);
  const Relax<T> rp = relax_of<T>(sp);
  // every array is streamed once per reverse step: non-temporal accesses
  using Planes = typename std::conditional<BUF, BufPlanes<T, true>, PtrPlanes<T, true>>::type;
  const Planes st_in(const_cast<T*>(state) + sp.offset, sp.pstride);
  const Planes lam_src(const_cast<T*>(lam_in) + sp.offset, sp.pstride);
  const Planes lam_dst(lam_out + sp.offset, sp.pstride);

  T g[Q], nu[Q];
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    g[i] = st_in.load(i, c.cell);
    nu[i] = lam_src.load(i, neighbour<i, +1>(c));
  });

  // forward intermediates, as in kbc_collide
  const Macro<T> m = macroscopic(g);
  T fneq[Q];
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    fneq[i] = g[i] - geq<i>(m);
  });
  const Shear<T> s = shear_coefficients(fneq);
  T A = T(0), B = T(0);
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const T r = recip(T(weight(i)) + geq<i>(m));
    if constexpr (nonzeros(i) == 1 || nonzeros(i) == 2) {
      const T ds = shear_part<i>(s);
      const T dh = fneq[i] - ds;
      A += ds * dh * r;
      B += dh * dh * r;
    } else {
      B += fneq[i] * fneq[i] * r;
    }
  });
  const bool active = B > T(1e-30);
  T gamma = T(2);
  if (active) gamma = rp.two_over_omega - rp.kappa * (A / B);
  const T t = T(0.5) * rp.omega * gamma;

  // reverse sweep. ga: adjoint of g (direct path g* = g - ...)
  T tbar = T(0);
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr (nonzeros(i) == 1 || nonzeros(i) == 2) tbar -= nu[i] * (fneq[i] - shear_part<i>(s));
    else tbar -= nu[i] * fneq[i];
  });
  T Abar = T(0), Bbar = T(0);
  if (active) {
    const T gbar = T(0.5) * rp.omega * tbar;
    Abar = -rp.kappa * gbar / B;
    Bbar = rp.kappa * gbar * (A / B) / B;  // B * B would underflow in float
  }
  // adjoints of fneq (through dh and the weights) and of the shear coefficients
  T fbar[Q], geqbar[Q];
  T dsxb = T(0), dsyb = T(0), dszb = T(0), exyb = T(0), exzb = T(0), eyzb = T(0);
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const T r = recip(T(weight(i)) + geq<i>(m));
    T dsb, dhb, rbar;
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
  static_for<0, Q>([&](auto ic) {
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
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const T si = T(weight(i)) * geqbar[i];
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
  static_for<0, Q>([&](auto ic) {
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
template <typename T>
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
  static_for<0, Q>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    const double li = double(ld(lb + size_t(i) * sp.pstride, cell)) * weight(i);
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

// One 16-byte element per thread (the fastest plain copy measured on gfx950).
__global__ void __launch_bounds__(256) stream_copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                          size_t n4) {
  const size_t i = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (i < n4) dst[i] = src[i];
}

template <typename T, int BLOCK, StepKind KIND>
hipError_t launch_step_t(const StepLaunch& L, hipStream_t s) {
  const bool buf = L.buffer_ok;
  StepArgs<T> a;
  a.pop = static_cast<T*>(L.pop);
  a.dst = static_cast<T*>(L.dst);
  a.samples = L.samples;
  a.segs = L.segs;
  a.nseg = L.nseg;
  a.total_blocks = L.total_blocks;
  a.xcd_remap = L.xcd_remap;
  a.flags = L.flags;
  a.partials = L.partials;
  const dim3 grid(L.total_blocks), blk(BLOCK);
  if (buf && L.nontemporal)
    hipLaunchKernelGGL((kbc_step_kernel<T, BLOCK, KIND, true, true>), grid, blk, 0, s, a);
  else if (buf)
    hipLaunchKernelGGL((kbc_step_kernel<T, BLOCK, KIND, true, false>), grid, blk, 0, s, a);
  else if (L.nontemporal)
    hipLaunchKernelGGL((kbc_step_kernel<T, BLOCK, KIND, false, true>), grid, blk, 0, s, a);
  else
    hipLaunchKernelGGL((kbc_step_kernel<T, BLOCK, KIND, false, false>), grid, blk, 0, s, a);
  return hipGetLastError();
}

template <typename T, StepKind KIND>
hipError_t launch_step_b(const StepLaunch& L, hipStream_t s) {
  switch (L.block) {
    case 128: return launch_step_t<T, 128, KIND>(L, s);
    case 256: return launch_step_t<T, 256, KIND>(L, s);
    case 512: return launch_step_t<T, 512, KIND>(L, s);
    case 1024:
      if constexpr (std::is_same<T, float>::value) return launch_step_t<T, 1024, KIND>(L, s);
      else return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_step_k(StepKind kind, const StepLaunch& L, hipStream_t s) {
  switch (kind) {
    case kStep: return launch_step_b<T, kStep>(L, s);
    case kStepRecord: return launch_step_b<T, kStepRecord>(L, s);
    case kReduceOnly: return launch_step_b<T, kReduceOnly>(L, s);
    case kPush: return launch_step_b<T, kPush>(L, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_step(int precision, StepKind kind, const StepLaunch& L, hipStream_t s) {
  return precision == 0 ? launch_step_k<double>(kind, L, s) : launch_step_k<float>(kind, L, s);
}

hipError_t launch_record_finalize(const double* partials, const Seg* segs, int32_t nseg, const DevSample* samples,
                                  double* out, hipStream_t s) {
  hipLaunchKernelGGL(record_finalize_kernel, dim3(nseg), dim3(256), 0, s, partials, segs, samples, out);
  return hipGetLastError();
}

hipError_t launch_init(int precision, void* pop, const DevSample* samples, const Seg* segs, int32_t nseg,
                       int32_t total_blocks, const double* ycoef, hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(init_kernel<double>, dim3(total_blocks), dim3(256), 0, s, static_cast<double*>(pop), samples,
                       segs, nseg, ycoef);
  else
    hipLaunchKernelGGL(init_kernel<float>, dim3(total_blocks), dim3(256), 0, s, static_cast<float*>(pop), samples,
                       segs, nseg, ycoef);
  return hipGetLastError();
}

hipError_t launch_moments(int precision, const void* pop, const DevSample* samples, int32_t sample, int32_t n,
                          int32_t parity, double* rho, double* u, hipStream_t s) {
  const unsigned blocks = unsigned((uint64_t(n) * n * n) / 256);
  if (precision == 0)
    hipLaunchKernelGGL(moments_kernel<double>, dim3(blocks), dim3(256), 0, s, static_cast<const double*>(pop), samples,
                       sample, parity, rho, u);
  else
    hipLaunchKernelGGL(moments_kernel<float>, dim3(blocks), dim3(256), 0, s, static_cast<const float*>(pop), samples,
                       sample, parity, rho, u);
  return hipGetLastError();
}

hipError_t launch_get_state(int precision, const void* pop, const DevSample* samples, int32_t sample, int32_t n,
                            int32_t parity, double* f, hipStream_t s) {
  const unsigned blocks = unsigned((uint64_t(n) * n * n) / 256);
  if (precision == 0)
    hipLaunchKernelGGL(get_state_kernel<double>, dim3(blocks), dim3(256), 0, s, static_cast<const double*>(pop),
                       samples, sample, parity, f);
  else
    hipLaunchKernelGGL(get_state_kernel<float>, dim3(blocks), dim3(256), 0, s, static_cast<const float*>(pop),
                       samples, sample, parity, f);
  return hipGetLastError();
}

hipError_t launch_set_state(int precision, void* pop, const DevSample* samples, int32_t sample, int32_t n,
                            int32_t parity, const double* f, hipStream_t s) {
  const unsigned blocks = unsigned((uint64_t(n) * n * n) / 256);
  if (precision == 0)
    hipLaunchKernelGGL(set_state_kernel<double>, dim3(blocks), dim3(256), 0, s, static_cast<double*>(pop), samples,
                       sample, parity, f);
  else
    hipLaunchKernelGGL(set_state_kernel<float>, dim3(blocks), dim3(256), 0, s, static_cast<float*>(pop), samples,
                       sample, parity, f);
  return hipGetLastError();
}

hipError_t launch_gather_cells(int precision, const void* pop, const DevSample* samples, int32_t sample, int32_t parity,
                               const int64_t* cells, int32_t count, double* f, hipStream_t s) {
  const unsigned blocks = unsigned((count + 63) / 64);
  if (precision == 0)
    hipLaunchKernelGGL(gather_cells_kernel<double>, dim3(blocks), dim3(64), 0, s, static_cast<const double*>(pop),
                       samples, sample, parity, cells, count, f);
  else
    hipLaunchKernelGGL(gather_cells_kernel<float>, dim3(blocks), dim3(64), 0, s, static_cast<const float*>(pop),
                       samples, sample, parity, cells, count, f);
  return hipGetLastError();
}

hipError_t launch_poison(int precision, void* pop, const DevSample* samples, int32_t sample, int32_t parity,
                         int64_t cell, int32_t i, hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(poison_kernel<double>, dim3(1), dim3(1), 0, s, static_cast<double*>(pop), samples, sample,
                       parity, uint32_t(cell), i);
  else
    hipLaunchKernelGGL(poison_kernel<float>, dim3(1), dim3(1), 0, s, static_cast<float*>(pop), samples, sample, parity,
                       uint32_t(cell), i);
  return hipGetLastError();
}

hipError_t launch_canonical_copy(int precision, const void* pop, void* dst, const DevSample* samples, const Seg* segs,
                                 int32_t nseg, int32_t total_blocks, hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(canonical_copy_kernel<double>, dim3(total_blocks), dim3(256), 0, s,
                       static_cast<const double*>(pop), static_cast<double*>(dst), samples, segs, nseg);
  else
    hipLaunchKernelGGL(canonical_copy_kernel<float>, dim3(total_blocks), dim3(256), 0, s,
                       static_cast<const float*>(pop), static_cast<float*>(dst), samples, segs, nseg);
  return hipGetLastError();
}

hipError_t launch_adjoint_seed(int precision, const void* pop, void* lam, const DevSample* samples, const Seg* segs,
                               int32_t nseg, int32_t total_blocks, double inv_m, hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(adjoint_seed_kernel<double>, dim3(total_blocks), dim3(256), 0, s,
                       static_cast<const double*>(pop), static_cast<double*>(lam), samples, segs, nseg, inv_m);
  else
    hipLaunchKernelGGL(adjoint_seed_kernel<float>, dim3(total_blocks), dim3(256), 0, s,
                       static_cast<const float*>(pop), static_cast<float*>(lam), samples, segs, nseg, inv_m);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_step_t(const void* state, const void* lam_in, void* lam_out, const DevSample* samples,
                                 const Seg* segs, int32_t nseg, int32_t total_blocks, int32_t buffer_ok,
                                 hipStream_t s) {
  const T* a = static_cast<const T*>(state);
  const T* b = static_cast<const T*>(lam_in);
  T* o = static_cast<T*>(lam_out);
  if (buffer_ok)
    hipLaunchKernelGGL((adjoint_step_kernel<T, true>), dim3(total_blocks), dim3(256), 0, s, a, b, o, samples, segs,
                       nseg);
  else
    hipLaunchKernelGGL((adjoint_step_kernel<T, false>), dim3(total_blocks), dim3(256), 0, s, a, b, o, samples, segs,
                       nseg);
  return hipGetLastError();
}

hipError_t launch_adjoint_step(int precision, const void* state, const void* lam_in, void* lam_out,
                               const DevSample* samples, const Seg* segs, int32_t nseg, int32_t total_blocks,
                               int32_t buffer_ok, hipStream_t s) {
  if (precision == 0)
    return launch_adjoint_step_t<double>(state, lam_in, lam_out, samples, segs, nseg, total_blocks, buffer_ok, s);
  return launch_adjoint_step_t<float>(state, lam_in, lam_out, samples, segs, nseg, total_blocks, buffer_ok, s);
}

hipError_t launch_init_adjoint(int precision, const void* lam, const DevSample* samples, const Seg* segs,
                               int32_t nseg, int32_t total_blocks, const double* ycoef, double* partials,
                               hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(init_adjoint_kernel<double>, dim3(total_blocks), dim3(256), 0, s,
                       static_cast<const double*>(lam), samples, segs, nseg, ycoef, partials);
  else
    hipLaunchKernelGGL(init_adjoint_kernel<float>, dim3(total_blocks), dim3(256), 0, s,
                       static_cast<const float*>(lam), samples, segs, nseg, ycoef, partials);
  return hipGetLastError();
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

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const size_t n4 = bytes / 16;
  const size_t blocks = (n4 + 255) / 256;
  if (blocks == 0) return hipSuccess;
  if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(stream_copy_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<const float4*>(src),
                     static_cast<float4*>(dst), n4);
  return hipGetLastError();
}

}  // namespace mclbm
