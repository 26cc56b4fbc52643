// FP64 observables of one sample's velocity field (gfx950):
//   * 3-D discrete Fourier transform by radix-2 transforms along each axis,
//     a block of 256 threads transforming LINES lines at once in LDS;
//   * the power spectral density Psi(k) = sum_a |F(u_a)(k)|^2;
//   * the shell energy spectrum E(kappa) = 4 pi / |S_kappa| sum_{S_kappa}
//     |k|^2 / 2 * Psi(k) / N^6 (eqs. (dftCoeff), (energySpecDisc));
//   * the autocorrelation R_h = N^-6 F^-1(Psi)_h with an unnormalised inverse
//     and the structure function S2(r) = 1/|C_r| sum_{h in C_r} 2 (R_0 - R_h)
//     (Lemma (structureFunctionSpectral), eq. (SF_single_spec2));
//   * point values of all samples at the q^3 nodes common to every
//     resolution, and the 1-point Wasserstein distance between two such
//     ensembles by sorting (Algorithm 2, eq. (wassersteinPermutations)).
// Shells hold the integer vectors (minimum image, components in
// {-N/2+1, ..., N/2}) whose length rounds to the shell index; blocks
// enumerate the (z, y) rows of a shell and the one or two x-intervals of each
// row, so every sum runs in a fixed order (results do not depend on
// scheduling).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "lattice.h"

namespace mclbm {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int N>
constexpr int log2_of() {
  int l = 0;
  while ((1 << l) < N) ++l;
  return l;
}

// Address of element i of line `line` along `axis` in an N^3 array ([z][y][x]).
template <int N>
__device__ __forceinline__ size_t line_offset(int axis, int line, int i) {
  if (axis == 0) return size_t(line) * N + i;                                    // x: line = z*N + y
  if (axis == 1) return size_t(line / N) * N * N + size_t(i) * N + (line % N);   // y: line = z*N + x
  return size_t(i) * N * N + line;                                               // z: line = y*N + x
}

// Radix-2 decimation-in-time transform of LINES lines along `axis`, in place.
// sign = -1: forward e^{-2 pi i k n / N}; +1: unnormalised inverse.
// real_in: the input is real (double array `rin` of N^3), written as complex.
template <int N, int LINES>
__global__ void __launch_bounds__(256)
    fft_axis_kernel(double2* data, const double* rin, int axis, int sign, size_t comp_stride_c, size_t comp_stride_r) {
  constexpr int LOG = log2_of<N>();
  __shared__ double2 sh[LINES][N];
  __shared__ double2 tw[N / 2 > 0 ? N / 2 : 1];
  double2* d = data + size_t(blockIdx.y) * comp_stride_c;
  const double* r = rin ? rin + size_t(blockIdx.y) * comp_stride_r : nullptr;
  for (int k = threadIdx.x; k < N / 2; k += 256) {
    double s, c;
    sincospi(2.0 * k / N, &s, &c);
    tw[k] = make_double2(c, sign * s);
  }
  const int line0 = blockIdx.x * LINES;
  for (int e = threadIdx.x; e < LINES * N; e += 256) {
    int l, i;
    if (axis == 0) {
      l = e / N;
      i = e % N;
    } else {
      i = e / LINES;
      l = e % LINES;
    }
    const size_t off = line_offset<N>(axis, line0 + l, i);
    const double2 v = r ? make_double2(r[off], 0.0) : d[off];
    const int rev = int(__brev(unsigned(i)) >> (32 - LOG));
    sh[l][rev] = v;
  }
  __syncthreads();
  for (int half = 1; half < N; half <<= 1) {
    const int stride = N / (2 * half);
    for (int b = threadIdx.x; b < LINES * (N / 2); b += 256) {
      const int l = b / (N / 2), j = b % (N / 2);
      const int pos = j % half, grp = j / half;
      const int i0 = grp * 2 * half + pos, i1 = i0 + half;
      const double2 a = sh[l][i0];
      const double2 t = cmul(tw[pos * stride], sh[l][i1]);
      sh[l][i0] = make_double2(a.x + t.x, a.y + t.y);
      sh[l][i1] = make_double2(a.x - t.x, a.y - t.y);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < LINES * N; e += 256) {
    int l, i;
    if (axis == 0) {
      l = e / N;
      i = e % N;
    } else {
      i = e / LINES;
      l = e % LINES;
    }
    d[line_offset<N>(axis, line0 + l, i)] = sh[l][i];
  }
}

// Psi(k) = sum over 3 components of |X(k)|^2, written as (Psi, 0) into out.
__global__ void __launch_bounds__(256) psd_kernel(const double2* x, size_t n3, double2* out) {
  const size_t k = size_t(blockIdx.x) * 256 + threadIdx.x;
  if (k >= n3) return;
  const double2 a = x[k], b = x[n3 + k], c = x[2 * n3 + k];
  out[k] = make_double2(a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y + c.x * c.x + c.y * c.y, 0.0);
}

__device__ __forceinline__ int64_t isqrt_floor(int64_t v) {
  if (v <= 0) return 0;
  int64_t r = int64_t(sqrt(double(v)));
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// Shell sums over the real parts of data (N^3, minimum-image index vectors),
// in two passes.
// Pass 1 (one wave per (z, y) row, s = hz^2 + hy^2): the row is folded by
// |hx| = m into LDS, v[m] = value(+m) + value(-m) (one term at m = 0 and
// m = N/2), then lane r sums v over the m-interval whose |h| rounds to r and
// writes rowbins[r][row] (and the number of lags, rowcnt[r][row]).
// Pass 2 (one block per shell): sums its rowbins column in a fixed order.
// mode 0 (spectrum): value = |k|^2/2 * v; mode 1 (structure function):
// value = 2 (v(0) - v(h)).
__global__ void __launch_bounds__(256) shell_rows_kernel(const double2* data, int n, int mode, double* rowbins,
                                                         double* rowcnt) {
  __shared__ double sh[4][513];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rows = n * n;
  const int row = blockIdx.x * 4 + wave;
  const int half = n / 2;
  if (row < rows) {
    const int iz = row / n, iy = row % n;
    const int hz = iz <= half ? iz : iz - n, hy = iy <= half ? iy : iy - n;
    const int64_t s = int64_t(hz) * hz + int64_t(hy) * hy;
    const size_t base = size_t(row) * n;
    const double v0 = data[0].x;
    for (int m = lane; m <= half; m += 64) {
      const double k2 = double(s) + double(m) * m;
      const double a = data[base + m].x;
      double v = mode == 0 ? 0.5 * k2 * a : 2.0 * (v0 - a);
      if (m >= 1 && m <= half - 1) {
        const double b = data[base + (n - m)].x;
        v += mode == 0 ? 0.5 * k2 * b : 2.0 * (v0 - b);
      }
      sh[wave][m] = v;
    }
  }
  __syncthreads();
  if (row < rows) {
    const int iz = row / n, iy = row % n;
    const int hz = iz <= half ? iz : iz - n, hy = iy <= half ? iy : iy - n;
    const int64_t s = int64_t(hz) * hz + int64_t(hy) * hy;
    for (int r = lane; r <= half; r += 64) {
      // m^2 in [ceil(((2r-1)^2 - 4s)/4), floor(((2r+1)^2 - 1 - 4s)/4)], m in [0, N/2]
      double sum = 0.0, cnt = 0.0;
      const int64_t lo2 = r == 0 ? 0 : int64_t(2 * r - 1) * (2 * r - 1);
      const int64_t top = int64_t(2 * r + 1) * (2 * r + 1) - 1 - 4 * s;
      if (top >= 0) {
        const int64_t m2max = top / 4;
        const int64_t bot = lo2 - 4 * s;
        const int64_t m2min = bot <= 0 ? 0 : (bot + 3) / 4;
        if (m2min <= m2max) {
          int64_t a = isqrt_floor(m2min);
          if (a * a < m2min) ++a;
          int64_t b = isqrt_floor(m2max);
          if (b > half) b = half;
          for (int64_t m = a; m <= b; ++m) {
            sum += sh[wave][m];
            cnt += (m == 0 || m == half) ? 1.0 : 2.0;
          }
        }
      }
      rowbins[size_t(r) * rows + row] = sum;
      rowcnt[size_t(r) * rows + row] = cnt;
    }
  }
}

__global__ void __launch_bounds__(256) shell_sum_kernel(const double* rowbins, const double* rowcnt, int n, int mode,
                                                        double* out) {
  const int rows = n * n;
  const int r = mode == 0 ? int(blockIdx.x) : int(blockIdx.x) + 1;
  __shared__ double sa[256], sc[256];
  double acc = 0.0, cnt = 0.0;
  for (int k = threadIdx.x; k < rows; k += 256) {
    acc += rowbins[size_t(r) * rows + k];
    cnt += rowcnt[size_t(r) * rows + k];
  }
  sa[threadIdx.x] = acc;
  sc[threadIdx.x] = cnt;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      sa[threadIdx.x] += sa[threadIdx.x + st];
      sc[threadIdx.x] += sc[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double norm = 1.0 / (double(n) * n * n) / (double(n) * n * n);
    const double sum = sa[0] * norm, c = sc[0];
    if (mode == 0) out[blockIdx.x] = c > 0 ? 4.0 * M_PI / c * sum : 0.0;
    else out[blockIdx.x] = c > 0 ? sum / c : 0.0;
  }
}

// Velocity of every sample at the q^3 nodes x = (n/q) * j: out[s][3][q^3].
template <int QN, typename T>
__global__ void __launch_bounds__(64) point_values_kernel(const T* pop, const DevSample* samples, const Seg* segs,
                                                          int q, double* out) {
  const Seg sg = segs[blockIdx.y];
  const DevSample& sp = samples[sg.sample];
  const int l = sp.log2n;
  const int n = 1 << l;
  const int q3 = q * q * q;
  const int j = blockIdx.x * 64 + threadIdx.x;
  if (j >= q3) return;
  const int step = n / q;
  const int jx = j % q, jy = (j / q) % q, jz = j / (q * q);
  const uint32_t msk = uint32_t(n - 1);
  const uint32_t x = uint32_t(jx * step), y = uint32_t(jy * step), z = uint32_t(jz * step);
  const T* base = pop + sp.offset;
  const bool odd = sg.parity & 1;
  double d = 0.0, jxs = 0.0, jys = 0.0, jzs = 0.0;
  for (int i = 0; i < Q; ++i) {
    if (!in_lattice<QN>(i)) continue;
    size_t idx;
    int slot;
    if (!odd) {
      idx = (size_t(z) << (2 * l)) + (size_t(y) << l) + x;
      slot = plane_of<QN>(i);
    } else {
      const uint32_t xs = (x - uint32_t(cx(i))) & msk, ys = (y - uint32_t(cy(i))) & msk,
                     zs = (z - uint32_t(cz(i))) & msk;
      idx = (size_t(zs) << (2 * l)) + (size_t(ys) << l) + xs;
      slot = plane_of<QN>(opposite(i));
    }
    const double v = double(base[size_t(slot) * sp.pstride + idx]);
    d += v;
    jxs += cx(i) * v;
    jys += cy(i) * v;
    jzs += cz(i) * v;
  }
  const double rho = 1.0 + d;
  double* o = out + size_t(sg.sample) * 3 * q3;
  o[j] = jxs / rho;
  o[q3 + j] = jys / rho;
  o[2 * q3 + j] = jzs / rho;
}

// One block per (component, node): sort the m values of both ensembles and
// average |a_(i) - b_(i)| (bitonic sort in LDS, m <= 4096).
__global__ void __launch_bounds__(256) w1_column_kernel(const double* a, const double* b, int m, int q3, int p2,
                                                        double* col) {
  __shared__ double sa[4096], sb[4096];
  const int c = blockIdx.x;  // column = comp * q3 + node
  for (int i = threadIdx.x; i < p2; i += 256) {
    sa[i] = i < m ? a[size_t(i) * 3 * q3 + c] : 1.0e308;
    sb[i] = i < m ? b[size_t(i) * 3 * q3 + c] : 1.0e308;
  }
  __syncthreads();
  for (int k = 2; k <= p2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < p2; i += 256) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const bool up = (i & k) == 0;
          double x = sa[i], y = sa[ixj];
          if ((x > y) == up) {
            sa[i] = y;
            sa[ixj] = x;
          }
          x = sb[i];
          y = sb[ixj];
          if ((x > y) == up) {
            sb[i] = y;
            sb[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) acc += fabs(sa[i] - sb[i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) col[c] = red[0] / m;
}

// out[c] = (1/q^3) sum over nodes of the column distances of component c.
__global__ void __launch_bounds__(256) w1_reduce_kernel(const double* col, int q3, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < q3; i += 256) acc += col[size_t(blockIdx.x) * q3 + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0] / q3;
}

template <int N>
hipError_t fft3_t(double2* data, const double* rin, int ncomp, int sign, hipStream_t s) {
  constexpr int LINES = N >= 512 ? 4 : (N >= 256 ? 8 : 16);
  const unsigned blocks = unsigned((N * N) / LINES);
  const size_t n3 = size_t(N) * N * N;
  for (int axis = 0; axis < 3; ++axis) {
    hipLaunchKernelGGL((fft_axis_kernel<N, LINES>), dim3(blocks, ncomp), dim3(256), 0, s, data,
                       axis == 0 ? rin : nullptr, axis, sign, n3, n3);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_fft3(int n, double2* data, const double* rin, int ncomp, int sign, hipStream_t s) {
  switch (n) {
    case 8: return fft3_t<8>(data, rin, ncomp, sign, s);
    case 16: return fft3_t<16>(data, rin, ncomp, sign, s);
    case 32: return fft3_t<32>(data, rin, ncomp, sign, s);
    case 64: return fft3_t<64>(data, rin, ncomp, sign, s);
    case 128: return fft3_t<128>(data, rin, ncomp, sign, s);
    case 256: return fft3_t<256>(data, rin, ncomp, sign, s);
    case 512: return fft3_t<512>(data, rin, ncomp, sign, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_psd(const double2* x, size_t n3, double2* out, hipStream_t s) {
  hipLaunchKernelGGL(psd_kernel, dim3(unsigned((n3 + 255) / 256)), dim3(256), 0, s, x, n3, out);
  return hipGetLastError();
}

size_t shell_scratch_doubles(int n) { return size_t(2) * (n / 2 + 1) * size_t(n) * n; }

hipError_t launch_shells(const double2* data, int n, int mode, double* scratch, double* out, hipStream_t s) {
  const size_t table = size_t(n / 2 + 1) * size_t(n) * n;
  double* rowbins = scratch;
  double* rowcnt = scratch + table;
  hipLaunchKernelGGL(shell_rows_kernel, dim3(unsigned((n * n + 3) / 4)), dim3(256), 0, s, data, n, mode, rowbins,
                     rowcnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned bins = mode == 0 ? unsigned(n / 2 + 1) : unsigned(n / 2);
  hipLaunchKernelGGL(shell_sum_kernel, dim3(bins), dim3(256), 0, s, rowbins, rowcnt, n, mode, out);
  return hipGetLastError();
}

hipError_t launch_point_values(int lattice, int precision, const void* pop, const DevSample* samples,
                               const Seg* segs, int32_t nseg, int q, double* out, hipStream_t s) {
  const dim3 grid(unsigned((q * q * q + 63) / 64), unsigned(nseg));
  if (lattice == 27 && precision == 0)
    hipLaunchKernelGGL((point_values_kernel<27, double>), grid, dim3(64), 0, s, static_cast<const double*>(pop),
                       samples, segs, q, out);
  else if (lattice == 27)
    hipLaunchKernelGGL((point_values_kernel<27, float>), grid, dim3(64), 0, s, static_cast<const float*>(pop),
                       samples, segs, q, out);
  else if (lattice == 19 && precision == 0)
    hipLaunchKernelGGL((point_values_kernel<19, double>), grid, dim3(64), 0, s, static_cast<const double*>(pop),
                       samples, segs, q, out);
  else if (lattice == 19)
    hipLaunchKernelGGL((point_values_kernel<19, float>), grid, dim3(64), 0, s, static_cast<const float*>(pop),
                       samples, segs, q, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_w1(const double* a, const double* b, int m, int q, double* col, double* out, hipStream_t s) {
  const int q3 = q * q * q;
  int p2 = 1;
  while (p2 < m) p2 <<= 1;
  hipLaunchKernelGGL(w1_column_kernel, dim3(unsigned(3 * q3)), dim3(256), 0, s, a, b, m, q3, p2, col);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(w1_reduce_kernel, dim3(3), dim3(256), 0, s, col, q3, out);
  return hipGetLastError();
}

}  // namespace mclbm
