// FP64 observables of one sample's velocity field (gfx950):
//   * the power spectral density Psi(k) = sum_a |F(u_a)(k)|^2 of the
//     three velocity components (unnormalised forward transform);
//   * the shell energy spectrum E(kappa) = 4 pi / |S_kappa| sum_{S_kappa}
//     |k|^2 / 2 * Psi(k) / N^6 (eqs. (dftCoeff), (energySpecDisc));
//   * the autocorrelation R_h = N^-6 F^-1(Psi)_h with an unnormalised inverse
//     and the structure function S2(r) = 1/|C_r| sum_{h in C_r} 2 (R_0 - R_h)
//     (Lemma (structureFunctionSpectral), eq. (SF_single_spec2));
//   * point values of all samples at the q^3 nodes common to every
//     resolution, and the 1-point Wasserstein distance between two such
//     ensembles by sorting (Algorithm 2, eq. (wassersteinPermutations)).
//
// The velocity is real, so its transform is stored for kx = 0..N/2 only
// (the rest follows by conjugate symmetry), fields [z][y][kx], and the
// pipeline is five passes over HBM:
//   1. x: velocities from the populations (either AA parity) and the
//      forward transform along x of the three components, per row in LDS;
//   2. y, 3. z: forward transforms along y and z of the three fields;
//   4. per z-line: Psi, its shell sums for the spectrum, its total (R_0),
//      and the inverse transform along z of Psi, written over field 0;
//   5. inverse along y; 6. per x-row: the inverse along x (conjugate-
//      symmetric fill, real result R_h) and its shell sums for S2.
// Radix-2 decimation-in-time transforms of whole lines in LDS, twiddles by
// sincospi. Shells hold the integer vectors (minimum image, components in
// {-N/2+1, ..., N/2}) whose length rounds to the shell index. Every shell sum
// is taken per line in a fixed order (the line folded by the magnitude of
// its own coordinate, the lengths of a shell forming an interval of it), and
// then over lines in a fixed order: results do not depend on scheduling.
// A half-spectrum mode 0 < kx < N/2 stands for itself and its conjugate
// partner at -k, which has the same length: weight 2.
#include <hip/hip_runtime.h>

#include "lbm_device.h"

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

template <int N>
__device__ __forceinline__ int bitrev(int i) {
  return int(__brev(unsigned(i)) >> (32 - log2_of<N>()));
}

// e^{sign 2 pi i k / N}, k < N/2
template <int N>
__device__ __forceinline__ void make_twiddles(double2* tw, int sign) {
  for (int k = threadIdx.x; k < N / 2; k += blockDim.x) {
    double s, c;
    sincospi(2.0 * k / N, &s, &c);
    tw[k] = make_double2(c, sign * s);
  }
}

// In-place butterflies of nl lines of length N (line l at sh + l N) loaded in
// bit-reversed order (decimation in time); every thread of the block takes
// part and the caller synchronises after loading. Two consecutive radix-2
// stages (spans h and 2h) run as one radix-4 step in registers: a thread
// takes the four values i0 + {0, 1, 2, 3} h, applies the span-h pairs (one
// twiddle) and then the span-2h pairs (two twiddles), so LDS is read and
// written once per two stages. An odd number of stages starts with one
// radix-2 stage.
template <int N>
__device__ __forceinline__ void butterflies(double2* sh, int nl, const double2* tw) {
  constexpr int LOG = log2_of<N>();
  int half = 1;
  if (LOG & 1) {
    for (int b = threadIdx.x; b < nl * (N / 2); b += blockDim.x) {
      const int l = b / (N / 2), j = b % (N / 2);
      double2* ln = sh + l * N + 2 * j;
      const double2 a = ln[0], c = ln[1];
      ln[0] = make_double2(a.x + c.x, a.y + c.y);
      ln[1] = make_double2(a.x - c.x, a.y - c.y);
    }
    __syncthreads();
    half = 2;
  }
  for (; half < N; half <<= 2) {
    const int sa = N / (2 * half), sb = N / (4 * half);  // twiddle strides of the two stages
    for (int b = threadIdx.x; b < nl * (N / 4); b += blockDim.x) {
      const int l = b / (N / 4), j = b % (N / 4);
      const int pos = j % half, grp = j / half;
      double2* ln = sh + l * N + grp * 4 * half + pos;
      const double2 x0 = ln[0], x1 = ln[half], x2 = ln[2 * half], x3 = ln[3 * half];
      // span h: (x0, x1) and (x2, x3), twiddle tw[pos * sa]
      const double2 wa = tw[pos * sa];
      const double2 t1 = cmul(wa, x1), t3 = cmul(wa, x3);
      const double2 y0 = make_double2(x0.x + t1.x, x0.y + t1.y), y1 = make_double2(x0.x - t1.x, x0.y - t1.y);
      const double2 y2 = make_double2(x2.x + t3.x, x2.y + t3.y), y3 = make_double2(x2.x - t3.x, x2.y - t3.y);
      // span 2h: (y0, y2) with tw[pos * sb], (y1, y3) with tw[(pos + h) * sb]
      const double2 u2 = cmul(tw[pos * sb], y2), u3 = cmul(tw[(pos + half) * sb], y3);
      ln[0] = make_double2(y0.x + u2.x, y0.y + u2.y);
      ln[2 * half] = make_double2(y0.x - u2.x, y0.y - u2.y);
      ln[half] = make_double2(y1.x + u3.x, y1.y + u3.y);
      ln[3 * half] = make_double2(y1.x - u3.x, y1.y - u3.y);
    }
    __syncthreads();
  }
}

// A batch of samples shares one launch: blockIdx.z is the sample's place in
// the batch, and its work area starts wstride bytes after the previous one.
template <typename P>
__device__ __forceinline__ P* in_batch(P* p, size_t wstride) {
  using B = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<B*>(p) + size_t(blockIdx.z) * wstride);
}

__device__ __forceinline__ int64_t isqrt_floor(int64_t v) {
  if (v <= 0) return 0;
  int64_t r = int64_t(sqrt(double(v)));
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// Sum of v[m] over the m in [0, half] with round(sqrt(s + m^2)) == r, and the
// number of lattice vectors they stand for (m and -m: 2, except m = 0 and
// m = half): m^2 in [ceil(((2r-1)^2 - 4s)/4), floor(((2r+1)^2 - 1 - 4s)/4)].
__device__ __forceinline__ void shell_interval(const double* v, int half, int64_t s, int r, double& sum,
                                               double& cnt) {
  sum = 0.0;
  cnt = 0.0;
  const int64_t lo2 = r == 0 ? 0 : int64_t(2 * r - 1) * (2 * r - 1);
  const int64_t top = int64_t(2 * r + 1) * (2 * r + 1) - 1 - 4 * s;
  if (top < 0) return;
  const int64_t m2max = top / 4;
  const int64_t bot = lo2 - 4 * s;
  const int64_t m2min = bot <= 0 ? 0 : (bot + 3) / 4;
  if (m2min > m2max) return;
  int64_t a = isqrt_floor(m2min);
  if (a * a < m2min) ++a;
  int64_t b = isqrt_floor(m2max);
  if (b > half) b = half;
  for (int64_t m = a; m <= b; ++m) {
    sum += v[m];
    cnt += (m == 0 || m == half) ? 1.0 : 2.0;
  }
}

// Pass 1: ROWS rows (z, y) per block. Velocities of the row's nodes from
// the populations (the parity selects the AA slots), forward transform
// along x of the three components, kx = 0..N/2 written to
// h[c][(z N + y) NH + kx].
template <int QN, typename T, int N>
__global__ void __launch_bounds__(256)
    fwd_x_kernel(const T* pop, const DevSample* samples, int sample0, int parity, double2* h0, size_t wstride) {
  constexpr int ROWS = N >= 512 ? 1 : 512 / N;
  constexpr int NH = N / 2 + 1;
  __shared__ double2 sh[3 * ROWS * N];
  __shared__ double2 tw[N / 2];
  const DevSample& sp = samples[sample0 + blockIdx.z];
  double2* h = in_batch(h0, wstride);
  const size_t row0 = size_t(blockIdx.x) * ROWS;
  make_twiddles<N>(tw, -1);
  const T* base = pop + sp.offset;
  for (int e = threadIdx.x; e < ROWS * N; e += 256) {
    const int r = e / N, x = e % N;
    const Cell c = make_cell(uint32_t((row0 + r) * N + x), sp.log2n);
    T g[Q];
    load_state<QN>(base, sp.pstride, c, parity & 1, g);
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
    const int rv = bitrev<N>(x);
    sh[(0 * ROWS + r) * N + rv] = make_double2(jx / rho, 0.0);
    sh[(1 * ROWS + r) * N + rv] = make_double2(jy / rho, 0.0);
    sh[(2 * ROWS + r) * N + rv] = make_double2(jz / rho, 0.0);
  }
  __syncthreads();
  butterflies<N>(sh, 3 * ROWS, tw);
  const size_t field = size_t(N) * N * NH;
  for (int e = threadIdx.x; e < 3 * ROWS * NH; e += 256) {
    const int cl = e / NH, kx = e % NH;
    const int comp = cl / ROWS, r = cl % ROWS;
    h[comp * field + (row0 + r) * NH + kx] = sh[cl * N + kx];
  }
}

// Passes 2, 3, 5: transform along y (axis 1) or z (axis 2) of the fields
// h + c * N N NH, c = blockIdx.y; LINES lines (outer, kx) per block, outer =
// z (axis 1) or y (axis 2), consecutive kx. sign -1 forward, +1 inverse.
template <int N, int LINES>
__global__ void __launch_bounds__(256) fft_half_kernel(double2* h0, int axis, int sign, size_t wstride) {
  constexpr int NH = N / 2 + 1;
  __shared__ double2 sh[LINES * N];
  __shared__ double2 tw[N / 2];
  double2* d = in_batch(h0, wstride) + size_t(blockIdx.y) * N * N * NH;
  make_twiddles<N>(tw, sign);
  const int line0 = blockIdx.x * LINES;
  for (int e = threadIdx.x; e < LINES * N; e += 256) {
    const int i = e / LINES, l = e % LINES;
    const int line = line0 + l, outer = line / NH, kx = line % NH;
    const size_t off = axis == 1 ? (size_t(outer) * N + i) * NH + kx : (size_t(i) * N + outer) * NH + kx;
    sh[l * N + bitrev<N>(i)] = d[off];
  }
  __syncthreads();
  butterflies<N>(sh, LINES, tw);
  for (int e = threadIdx.x; e < LINES * N; e += 256) {
    const int i = e / LINES, l = e % LINES;
    const int line = line0 + l, outer = line / NH, kx = line % NH;
    const size_t off = axis == 1 ? (size_t(outer) * N + i) * NH + kx : (size_t(i) * N + outer) * NH + kx;
    d[off] = sh[l * N + i];
  }
}

// Pass 4: LINES z-lines (y, kx) per block. Psi at every kz; per line, the
// shell sums of |k|^2/2 Psi (the line folded by |kz|) into
// sbins[line][kappa] with the number of modes in scnt[line][kappa], and the
// sum of Psi into sbins[line][N/2 + 1], all weighted by the kx weight (rows
// of N/2 + 2 values). Then the inverse transform of Psi along z, written
// over field 0.
template <int N, int LINES>
__global__ void __launch_bounds__(256) psd_zinv_kernel(double2* h0, double* sbins0, double* scnt0, size_t wstride) {
  constexpr int NH = N / 2 + 1, HALF = N / 2;
  __shared__ double2 sh[LINES * N];
  __shared__ double fold[LINES * (HALF + 1)];
  __shared__ double2 tw[N / 2];
  const size_t field = size_t(N) * N * NH;
  double2* h = in_batch(h0, wstride);
  double* sbins = in_batch(sbins0, wstride);
  double* scnt = in_batch(scnt0, wstride);
  make_twiddles<N>(tw, +1);
  const int line0 = blockIdx.x * LINES;
  for (int e = threadIdx.x; e < LINES * N; e += 256) {
    const int i = e / LINES, l = e % LINES;
    const int line = line0 + l, y = line / NH, kx = line % NH;
    const size_t off = (size_t(i) * N + y) * NH + kx;
    const double2 a = h[off], b = h[field + off], c = h[2 * field + off];
    const double psd = a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y + c.x * c.x + c.y * c.y;
    sh[l * N + bitrev<N>(i)] = make_double2(psd, 0.0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int l = wave; l < LINES; l += 4) {
    const int line = line0 + l, y = line / NH, kx = line % NH;
    const int ky = y <= HALF ? y : y - N;
    const int64_t s = int64_t(kx) * kx + int64_t(ky) * ky;
    const double2* ln = sh + l * N;
    double total = 0.0;
    for (int m = lane; m <= HALF; m += 64) {
      double v = ln[bitrev<N>(m)].x;
      if (m >= 1 && m <= HALF - 1) v += ln[bitrev<N>(N - m)].x;
      total += v;
      fold[l * (HALF + 1) + m] = 0.5 * (double(s) + double(m) * m) * v;
    }
    total = wave_sum(total);
    if (lane == 0) {
      const double wkx = (kx == 0 || kx == HALF) ? 1.0 : 2.0;
      sbins[size_t(line) * (HALF + 2) + HALF + 1] = wkx * total;
      scnt[size_t(line) * (HALF + 2) + HALF + 1] = 0.0;
    }
  }
  __syncthreads();
  for (int l = wave; l < LINES; l += 4) {
    const int line = line0 + l, y = line / NH, kx = line % NH;
    const int ky = y <= HALF ? y : y - N;
    const int64_t s = int64_t(kx) * kx + int64_t(ky) * ky;
    const double wkx = (kx == 0 || kx == HALF) ? 1.0 : 2.0;
    for (int r = lane; r <= HALF; r += 64) {
      double sum, cnt;
      shell_interval(fold + l * (HALF + 1), HALF, s, r, sum, cnt);
      sbins[size_t(line) * (HALF + 2) + r] = wkx * sum;
      scnt[size_t(line) * (HALF + 2) + r] = wkx * cnt;
    }
  }
  butterflies<N>(sh, LINES, tw);
  for (int e = threadIdx.x; e < LINES * N; e += 256) {
    const int i = e / LINES, l = e % LINES;
    const int line = line0 + l, y = line / NH, kx = line % NH;
    h[(size_t(i) * N + y) * NH + kx] = sh[l * N + i];
  }
}

// Pass 6: ROWS x-rows (z, y) per block of field 0 (Psi transformed back along
// z and y): the conjugate-symmetric fill of kx = N/2+1..N-1, the inverse
// transform along x (R_h times N^6, real), and per row the shell sums of
// 2 (R_0 - R_h) folded by |hx| into rbins[row][r], with the number of lags in
// rcnt[row][r] (rows of N/2 + 2 values). r0: R_0 times N^6 (the sum of Psi).
template <int N>
__global__ void __launch_bounds__(256)
    inv_x_rows_kernel(const double2* h0, const double* r00, double* rbins0, double* rcnt0, size_t wstride) {
  constexpr int NH = N / 2 + 1, HALF = N / 2;
  constexpr int ROWS = (N * N < 1024 / N) ? N * N : 1024 / N;
  __shared__ double2 sh[ROWS * N];
  __shared__ double fold[ROWS * (HALF + 1)];
  __shared__ double2 tw[N / 2];
  const double2* h = in_batch(h0, wstride);
  const double* r0 = in_batch(r00, wstride);
  double* rbins = in_batch(rbins0, wstride);
  double* rcnt = in_batch(rcnt0, wstride);
  make_twiddles<N>(tw, +1);
  const int row0 = blockIdx.x * ROWS;
  for (int e = threadIdx.x; e < ROWS * N; e += 256) {
    const int r = e / N, k = e % N;
    const size_t rowoff = size_t(row0 + r) * NH;
    double2 v;
    if (k <= HALF) {
      v = h[rowoff + k];
    } else {
      const double2 c = h[rowoff + (N - k)];
      v = make_double2(c.x, -c.y);
    }
    sh[r * N + bitrev<N>(k)] = v;
  }
  __syncthreads();
  butterflies<N>(sh, ROWS, tw);
  const double R0 = *r0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int r = wave; r < ROWS; r += 4) {
    for (int m = lane; m <= HALF; m += 64) {
      double v = 2.0 * (R0 - sh[r * N + m].x);
      if (m >= 1 && m <= HALF - 1) v += 2.0 * (R0 - sh[r * N + (N - m)].x);
      fold[r * (HALF + 1) + m] = v;
    }
  }
  __syncthreads();
  for (int r = wave; r < ROWS; r += 4) {
    const int row = row0 + r, iz = row / N, iy = row % N;
    const int hz = iz <= HALF ? iz : iz - N, hy = iy <= HALF ? iy : iy - N;
    const int64_t s = int64_t(hz) * hz + int64_t(hy) * hy;
    for (int sh_r = lane; sh_r <= HALF; sh_r += 64) {
      double sum, cnt;
      shell_interval(fold + r * (HALF + 1), HALF, s, sh_r, sum, cnt);
      rbins[size_t(row) * (HALF + 2) + sh_r] = sum;
      rcnt[size_t(row) * (HALF + 2) + sh_r] = cnt;
    }
  }
}

// Shell reduction, stage 1: block b sums rows [b CHUNK, (b+1) CHUNK) of the
// row-major tables bins / cnts (width values per row) column by column, in
// row order, into psum[b][col] / pcnt[b][col].
constexpr int kShellChunk = 32;

__global__ void __launch_bounds__(256) shell_partial_kernel(const double* bins0, const double* cnts0, int rows,
                                                            int width, double* psum0, double* pcnt0, size_t wstride) {
  const double* bins = in_batch(bins0, wstride);
  const double* cnts = in_batch(cnts0, wstride);
  double* psum = in_batch(psum0, wstride);
  double* pcnt = in_batch(pcnt0, wstride);
  const int r0 = blockIdx.x * kShellChunk;
  const int r1 = r0 + kShellChunk < rows ? r0 + kShellChunk : rows;
  for (int col = threadIdx.x; col < width; col += 256) {
    double a = 0.0, c = 0.0;
#pragma unroll 8
    for (int r = r0; r < r1; ++r) {
      a += bins[size_t(r) * width + col];
      c += cnts[size_t(r) * width + col];
    }
    psum[size_t(blockIdx.x) * width + col] = a;
    pcnt[size_t(blockIdx.x) * width + col] = c;
  }
}

// Stage 2, one block per column: the partials summed over the chunks (thread
// t takes chunks t, t + 256, ..., then a fixed tree). mode 0 (spectrum):
// out[kappa] = 4 pi / count * sum / N^6 for kappa = 0..N/2 (out may be NULL),
// and column N/2 + 1 (the sum of Psi, R_0 times N^6) into *r0. mode 1
// (structure function): out[r - 1] = sum / count / N^6 for r = 1..N/2.
__global__ void __launch_bounds__(256) shell_final_kernel(const double* psum0, const double* pcnt0, int chunks,
                                                          int width, int n, int mode, double* out0, double* r00,
                                                          size_t wstride) {
  __shared__ double sa[256], sc[256];
  const double* psum = in_batch(psum0, wstride);
  const double* pcnt = in_batch(pcnt0, wstride);
  double* out = out0 ? out0 + size_t(blockIdx.z) * (mode == 0 ? n / 2 + 1 : n / 2) : nullptr;
  double* r0 = r00 ? in_batch(r00, wstride) : nullptr;
  const int col = blockIdx.x;
  double a = 0.0, c = 0.0;
  for (int b = threadIdx.x; b < chunks; b += 256) {
    a += psum[size_t(b) * width + col];
    c += pcnt[size_t(b) * width + col];
  }
  sa[threadIdx.x] = a;
  sc[threadIdx.x] = c;
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
    const int half = n / 2;
    const double sum = sa[0], cnt = sc[0];
    if (mode == 0) {
      if (col <= half && out) out[col] = cnt > 0 ? 4.0 * M_PI / cnt * sum * norm : 0.0;
      if (col == half + 1 && r0) *r0 = sum;
    } else if (col >= 1 && col <= half) {
      out[col - 1] = cnt > 0 ? sum * norm / cnt : 0.0;
    }
  }
}

// Velocity of every sample at the q^3 nodes x = (n/q) * j: out[s][3][q^3].
template <int QN, typename T>
__global__ void __launch_bounds__(64) point_values_kernel(const T* pop, const DevSample* samples, const Seg* segs,
                                                          int q, int physical, double* out) {
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
  const double rho = physical ? (1.0 + d) * sp.u0 : 1.0 + d;   // u / u0 or u
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

// One block per sample: the eight sums of the relative L1 sample error
// (numerator and denominator for the three components and for the Euclidean
// length of the vector) over the q^3 nodes, then their four ratios.
__global__ void __launch_bounds__(256) sample_error_kernel(const double* a, const double* b, int q3, double* ratio) {
  const size_t base = size_t(blockIdx.x) * 3 * q3;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < q3; j += 256) {
    double d2 = 0.0, r2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double x = a[base + size_t(c) * q3 + j], r = b[base + size_t(c) * q3 + j];
      acc[2 * c] += fabs(x - r);
      acc[2 * c + 1] += fabs(r);
      d2 += (x - r) * (x - r);
      r2 += r * r;
    }
    acc[6] += sqrt(d2);
    acc[7] += sqrt(r2);
  }
  __shared__ double red[8][256];
  for (int k = 0; k < 8; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int k = 0; k < 8; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x < 4) ratio[size_t(blockIdx.x) * 4 + threadIdx.x] = red[2 * threadIdx.x][0] / red[2 * threadIdx.x + 1][0];
}

// out[k] = mean over the m samples of ratio[m][k], one block per k.
__global__ void __launch_bounds__(256) sample_mean_kernel(const double* ratio, int m, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) acc += ratio[size_t(i) * 4 + blockIdx.x];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0] / m;
}

// Column statistics of x[m][ld] over its m rows, one block per column: the
// mean by a fixed-order sum, then the spread about it (second pass) with the
// 1/(m - 1) normalisation of the empirical variance.
__global__ void __launch_bounds__(256) ensemble_moments_kernel(const double* x, int m, int64_t ld, double* mean,
                                                               double* sd) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) acc += x[size_t(i) * ld + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double mu = red[0] / m;
  if (threadIdx.x == 0) mean[c] = mu;
  if (!sd) return;
  __syncthreads();  // every thread has read red[0]
  acc = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) {
    const double v = x[size_t(i) * ld + c] - mu;
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) sd[c] = sqrt(red[0] / (m - 1));
}

// Sample-wise compensation of the spectra and structure functions of the
// samples sample0.. (one n): element j of a row of width n + 1 is kappa = j
// of the spectrum for j <= n/2, else lag r = j - n/2 of the structure
// function. Velocities in units of the sample's u0; lags in physical units.
__global__ void __launch_bounds__(256) compensate_kernel(const DevSample* samples, int sample0, int count, int n,
                                                         const double* d, const double* s2, const double* ek,
                                                         double* s2c, double* ekc) {
  constexpr double kKolmogorov = 1.5;
  const int half = n / 2, width = n + 1;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= count * width) return;
  const int s = e / width, j = e % width;
  const double u0 = samples[sample0 + s].u0;
  const double ds = d[s];
  if (j <= half) {
    if (ek) {
      const size_t o = size_t(s) * (half + 1) + j;
      ekc[o] = pow(double(j), 5.0 / 3.0) * (ek[o] / (u0 * u0)) / (kKolmogorov * cbrt(ds * ds));
    }
  } else if (s2) {
    const int r = j - half;
    const size_t o = size_t(s) * half + (r - 1);
    const double dr = ds * (r * 2.0 * M_PI / n);
    s2c[o] = (s2[o] / (u0 * u0)) / cbrt(dr * dr);
  }
}

// LINES for the transforms along y and z (LDS: LINES * N complex doubles);
// it divides N, so it divides the N (N/2 + 1) lines of a field
template <int N>
constexpr int half_lines() {
  return N >= 512 ? 4 : (N >= 256 ? 8 : (N >= 16 ? 16 : 8));
}

struct ObsWork {
  double2* h;       // 3 fields of N * N * NH complex
  double* sbins;    // N NH rows of N/2 + 2
  double* scnt;     // N NH rows of N/2 + 2
  double* rbins;    // N N rows of N/2 + 2
  double* rcnt;     // N N rows of N/2 + 2
  double* psum;     // one row of N/2 + 2 per chunk of N N rows
  double* pcnt;
  double* r0;       // 1
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

size_t chunks_of(size_t rows) { return (rows + kShellChunk - 1) / kShellChunk; }

// bytes of one sample's work area (a multiple of 256)
size_t sample_work_bytes(int n) {
  const size_t nh = size_t(n / 2 + 1), lines = size_t(n) * nh, rows = size_t(n) * n, width = size_t(n / 2 + 2);
  return align256(3 * rows * nh * sizeof(double2)) + 2 * align256(lines * width * sizeof(double)) +
         2 * align256(rows * width * sizeof(double)) + 2 * align256(chunks_of(rows) * width * sizeof(double)) +
         align256(sizeof(double));
}

ObsWork carve(void* work, int n) {
  const size_t nh = size_t(n / 2 + 1), lines = size_t(n) * nh, rows = size_t(n) * n, width = size_t(n / 2 + 2);
  char* p = static_cast<char*>(work);
  ObsWork w;
  w.h = reinterpret_cast<double2*>(p);
  p += align256(3 * rows * nh * sizeof(double2));
  w.sbins = reinterpret_cast<double*>(p);
  p += align256(lines * width * sizeof(double));
  w.scnt = reinterpret_cast<double*>(p);
  p += align256(lines * width * sizeof(double));
  w.rbins = reinterpret_cast<double*>(p);
  p += align256(rows * width * sizeof(double));
  w.rcnt = reinterpret_cast<double*>(p);
  p += align256(rows * width * sizeof(double));
  w.psum = reinterpret_cast<double*>(p);
  p += align256(chunks_of(rows) * width * sizeof(double));
  w.pcnt = reinterpret_cast<double*>(p);
  p += align256(chunks_of(rows) * width * sizeof(double));
  w.r0 = reinterpret_cast<double*>(p);
  return w;
}

template <int QN, typename T, int N>
hipError_t observables_t(const T* pop, const DevSample* samples, int sample0, int count, int parity, void* work,
                         double* s2, double* ek, hipStream_t s) {
  constexpr int NH = N / 2 + 1, L = half_lines<N>();
  constexpr int ROWS_X = N >= 512 ? 1 : 512 / N;
  constexpr int ROWS_R = (N * N < 1024 / N) ? N * N : 1024 / N;
  constexpr int W = N / 2 + 2;
  static_assert(N % L == 0 && (N * N) % ROWS_X == 0 && (N * N) % ROWS_R == 0, "launch shapes must tile the field");
  const ObsWork w = carve(work, N);
  const size_t ws = sample_work_bytes(N);
  const unsigned z = unsigned(count);
  const int lines = N * NH, rows = N * N;
  const int lchunks = int(chunks_of(lines)), rchunks = int(chunks_of(rows));
  hipLaunchKernelGGL((fwd_x_kernel<QN, T, N>), dim3(N * N / ROWS_X, 1, z), dim3(256), 0, s, pop, samples, sample0,
                     parity, w.h, ws);
  hipLaunchKernelGGL((fft_half_kernel<N, L>), dim3(lines / L, 3, z), dim3(256), 0, s, w.h, 1, -1, ws);
  hipLaunchKernelGGL((fft_half_kernel<N, L>), dim3(lines / L, 3, z), dim3(256), 0, s, w.h, 2, -1, ws);
  hipLaunchKernelGGL((psd_zinv_kernel<N, L>), dim3(lines / L, 1, z), dim3(256), 0, s, w.h, w.sbins, w.scnt, ws);
  hipLaunchKernelGGL(shell_partial_kernel, dim3(lchunks, 1, z), dim3(256), 0, s, w.sbins, w.scnt, lines, W, w.psum,
                     w.pcnt, ws);
  hipLaunchKernelGGL(shell_final_kernel, dim3(W, 1, z), dim3(256), 0, s, w.psum, w.pcnt, lchunks, W, N, 0, ek, w.r0,
                     ws);
  if (s2) {
    hipLaunchKernelGGL((fft_half_kernel<N, L>), dim3(lines / L, 1, z), dim3(256), 0, s, w.h, 1, +1, ws);
    hipLaunchKernelGGL((inv_x_rows_kernel<N>), dim3(N * N / ROWS_R, 1, z), dim3(256), 0, s, w.h, w.r0, w.rbins,
                       w.rcnt, ws);
    hipLaunchKernelGGL(shell_partial_kernel, dim3(rchunks, 1, z), dim3(256), 0, s, w.rbins, w.rcnt, rows, W, w.psum,
                       w.pcnt, ws);
    hipLaunchKernelGGL(shell_final_kernel, dim3(W, 1, z), dim3(256), 0, s, w.psum, w.pcnt, rchunks, W, N, 1, s2,
                       nullptr, ws);
  }
  return hipGetLastError();
}

template <int QN, typename T>
hipError_t observables_n(int n, const void* pop, const DevSample* samples, int sample0, int count, int parity,
                         void* work, double* s2, double* ek, hipStream_t s) {
  const T* p = static_cast<const T*>(pop);
  switch (n) {
    case 8: return observables_t<QN, T, 8>(p, samples, sample0, count, parity, work, s2, ek, s);
    case 16: return observables_t<QN, T, 16>(p, samples, sample0, count, parity, work, s2, ek, s);
    case 32: return observables_t<QN, T, 32>(p, samples, sample0, count, parity, work, s2, ek, s);
    case 64: return observables_t<QN, T, 64>(p, samples, sample0, count, parity, work, s2, ek, s);
    case 128: return observables_t<QN, T, 128>(p, samples, sample0, count, parity, work, s2, ek, s);
    case 256: return observables_t<QN, T, 256>(p, samples, sample0, count, parity, work, s2, ek, s);
    case 512: return observables_t<QN, T, 512>(p, samples, sample0, count, parity, work, s2, ek, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

size_t observables_work_bytes(int n, int count) { return sample_work_bytes(n) * size_t(count); }

hipError_t launch_observables(int q, int precision, const void* pop, const DevSample* samples, int32_t sample0,
                              int32_t count, int32_t n, int32_t parity, void* work, double* s2, double* ek,
                              hipStream_t s) {
  if (q == 27) {
    return precision == 0 ? observables_n<27, double>(n, pop, samples, sample0, count, parity, work, s2, ek, s)
                          : observables_n<27, float>(n, pop, samples, sample0, count, parity, work, s2, ek, s);
  }
  if (q == 19) {
    return precision == 0 ? observables_n<19, double>(n, pop, samples, sample0, count, parity, work, s2, ek, s)
                          : observables_n<19, float>(n, pop, samples, sample0, count, parity, work, s2, ek, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_point_values(int lattice, int precision, const void* pop, const DevSample* samples,
                               const Seg* segs, int32_t nseg, int q, int physical, double* out, hipStream_t s) {
  const dim3 grid(unsigned((q * q * q + 63) / 64), unsigned(nseg));
  if (lattice == 27 && precision == 0)
    hipLaunchKernelGGL((point_values_kernel<27, double>), grid, dim3(64), 0, s, static_cast<const double*>(pop),
                       samples, segs, q, physical, out);
  else if (lattice == 27)
    hipLaunchKernelGGL((point_values_kernel<27, float>), grid, dim3(64), 0, s, static_cast<const float*>(pop),
                       samples, segs, q, physical, out);
  else if (lattice == 19 && precision == 0)
    hipLaunchKernelGGL((point_values_kernel<19, double>), grid, dim3(64), 0, s, static_cast<const double*>(pop),
                       samples, segs, q, physical, out);
  else if (lattice == 19)
    hipLaunchKernelGGL((point_values_kernel<19, float>), grid, dim3(64), 0, s, static_cast<const float*>(pop),
                       samples, segs, q, physical, out);
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

hipError_t launch_sample_error(const double* a, const double* b, int m, int q, double* ratio, double* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(sample_error_kernel, dim3(unsigned(m)), dim3(256), 0, s, a, b, q * q * q, ratio);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sample_mean_kernel, dim3(4), dim3(256), 0, s, ratio, m, out);
  return hipGetLastError();
}

hipError_t launch_ensemble_moments(const double* x, int m, int k, int64_t ld, double* mean, double* sd,
                                   hipStream_t s) {
  hipLaunchKernelGGL(ensemble_moments_kernel, dim3(unsigned(k)), dim3(256), 0, s, x, m, ld, mean, sd);
  return hipGetLastError();
}

hipError_t launch_compensate(const DevSample* samples, int sample0, int count, int n, const double* d,
                             const double* s2, const double* ek, double* s2c, double* ekc, hipStream_t s) {
  const int total = count * (n + 1);
  hipLaunchKernelGGL(compensate_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, samples, sample0, count,
                     n, d, s2, ek, s2c, ekc);
  return hipGetLastError();
}

}  // namespace mclbm
