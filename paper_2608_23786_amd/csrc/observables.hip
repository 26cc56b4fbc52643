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
// (the rest follows by conjugate symmetry), fields [z][y][kx]. A shell C_r
// is closed under a change of sign of any lag component, so S2 needs R only
// summed over the lags that fold to f = (|hx|, |hy|, |hz|), f_a = 0..N/2:
// X(f) = sum_{h -> f} R_h = N^-6 sum_k Psi(k) prod_a mu(f_a) cos(2 pi k_a f_a / N)
// with mu(0) = mu(N/2) = 1 and mu = 2 otherwise (the lags behind f_a). The
// inverse transforms therefore run as cosine sums that keep f_a = 0..N/2,
// which shrinks each axis' output to about half. The pipeline is five
// passes over HBM:
//   1. x: velocities from the populations (either AA parity), or from the
//      velocity a record tick captured, and the forward transform along x
//      of the three components, per row in LDS (two real components share
//      one complex transform);
//   2. y: forward transforms along y of the three fields;
//   3. per z-line: the forward transforms along z of the three fields,
//      Psi, its shell sums for the spectrum, its total (R_0), and the
//      folded inverse along z, G[ky][kx][f_z] (real);
//   4. y: the folded inverse along y of G, H[f_y][kx][f_z] (two real lines
//      per complex transform);
//   5. per row (f_y, f_z): the folded inverse along x (H is even in kx once
//      y and z are folded, so its transform is real; two rows per complex
//      transform), X(f), and the shell sums for S2.
// Radix-2/4 decimation-in-time transforms of whole lines in LDS (padded
// against bank conflicts), the first and last stage in registers of the
// thread that loads or keeps a quartet of the line, twiddles by sincospi;
// each launch hands every XCD
// a contiguous run of blocks, so that blocks sharing cache lines share an
// L2. Shells hold the integer vectors (minimum image, components in
// {-N/2+1, ..., N/2}) whose length rounds to the shell index. Every shell sum
// is taken per line (the line folded by the magnitude of its own
// coordinate, the lengths of a shell forming an interval of it), then over
// the lines of a block, then over blocks, each in a fixed order: results do
// not depend on scheduling. The number of vectors in a shell depends on N
// only and is counted exactly in the last stage. A half-spectrum mode
// 0 < kx < N/2 stands for itself and its conjugate partner at -k, which has
// the same length: weight 2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "lbm_device.h"

namespace mclbm {
namespace {

// Lines per block of the transforms along y and z (LDS: about LINES * N
// complex doubles); it divides n, so it divides the n (n/2 + 1) lines of a
// field.
constexpr int half_lines(int n) { return n >= 512 ? 4 : (n >= 256 ? 8 : (n >= 16 ? 16 : 8)); }

// Lines per block of the z pass (its LDS holds the lines and Psi of each)
constexpr int z_lines(int n) { return n == 128 ? 8 : half_lines(n); }

// Pairs of real lines per block of the folded inverse passes along y and x
// (one complex transform per pair; LDS: about PAIRS * N complex doubles)
constexpr int cos_pairs(int n) { return n >= 512 ? 4 : (n >= 128 ? 8 : 16); }

// Lines of the folded passes: (N/2 + 1)^2 per value of the other index
constexpr size_t folded_lines(int n) { return size_t(n / 2 + 1) * (n / 2 + 1); }

// rows of the spectrum's and the structure function's shell tables: one
// per block of the pass that writes them
constexpr size_t spectrum_bin_rows(int n) { return size_t(n) * (n / 2 + 1) / z_lines(n); }
constexpr size_t sf_bin_rows(int n) { return (folded_lines(n) + 2 * cos_pairs(n) - 1) / (2 * cos_pairs(n)); }

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

// LDS slot of element p of a line (or of the twiddle table): one spare slot
// after every 16 complex values (256 bytes), so that the bit-reversed and
// strided accesses of a wave spread over the LDS banks instead of landing
// on a few of them.
__device__ __forceinline__ int lds_pos(int p) { return p + (p >> 4); }

// LDS slots from one line of N complex values to the next: the padded line
// plus one slot, an odd number of 16-byte slots, so that the lanes of a wave
// that touch the same element of consecutive lines (the loads and stores of
// the y and z passes, where consecutive lanes take consecutive lines to keep
// their global accesses contiguous) fall on different banks.
template <int N>
constexpr int lds_line() {
  return N + N / 16 + 1;
}

// e^{sign 2 pi i k / N}, k < N/2, at tw[lds_pos(k)]
template <int N>
__device__ __forceinline__ void make_twiddles(double2* tw, int sign) {
  for (int k = threadIdx.x; k < N / 2; k += blockDim.x) {
    double s, c;
    sincospi(2.0 * k / N, &s, &c);
    tw[lds_pos(k)] = make_double2(c, sign * s);
  }
}

// Transforms of whole lines in LDS, decimation in time (bit-reversed
// input, radix-4 steps of two radix-2 stages, an odd number of stages
// starting with one radix-2 stage), with the first and the last stage in
// registers, for a thread that holds a quartet of a line: the elements r, r + N/4, r + N/2,
// r + 3N/4 (natural order, r < N/4). The first stage of the
// decimation-in-time transform combines exactly such a quartet: with an
// even number of radix-2 stages, the first radix-4 step reads bit-reversed
// positions 4j..4j+3, which hold elements r, r + N/2, r + N/4, r + 3N/4 for
// j = bitrev(r) / 4; with an odd number, the first radix-2 stage pairs
// (r, r + N/2) at positions 2 j1, 2 j1 + 1 (j1 = bitrev(r) / 2) and
// (r + N/4, r + 3N/4) at 2 j2, 2 j2 + 1 (j2 = bitrev(r + N/4) / 2). The last
// radix-4 step (span N/4) leaves, for j < N/4, the outputs j, j + N/4,
// j + N/2, j + 3N/4 in one thread. So a quartet is loaded from memory, put
// through the first stage and written to LDS once; the middle steps run in
// LDS as above; the last step reads LDS once and hands the output quartet
// back in registers. Per transform that saves two of the LDS passes.
// sign: -1 forward, +1 inverse (the twiddle e^{sign i pi/2} of the first
// radix-4 step is (0, sign)).
template <int N>
__device__ __forceinline__ void first_stage_to_lds(double2* ln, int r, const double2 (&x)[4], int sign) {
  constexpr int LOG = log2_of<N>();
  if constexpr ((LOG & 1) == 0) {
    const int p = bitrev<N>(r);  // 4j
    const double2 y0 = make_double2(x[0].x + x[2].x, x[0].y + x[2].y);
    const double2 y1 = make_double2(x[0].x - x[2].x, x[0].y - x[2].y);
    const double2 y2 = make_double2(x[1].x + x[3].x, x[1].y + x[3].y);
    const double2 y3 = make_double2(x[1].x - x[3].x, x[1].y - x[3].y);
    const double2 u3 = cmul(make_double2(0.0, double(sign)), y3);
    ln[lds_pos(p)] = make_double2(y0.x + y2.x, y0.y + y2.y);
    ln[lds_pos(p + 2)] = make_double2(y0.x - y2.x, y0.y - y2.y);
    ln[lds_pos(p + 1)] = make_double2(y1.x + u3.x, y1.y + u3.y);
    ln[lds_pos(p + 3)] = make_double2(y1.x - u3.x, y1.y - u3.y);
  } else {
    const int p1 = bitrev<N>(r), p2 = bitrev<N>(r + N / 4);  // 2 j1, 2 j2
    ln[lds_pos(p1)] = make_double2(x[0].x + x[2].x, x[0].y + x[2].y);
    ln[lds_pos(p1 + 1)] = make_double2(x[0].x - x[2].x, x[0].y - x[2].y);
    ln[lds_pos(p2)] = make_double2(x[1].x + x[3].x, x[1].y + x[3].y);
    ln[lds_pos(p2 + 1)] = make_double2(x[1].x - x[3].x, x[1].y - x[3].y);
  }
}

// The radix-4 steps between the first stage and the last (spans 4, 16, ...
// or 2, 8, ... below N/4) over nl lines in LDS; every thread of the block
// takes part, and the block is synchronised after each step.
template <int N>
__device__ __forceinline__ void radix4_steps(double2* sh, int nl, const double2* tw, int half0) {
  for (int half = half0; half < N / 4; half <<= 2) {
    const int sa = N / (2 * half), sb = N / (4 * half);
    for (int b = threadIdx.x; b < nl * (N / 4); b += blockDim.x) {
      const int l = b / (N / 4), j = b % (N / 4);
      const int pos = j % half, grp = j / half;
      double2* ln = sh + l * lds_line<N>();
      const int i0 = grp * 4 * half + pos;
      const int p0 = lds_pos(i0), p1 = lds_pos(i0 + half), p2 = lds_pos(i0 + 2 * half), p3 = lds_pos(i0 + 3 * half);
      const double2 x0 = ln[p0], x1 = ln[p1], x2 = ln[p2], x3 = ln[p3];
      const double2 wa = tw[lds_pos(pos * sa)];
      const double2 t1 = cmul(wa, x1), t3 = cmul(wa, x3);
      const double2 y0 = make_double2(x0.x + t1.x, x0.y + t1.y), y1 = make_double2(x0.x - t1.x, x0.y - t1.y);
      const double2 y2 = make_double2(x2.x + t3.x, x2.y + t3.y), y3 = make_double2(x2.x - t3.x, x2.y - t3.y);
      const double2 u2 = cmul(tw[lds_pos(pos * sb)], y2), u3 = cmul(tw[lds_pos((pos + half) * sb)], y3);
      ln[p0] = make_double2(y0.x + u2.x, y0.y + u2.y);
      ln[p2] = make_double2(y0.x - u2.x, y0.y - u2.y);
      ln[p1] = make_double2(y1.x + u3.x, y1.y + u3.y);
      ln[p3] = make_double2(y1.x - u3.x, y1.y - u3.y);
    }
    __syncthreads();
  }
}

template <int N>
__device__ __forceinline__ void middle_steps(double2* sh, int nl, const double2* tw) {
  radix4_steps<N>(sh, nl, tw, (log2_of<N>() & 1) ? 2 : 4);
}

// Every stage but the last of nl lines loaded into LDS in bit-reversed order
// (the first radix-2 stage of an odd number of stages included); the block
// is synchronised after each step.
template <int N>
__device__ __forceinline__ void all_but_last_steps(double2* sh, int nl, const double2* tw) {
  constexpr int LOG = log2_of<N>();
  if constexpr (LOG & 1) {
    for (int b = threadIdx.x; b < nl * (N / 2); b += blockDim.x) {
      const int l = b / (N / 2), j = b % (N / 2);
      double2* ln = sh + l * lds_line<N>();
      const int p0 = lds_pos(2 * j), p1 = lds_pos(2 * j + 1);
      const double2 a = ln[p0], c = ln[p1];
      ln[p0] = make_double2(a.x + c.x, a.y + c.y);
      ln[p1] = make_double2(a.x - c.x, a.y - c.y);
    }
    __syncthreads();
  }
  radix4_steps<N>(sh, nl, tw, (LOG & 1) ? 2 : 1);
}

// The last radix-4 step (span N/4) for outputs j, j + N/4, j + N/2, j + 3N/4
// of one line (j < N/4): o[m] is output j + m N/4.
template <int N>
__device__ __forceinline__ void last_step_from_lds(const double2* ln, int j, const double2* tw, double2 (&o)[4]) {
  constexpr int Q4 = N / 4;
  const double2 x0 = ln[lds_pos(j)], x1 = ln[lds_pos(j + Q4)], x2 = ln[lds_pos(j + 2 * Q4)],
                x3 = ln[lds_pos(j + 3 * Q4)];
  const double2 wa = tw[lds_pos(2 * j)];
  const double2 t1 = cmul(wa, x1), t3 = cmul(wa, x3);
  const double2 y0 = make_double2(x0.x + t1.x, x0.y + t1.y), y1 = make_double2(x0.x - t1.x, x0.y - t1.y);
  const double2 y2 = make_double2(x2.x + t3.x, x2.y + t3.y), y3 = make_double2(x2.x - t3.x, x2.y - t3.y);
  const double2 u2 = cmul(tw[lds_pos(j)], y2), u3 = cmul(tw[lds_pos(j + Q4)], y3);
  o[0] = make_double2(y0.x + u2.x, y0.y + u2.y);
  o[2] = make_double2(y0.x - u2.x, y0.y - u2.y);
  o[1] = make_double2(y1.x + u3.x, y1.y + u3.y);
  o[3] = make_double2(y1.x - u3.x, y1.y - u3.y);
}

// A batch of samples shares one launch: blockIdx.z is the sample's place in
// the batch, and its work area starts wstride bytes after the previous one.
template <typename P>
__device__ __forceinline__ P* in_batch(P* p, size_t wstride) {
  using B = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<B*>(p) + size_t(blockIdx.z) * wstride);
}

// floor(sqrt(v)) for 0 <= v < 2^24, which holds for every value the shell
// ranges meet (n <= 1024): the float square root is within a unit of it and
// the two loops correct it.
__device__ __forceinline__ int isqrt_floor(int v) {
  if (v <= 0) return 0;
  int r = int(sqrtf(float(v)));
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// The m in [0, half] with round(sqrt(s + m^2)) == r form the interval
// [a, b] (empty when a > b): m^2 in [ceil(((2r-1)^2 - 4s)/4),
// floor(((2r+1)^2 - 1 - 4s)/4)].
__device__ __forceinline__ void shell_range(int half, int s, int r, int& a, int& b) {
  a = 1;
  b = 0;
  const int lo2 = r == 0 ? 0 : (2 * r - 1) * (2 * r - 1);
  const int top = (2 * r + 1) * (2 * r + 1) - 1 - 4 * s;
  if (top < 0) return;
  const int m2max = top / 4;
  const int bot = lo2 - 4 * s;
  const int m2min = bot <= 0 ? 0 : (bot + 3) / 4;
  if (m2min > m2max) return;
  int lo = isqrt_floor(m2min);
  if (lo * lo < m2min) ++lo;
  int hi = isqrt_floor(m2max);
  if (hi > half) hi = half;
  a = lo;
  b = hi;
}

// Lattice vectors a folded index m stands for: m and -m, except m = 0 and
// m = half (the Nyquist value is present once).
__device__ __forceinline__ double fold_weight(int m, int half) { return (m == 0 || m == half) ? 1.0 : 2.0; }

// Lattice vectors standing behind the folded indices a..b
__device__ __forceinline__ double range_count(int half, int a, int b) {
  if (a > b) return 0.0;
  return 2.0 * (b - a + 1) - (a == 0 ? 1.0 : 0.0) - (b == half ? 1.0 : 0.0);
}

// x-rows per block of the forward transform along x: two nodes per thread,
// and an even number of rows (two rows share one transform of uz)
constexpr int fwd_rows(int n) { return n >= 256 ? 2 : 512 / n; }

// Pass 1: ROWS rows (z, y) per block. Velocities of the rows' nodes from the
// populations (the parity selects the AA slots; consecutive threads take
// consecutive nodes of a row, so every population plane is read in
// contiguous runs), or, with FROM_U, read from the velocity a record tick
// captured (u + voffset, three planes of N^3; pop and parity unused), and
// the forward transform along x of the three
// components, kx = 0..N/2 written to h[c][(z N + y) NH + kx]. The components
// are real, so two share one complex transform: ux + i uy of each row, and
// uz of a pair of rows, loaded into LDS in bit-reversed order; the two
// spectra of a line are separated afterwards from Z(k) and Z(N - k):
// A(k) = (Z(k) + conj Z(N - k)) / 2, B(k) = (Z(k) - conj Z(N - k)) / 2i.
template <int QN, typename T, int N, bool FROM_U>
__global__ void __launch_bounds__(256) fwd_x_kernel(const T* pop, const double* u, const DevSample* samples,
                                                    int sample0, int parity, double2* h0, size_t wstride) {
  constexpr int ROWS = fwd_rows(N), PAIRS = ROWS / 2, LINES = ROWS + PAIRS;
  constexpr int NH = N / 2 + 1, Q4 = N / 4;
  constexpr int LS = lds_line<N>();
  __shared__ double2 sh[LINES * LS];
  __shared__ double2 tw[lds_line<N / 2>()];
  const DevSample& sp = samples[sample0 + blockIdx.z];
  double2* h = in_batch(h0, wstride);
  const size_t row0 = size_t(remap_block(blockIdx.x, gridDim.x, 1)) * ROWS;
  make_twiddles<N>(tw, -1);
  double* shd = reinterpret_cast<double*>(sh);
  for (int e = threadIdx.x; e < ROWS * N; e += 256) {
    const int r = e / N, x = e % N;
    const uint32_t cell = uint32_t((row0 + r) * N + x);
    double ux, uy, uz;
    if constexpr (FROM_U) {
      constexpr size_t plane = size_t(N) * N * N;
      const double* ub = u + sp.voffset;
      ux = ub[cell];
      uy = ub[plane + cell];
      uz = ub[2 * plane + cell];
    } else {
      T g[Q];
      load_state<QN>(pop + sp.offset, sp.pstride, make_cell(cell, sp.log2n), parity & 1, g);
      node_velocity<QN>(g, ux, uy, uz);
    }
    const int rv = lds_pos(bitrev<N>(x));
    sh[r * LS + rv] = make_double2(ux, uy);
    shd[2 * ((ROWS + r / 2) * LS + rv) + (r & 1)] = uz;
  }
  __syncthreads();
  all_but_last_steps<N>(sh, LINES, tw);
  // the last step, its outputs back into the slots it read (the same thread's)
  for (int e = threadIdx.x; e < LINES * Q4; e += 256) {
    const int l = e / Q4, j = e % Q4;
    double2 o[4];
    last_step_from_lds<N>(sh + l * LS, j, tw, o);
#pragma unroll
    for (int m = 0; m < 4; ++m) sh[l * LS + lds_pos(j + m * Q4)] = o[m];
  }
  __syncthreads();
  const size_t field = size_t(N) * N * NH;
  for (int e = threadIdx.x; e < LINES * NH; e += 256) {
    const int l = e / NH, k = e % NH;
    const double2 z = sh[l * LS + lds_pos(k)];
    const double2 zn = sh[l * LS + lds_pos((N - k) & (N - 1))];
    const double2 a = make_double2(0.5 * (z.x + zn.x), 0.5 * (z.y - zn.y));  // (Z(k) + conj Z(N-k)) / 2
    const double2 b = make_double2(0.5 * (z.y + zn.y), 0.5 * (zn.x - z.x));  // (Z(k) - conj Z(N-k)) / 2i
    if (l < ROWS) {
      h[(row0 + l) * NH + k] = a;
      h[field + (row0 + l) * NH + k] = b;
    } else {
      const int p = l - ROWS;
      h[2 * field + (row0 + 2 * p) * NH + k] = a;
      h[2 * field + (row0 + 2 * p + 1) * NH + k] = b;
    }
  }
}

// Pass 2: transform along y of the fields h + c * N N NH,
// c = blockIdx.y; LINES lines (z, kx) per block, consecutive kx, a quartet of
// a line per thread (consecutive threads take consecutive lines, so their
// global accesses are contiguous). sign -1 forward, +1 inverse.
template <int N, int LINES>
__global__ void __launch_bounds__(256) fft_y_kernel(double2* h0, int sign, size_t wstride) {
  constexpr int NH = N / 2 + 1, LS = lds_line<N>(), Q4 = N / 4;
  __shared__ double2 sh[LINES * LS];
  __shared__ double2 tw[lds_line<N / 2>()];
  double2* d = in_batch(h0, wstride) + size_t(blockIdx.y) * N * N * NH;
  make_twiddles<N>(tw, sign);
  const int line0 = remap_block(blockIdx.x, gridDim.x, 1) * LINES;
  for (int e = threadIdx.x; e < LINES * Q4; e += 256) {
    const int r = e / LINES, l = e % LINES;
    const int line = line0 + l, z = line / NH, kx = line % NH;
    double2 x[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) x[m] = d[(size_t(z) * N + r + m * Q4) * NH + kx];
    first_stage_to_lds<N>(sh + l * LS, r, x, sign);
  }
  __syncthreads();
  middle_steps<N>(sh, LINES, tw);
  for (int e = threadIdx.x; e < LINES * Q4; e += 256) {
    const int j = e / LINES, l = e % LINES;
    const int line = line0 + l, z = line / NH, kx = line % NH;
    double2 o[4];
    last_step_from_lds<N>(sh + l * LS, j, tw, o);
#pragma unroll
    for (int m = 0; m < 4; ++m) d[(size_t(z) * N + j + m * Q4) * NH + kx] = o[m];
  }
}

// Pass 3: LINES z-lines (y, kx) per block, a quartet of a line per thread
// (consecutive threads on consecutive lines). The forward transform along z
// of each of the three fields (already transformed along x and y), one
// field at a time in LDS, with Psi, the sum of |.|^2 over the fields, kept in
// registers (the quartets of a thread are the same for every field, and the
// inverse transform's first stage takes the same quartets). Psi then goes to
// the transform's LDS in natural order for the shell sums of |k|^2/2 Psi
// over the block's lines (each line folded by |kz| and weighted by its kx
// weight, the lines added in order) into sbins[block][kappa] and the sum of
// Psi into sbins[block][N/2 + 1] (rows of N/2 + 2 values); last, the folded
// inverse transform of Psi along z, G(f_z) = mu(f_z) Re F^-1(Psi)(f_z) for
// f_z = 0..N/2 (Psi is real, so that real part is even), written to
// g[(ky NH + kx)(N/2 + 1) + f_z]: the block's lines are consecutive (ky, kx),
// so it writes one contiguous run. One LDS area serves all three, which
// keeps a block at the transform's LDS.
template <int N, int LINES>
__global__ void __launch_bounds__(256) z_psd_kernel(const double2* h0, double* g0, double* sbins0, size_t wstride) {
  constexpr int NH = N / 2 + 1, HALF = N / 2, LS = lds_line<N>(), Q4 = N / 4;
  constexpr int PER = (LINES * Q4 + 255) / 256;  // quartets per thread
  __shared__ double2 sh[LINES * LS];
  __shared__ double tot[LINES];
  __shared__ double2 tw[lds_line<N / 2>()];
  // Psi of every line and the (line, shell) sums live in the transform's LDS
  // between the forward and the inverse transforms
  static_assert(sizeof(double) * LINES * (N + HALF + 1) <= sizeof(sh), "Psi and the line sums fit in the LDS");
  double* psi = reinterpret_cast<double*>(sh);
  double* part = psi + LINES * N;
  const size_t field = size_t(N) * N * NH;
  const double2* h = in_batch(h0, wstride);
  double* g = in_batch(g0, wstride);
  double* sbins = in_batch(sbins0, wstride);
  make_twiddles<N>(tw, -1);
  const int line0 = remap_block(blockIdx.x, gridDim.x, 1) * LINES;
  double ps[PER][4];
#pragma unroll
  for (int k = 0; k < PER; ++k)
#pragma unroll
    for (int m = 0; m < 4; ++m) ps[k][m] = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double2* d = h + c * field;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = threadIdx.x + 256 * k;
      if (e < LINES * Q4) {
        const int r = e / LINES, l = e % LINES;
        const int line = line0 + l, y = line / NH, kx = line % NH;
        double2 x[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) x[m] = d[(size_t(r + m * Q4) * N + y) * NH + kx];
        first_stage_to_lds<N>(sh + l * LS, r, x, -1);
      }
    }
    __syncthreads();
    middle_steps<N>(sh, LINES, tw);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = threadIdx.x + 256 * k;
      if (e < LINES * Q4) {
        double2 o[4];
        last_step_from_lds<N>(sh + (e % LINES) * LS, e / LINES, tw, o);
#pragma unroll
        for (int m = 0; m < 4; ++m) ps[k][m] += o[m].x * o[m].x + o[m].y * o[m].y;
      }
    }
    __syncthreads();  // the next field (or Psi) overwrites sh
  }
  // Psi in natural order; the inverse transform's twiddles are the
  // conjugates of the forward ones
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + 256 * k;
    if (e < LINES * Q4) {
      const int j = e / LINES, l = e % LINES;
#pragma unroll
      for (int m = 0; m < 4; ++m) psi[l * N + j + m * Q4] = ps[k][m];
    }
  }
  for (int k = threadIdx.x; k < N / 2; k += 256) tw[lds_pos(k)].y = -tw[lds_pos(k)].y;
  __syncthreads();
  // the total of Psi per line (R_0), one wave per line
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int l = wave; l < LINES; l += 4) {
    const int kx = (line0 + l) % NH;
    double total = 0.0;
    for (int i = lane; i < N; i += 64) total += psi[l * N + i];
    total = wave_sum(total);
    if (lane == 0) tot[l] = fold_weight(kx, HALF) * total;
  }
  // the shell sums of every (line, shell) pair over all threads, each line
  // folded by |kz|; then the block's lines added per shell in line order
  for (int e = threadIdx.x; e < LINES * (HALF + 1); e += 256) {
    const int l = e / (HALF + 1), r = e % (HALF + 1);
    const int line = line0 + l, y = line / NH, kx = line % NH;
    const int ky = y <= HALF ? y : y - N;
    const int sxy = kx * kx + ky * ky;
    int a, b;
    shell_range(HALF, sxy, r, a, b);
    const double* pl = psi + l * N;
    double sum = 0.0;
    for (int m = a; m <= b; ++m) {
      double v = pl[m];
      if (m >= 1 && m <= HALF - 1) v += pl[N - m];
      sum += 0.5 * (double(sxy) + double(m) * m) * v;
    }
    part[e] = fold_weight(kx, HALF) * sum;
  }
  __syncthreads();
  const size_t blk = size_t(line0 / LINES);
  for (int r = threadIdx.x; r <= HALF + 1; r += 256) {
    double sum = 0.0;
    for (int l = 0; l < LINES; ++l) sum += r == HALF + 1 ? tot[l] : part[l * (HALF + 1) + r];
    sbins[blk * (HALF + 2) + r] = sum;
  }
  __syncthreads();  // Psi and the sums are read; the inverse overwrites sh
  // the inverse transform of Psi along z, its first stage from the registers
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + 256 * k;
    if (e < LINES * Q4) {
      const int j = e / LINES, l = e % LINES;
      double2 x[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) x[m] = make_double2(ps[k][m], 0.0);
      first_stage_to_lds<N>(sh + l * LS, j, x, +1);
    }
  }
  __syncthreads();
  middle_steps<N>(sh, LINES, tw);
  // outputs j and j + N/4 of a quartet lie in 0..N/2 - 1, and j + N/2 is N/2
  // for j = 0; mu is 2 except at 0 and N/2
  double gv[PER][3];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + 256 * k;
    if (e < LINES * Q4) {
      const int j = e / LINES, l = e % LINES;
      double2 o[4];
      last_step_from_lds<N>(sh + l * LS, j, tw, o);
      gv[k][0] = (j == 0 ? 1.0 : 2.0) * o[0].x;
      gv[k][1] = 2.0 * o[1].x;
      gv[k][2] = o[2].x;
    }
  }
  __syncthreads();  // the transform's reads are done; sh stages the output
  constexpr int HP = HALF + 1;
  double* stage = reinterpret_cast<double*>(sh);
  static_assert(sizeof(double) * LINES * HP <= sizeof(sh), "the folded lines fit in the LDS");
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + 256 * k;
    if (e < LINES * Q4) {
      const int j = e / LINES, l = e % LINES;
      stage[l * HP + j] = gv[k][0];
      stage[l * HP + j + Q4] = gv[k][1];
      if (j == 0) stage[l * HP + HALF] = gv[k][2];
    }
  }
  __syncthreads();
  double* out = g + size_t(line0) * HP;
  for (int i = threadIdx.x; i < LINES * HP; i += 256) out[i] = stage[i];
}

// Pass 4: the folded inverse transform along y. Lines j = kx (N/2 + 1) + f_z
// of G[ky][j] (J = (N/2 + 1)^2 of them), 2 PAIRS consecutive lines per block
// (consecutive threads take consecutive lines, so each ky is read in one
// contiguous run); two real lines share one complex transform,
// Z = G_a + i G_b, and H[f_y][j] = mu(f_y) sum_ky G[ky][j] cos(2 pi ky f_y / N)
// is mu(f_y) Re of their transforms: Re A(f) = (Re Z(f) + Re Z(N - f)) / 2,
// Re B(f) = (Im Z(f) + Im Z(N - f)) / 2, for f_y = 0..N/2. Lines past J
// transform zeros and are not written.
template <int N, int PAIRS>
__global__ void __launch_bounds__(256) cos_y_kernel(const double* g0, double* hout0, size_t wstride) {
  constexpr int HALF = N / 2, HP = HALF + 1, J = HP * HP, LS = lds_line<N>(), Q4 = N / 4;
  constexpr int PER = (PAIRS * Q4 + 255) / 256;
  __shared__ double2 sh[PAIRS * LS];
  __shared__ double2 tw[lds_line<N / 2>()];
  const double* g = in_batch(g0, wstride);
  double* ho = in_batch(hout0, wstride);
  make_twiddles<N>(tw, +1);
  const int j0 = remap_block(blockIdx.x, gridDim.x, 1) * 2 * PAIRS;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + 256 * k;
    if (e < PAIRS * Q4) {
      const int r = e / PAIRS, p = e % PAIRS;
      const int ja = j0 + 2 * p, jb = ja + 1;
      double2 x[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const size_t row = size_t(r + m * Q4) * J;
        x[m] = make_double2(ja < J ? g[row + ja] : 0.0, jb < J ? g[row + jb] : 0.0);
      }
      first_stage_to_lds<N>(sh + p * LS, r, x, +1);
    }
  }
  __syncthreads();
  middle_steps<N>(sh, PAIRS, tw);
  // the last step, its outputs back into the slots it read (the same thread's)
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + 256 * k;
    if (e < PAIRS * Q4) {
      const int j = e / PAIRS, p = e % PAIRS;
      double2 o[4];
      last_step_from_lds<N>(sh + p * LS, j, tw, o);
#pragma unroll
      for (int m = 0; m < 4; ++m) sh[p * LS + lds_pos(j + m * Q4)] = o[m];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < HP * PAIRS; e += 256) {
    const int f = e / PAIRS, p = e % PAIRS;
    const int ja = j0 + 2 * p;
    if (ja >= J) continue;
    const double2 z = sh[p * LS + lds_pos(f)], zn = sh[p * LS + lds_pos((N - f) & (N - 1))];
    const bool edge = f == 0 || f == HALF;  // mu = 1 and Z(N - f) = Z(f)
    ho[size_t(f) * J + ja] = edge ? z.x : z.x + zn.x;
    if (ja + 1 < J) ho[size_t(f) * J + ja + 1] = edge ? z.y : z.y + zn.y;
  }
}

// Pass 5: the folded inverse transform along x and the shell sums of S2.
// Rows q = f_y (N/2 + 1) + f_z of H[f_y][kx][f_z] (lines along kx =
// 0..N/2), 2 PAIRS consecutive rows per block. With y and z folded, H is
// even in kx (a mode at -kx is the conjugate partner of one at kx with ky,
// kz negated, and the folds are even in those), so the transform of its
// even extension is real: two rows share one complex transform, Z = E_a +
// i E_b giving x_a + i x_b, and X(f) = mu(f_x) x(f_x) is N^6 times the sum
// of R_h over the lags that fold to f. The shell sums of
// 2 (mu(f) R_0 - X(f)) (mu(f) the number of those lags) over the block's
// rows (each row folded by f_x, the rows added in order) go to
// rbins[block][r] (rows of N/2 + 2 values, the last one 0). r0: R_0 times
// N^6 (the sum of Psi). Rows past (N/2 + 1)^2 transform zeros and add
// nothing.
template <int N, int PAIRS>
__global__ void __launch_bounds__(256)
    cos_x_kernel(const double* hin0, const double* r00, double* rbins0, size_t wstride) {
  constexpr int HALF = N / 2, HP = HALF + 1, J = HP * HP, LS = lds_line<N>(), Q4 = N / 4, ROWS = 2 * PAIRS;
  constexpr int PER = (PAIRS * Q4 + 255) / 256;
  // the transforms, then (as doubles) the rows' X values and their shell sums
  constexpr int SH = PAIRS * LS > ROWS * HP ? PAIRS * LS : ROWS * HP;
  __shared__ double2 sh[SH];
  __shared__ double2 tw[lds_line<N / 2>()];
  const double* hin = in_batch(hin0, wstride);
  const double* r0 = in_batch(r00, wstride);
  double* rbins = in_batch(rbins0, wstride);
  make_twiddles<N>(tw, +1);
  const int q0 = remap_block(blockIdx.x, gridDim.x, 1) * ROWS;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + 256 * k;
    if (e < PAIRS * Q4) {
      const int r = e / PAIRS, p = e % PAIRS;
      const int qa = q0 + 2 * p, qb = qa + 1;
      const size_t ba = size_t(qa / HP) * J + qa % HP, bb = size_t(qb / HP) * J + qb % HP;
      double2 x[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int kx = r + m * Q4, kf = kx <= HALF ? kx : N - kx;  // the even extension
        x[m] = make_double2(qa < J ? hin[ba + size_t(kf) * HP] : 0.0, qb < J ? hin[bb + size_t(kf) * HP] : 0.0);
      }
      first_stage_to_lds<N>(sh + p * LS, r, x, +1);
    }
  }
  __syncthreads();
  middle_steps<N>(sh, PAIRS, tw);
  // outputs j and j + N/4 of a quartet lie in 0..N/2 - 1, and j + N/2 is N/2
  // for j = 0
  double xv[PER][3][2];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + 256 * k;
    if (e < PAIRS * Q4) {
      const int j = e / PAIRS, p = e % PAIRS;
      double2 o[4];
      last_step_from_lds<N>(sh + p * LS, j, tw, o);
      const double w0 = j == 0 ? 1.0 : 2.0;
      xv[k][0][0] = w0 * o[0].x;
      xv[k][0][1] = w0 * o[0].y;
      xv[k][1][0] = 2.0 * o[1].x;
      xv[k][1][1] = 2.0 * o[1].y;
      xv[k][2][0] = o[2].x;
      xv[k][2][1] = o[2].y;
    }
  }
  __syncthreads();  // the transform's reads are done; sh holds the rows next
  double* xr = reinterpret_cast<double*>(sh);  // [ROWS][HP]
  double* part = xr + ROWS * HP;                // [ROWS][HP]
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = threadIdx.x + 256 * k;
    if (e < PAIRS * Q4) {
      const int j = e / PAIRS, p = e % PAIRS;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        double* row = xr + (2 * p + b) * HP;
        row[j] = xv[k][0][b];
        row[j + Q4] = xv[k][1][b];
        if (j == 0) row[HALF] = xv[k][2][b];
      }
    }
  }
  __syncthreads();
  const double R0 = *r0;
  for (int e = threadIdx.x; e < ROWS * HP; e += 256) {
    const int rho = e / HP, c = e % HP;
    const int q = q0 + rho;
    double sum = 0.0;
    if (q < J) {
      const int fy = q / HP, fz = q % HP;
      const double myz = fold_weight(fy, HALF) * fold_weight(fz, HALF);
      int a, b;
      shell_range(HALF, fy * fy + fz * fz, c, a, b);
      const double* row = xr + rho * HP;
      for (int m = a; m <= b; ++m) sum += 2.0 * (myz * fold_weight(m, HALF) * R0 - row[m]);
    }
    part[e] = sum;
  }
  __syncthreads();
  const size_t blk = size_t(q0 / ROWS);
  for (int c = threadIdx.x; c <= HALF + 1; c += 256) {
    double sum = 0.0;
    for (int r = 0; r < ROWS && c <= HALF; ++r) sum += part[r * HP + c];
    rbins[blk * (HALF + 2) + c] = sum;
  }
}

// Shell reduction, stage 1: block b sums rows [b CHUNK, (b+1) CHUNK) of the
// row-major table bins (width values per row) column by column, in row
// order, into psum[b][col].
constexpr int kShellChunk = 32;

__global__ void __launch_bounds__(256) shell_partial_kernel(const double* bins0, int rows, int width, double* psum0,
                                                            size_t wstride) {
  const double* bins = in_batch(bins0, wstride);
  double* psum = in_batch(psum0, wstride);
  const int r0 = blockIdx.x * kShellChunk;
  const int r1 = r0 + kShellChunk < rows ? r0 + kShellChunk : rows;
  for (int col = threadIdx.x; col < width; col += 256) {
    double a = 0.0;
#pragma unroll 8
    for (int r = r0; r < r1; ++r) a += bins[size_t(r) * width + col];
    psum[size_t(blockIdx.x) * width + col] = a;
  }
}

// Number of lattice vectors of each shell, one block per shell r = 0..N/2:
// the vectors with components in {-N/2+1, ..., N/2} whose length rounds to
// r, counted over (p, q, m) folded to p, q, m >= 0 (whole numbers, exact in
// any order). They depend on n only; the spectrum and the structure
// function of every sample of a call share them.
__global__ void __launch_bounds__(256) shell_count_kernel(int n, double* cnt) {
  __shared__ double sc[256];
  const int col = blockIdx.x, half = n / 2;
  double c = 0.0;
  for (int e = threadIdx.x; e < (half + 1) * (half + 1); e += 256) {
    const int p = e / (half + 1), q = e % (half + 1);
    int lo, hi;
    shell_range(half, p * p + q * q, col, lo, hi);
    c += fold_weight(p, half) * fold_weight(q, half) * range_count(half, lo, hi);
  }
  sc[threadIdx.x] = c;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sc[threadIdx.x] += sc[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) cnt[col] = sc[0];
}

// Stage 2, one block per column: the partials summed over the chunks (thread
// t takes chunks t, t + 256, ..., then a fixed tree), divided by the shell's
// number of vectors cnt[col] (shell_count_kernel). mode 0 (spectrum):
// out[kappa] = 4 pi / count * sum / N^6 for kappa = 0..N/2 (out may be NULL),
// and column N/2 + 1 (the sum of Psi, R_0 times N^6) into *r0. mode 1
// (structure function): out[r - 1] = sum / count / N^6 for r = 1..N/2.
__global__ void __launch_bounds__(256) shell_final_kernel(const double* psum0, const double* cnt, int chunks,
                                                          int width, int n, int mode, double* out0, double* r00,
                                                          size_t wstride) {
  __shared__ double sa[256];
  const double* psum = in_batch(psum0, wstride);
  double* out = out0 ? out0 + size_t(blockIdx.z) * (mode == 0 ? n / 2 + 1 : n / 2) : nullptr;
  double* r0 = r00 ? in_batch(r00, wstride) : nullptr;
  const int col = blockIdx.x, half = n / 2;
  double a = 0.0;
  for (int b = threadIdx.x; b < chunks; b += 256) a += psum[size_t(b) * width + col];
  sa[threadIdx.x] = a;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sa[threadIdx.x] += sa[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double norm = 1.0 / (double(n) * n * n) / (double(n) * n * n);
    const double sum = sa[0], cnt_c = col <= half ? cnt[col] : 0.0;
    if (mode == 0) {
      if (col <= half && out) out[col] = cnt_c > 0 ? 4.0 * M_PI / cnt_c * sum * norm : 0.0;
      if (col == half + 1 && r0) *r0 = sum;
    } else if (col >= 1 && col <= half) {
      out[col - 1] = cnt_c > 0 ? sum * norm / cnt_c : 0.0;
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


struct ObsWork {
  double2* h;       // 3 fields of N * N * NH complex; after pass 3, H
  double* g;        // N (N/2 + 1)^2: the folded z-transform G
  double* sbins;    // spectrum_bin_rows(N) rows of N/2 + 2
  double* rbins;    // sf_bin_rows(N) rows of N/2 + 2
  double* psum;     // one row of N/2 + 2 per chunk of either table
  double* r0;       // 1
  double* cnt;      // N/2 + 1 shell sizes (used in the first sample's area)
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

size_t chunks_of(size_t rows) { return (rows + kShellChunk - 1) / kShellChunk; }

// Byte sizes of the parts of one sample's work area (each a multiple of 256)
struct WorkSizes {
  size_t h, g, sbins, rbins, psum, r0, cnt;
  size_t total() const { return h + g + sbins + rbins + psum + r0 + cnt; }
};

WorkSizes work_sizes(int n) {
  const size_t nh = size_t(n / 2 + 1), width = size_t(n / 2 + 2);
  const size_t srows = spectrum_bin_rows(n), rrows = sf_bin_rows(n);
  WorkSizes z;
  z.h = align256(3 * size_t(n) * n * nh * sizeof(double2));
  z.g = align256(size_t(n) * folded_lines(n) * sizeof(double));
  z.sbins = align256(srows * width * sizeof(double));
  z.rbins = align256(rrows * width * sizeof(double));
  z.psum = align256(chunks_of(std::max(srows, rrows)) * width * sizeof(double));
  z.r0 = align256(sizeof(double));
  z.cnt = align256(width * sizeof(double));
  return z;
}

// bytes of one sample's work area (a multiple of 256)
size_t sample_work_bytes(int n) { return work_sizes(n).total(); }

ObsWork carve(void* work, int n) {
  const WorkSizes z = work_sizes(n);
  char* p = static_cast<char*>(work);
  ObsWork w;
  w.h = reinterpret_cast<double2*>(p);
  w.g = reinterpret_cast<double*>(p += z.h);
  w.sbins = reinterpret_cast<double*>(p += z.g);
  w.rbins = reinterpret_cast<double*>(p += z.sbins);
  w.psum = reinterpret_cast<double*>(p += z.rbins);
  w.r0 = reinterpret_cast<double*>(p += z.psum);
  w.cnt = reinterpret_cast<double*>(p += z.r0);
  return w;
}

template <int QN, typename T, int N, bool FROM_U>
hipError_t observables_t(const T* pop, const double* u, const DevSample* samples, int sample0, int count, int parity,
                         void* work, double* s2, double* ek, hipStream_t s) {
  constexpr int NH = N / 2 + 1, L = half_lines(N);
  constexpr int ROWS_X = fwd_rows(N);
  constexpr int PC = cos_pairs(N);
  constexpr int W = N / 2 + 2;
  static_assert(N % L == 0 && (N * N) % ROWS_X == 0, "launch shapes must tile the field");
  const ObsWork w = carve(work, N);
  const size_t ws = sample_work_bytes(N);
  const unsigned z = unsigned(count);
  const int lines = N * NH;
  const int srows = int(spectrum_bin_rows(N)), rrows = int(sf_bin_rows(N));
  const int lchunks = int(chunks_of(srows)), rchunks = int(chunks_of(rrows));
  hipLaunchKernelGGL((fwd_x_kernel<QN, T, N, FROM_U>), dim3(N * N / ROWS_X, 1, z), dim3(256), 0, s, pop, u, samples,
                     sample0, parity, w.h, ws);
  hipLaunchKernelGGL((fft_y_kernel<N, L>), dim3(lines / L, 3, z), dim3(256), 0, s, w.h, -1, ws);
  constexpr int LZ = z_lines(N);
  hipLaunchKernelGGL((z_psd_kernel<N, LZ>), dim3(lines / LZ, 1, z), dim3(256), 0, s, w.h, w.g, w.sbins, ws);
  hipLaunchKernelGGL(shell_partial_kernel, dim3(lchunks, 1, z), dim3(256), 0, s, w.sbins, srows, W, w.psum, ws);
  hipLaunchKernelGGL(shell_count_kernel, dim3(NH), dim3(256), 0, s, N, w.cnt);
  hipLaunchKernelGGL(shell_final_kernel, dim3(W, 1, z), dim3(256), 0, s, w.psum, w.cnt, lchunks, W, N, 0, ek, w.r0,
                     ws);
  if (s2) {
    double* hr = reinterpret_cast<double*>(w.h);
    hipLaunchKernelGGL((cos_y_kernel<N, PC>), dim3(rrows, 1, z), dim3(256), 0, s, w.g, hr, ws);
    hipLaunchKernelGGL((cos_x_kernel<N, PC>), dim3(rrows, 1, z), dim3(256), 0, s, hr, w.r0, w.rbins, ws);
    hipLaunchKernelGGL(shell_partial_kernel, dim3(rchunks, 1, z), dim3(256), 0, s, w.rbins, rrows, W, w.psum, ws);
    hipLaunchKernelGGL(shell_final_kernel, dim3(W, 1, z), dim3(256), 0, s, w.psum, w.cnt, rchunks, W, N, 1, s2,
                       nullptr, ws);
  }
  return hipGetLastError();
}

template <int QN, typename T, bool FROM_U>
hipError_t observables_n(int n, const void* pop, const double* u, const DevSample* samples, int sample0, int count,
                         int parity, void* work, double* s2, double* ek, hipStream_t s) {
  const T* p = static_cast<const T*>(pop);
  switch (n) {
    case 8: return observables_t<QN, T, 8, FROM_U>(p, u, samples, sample0, count, parity, work, s2, ek, s);
    case 16: return observables_t<QN, T, 16, FROM_U>(p, u, samples, sample0, count, parity, work, s2, ek, s);
    case 32: return observables_t<QN, T, 32, FROM_U>(p, u, samples, sample0, count, parity, work, s2, ek, s);
    case 64: return observables_t<QN, T, 64, FROM_U>(p, u, samples, sample0, count, parity, work, s2, ek, s);
    case 128: return observables_t<QN, T, 128, FROM_U>(p, u, samples, sample0, count, parity, work, s2, ek, s);
    case 256: return observables_t<QN, T, 256, FROM_U>(p, u, samples, sample0, count, parity, work, s2, ek, s);
    case 512: return observables_t<QN, T, 512, FROM_U>(p, u, samples, sample0, count, parity, work, s2, ek, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

size_t observables_work_bytes(int n, int count) { return sample_work_bytes(n) * size_t(count); }

hipError_t launch_observables(int q, int precision, const void* pop, const DevSample* samples, int32_t sample0,
                              int32_t count, int32_t n, int32_t parity, void* work, double* s2, double* ek,
                              hipStream_t s) {
  if (q == 27) {
    return precision == 0
               ? observables_n<27, double, false>(n, pop, nullptr, samples, sample0, count, parity, work, s2, ek, s)
               : observables_n<27, float, false>(n, pop, nullptr, samples, sample0, count, parity, work, s2, ek, s);
  }
  if (q == 19) {
    return precision == 0
               ? observables_n<19, double, false>(n, pop, nullptr, samples, sample0, count, parity, work, s2, ek, s)
               : observables_n<19, float, false>(n, pop, nullptr, samples, sample0, count, parity, work, s2, ek, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_observables_velocity(const double* u, const DevSample* samples, int32_t sample0, int32_t count,
                                       int32_t n, void* work, double* s2, double* ek, hipStream_t s) {
  return observables_n<27, double, true>(n, nullptr, u, samples, sample0, count, 0, work, s2, ek, s);
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

// Device scratch of the sample error for callers that cannot allocate: the
// per-sample ratios, 4 doubles per sample. Each GPU holds its own copy for the
// life of the process; its address is looked up once per device
// (hipGetSymbolAddress with that device current) and kept, and kernels
// receive that address, never the array's name, which in host code is only
// a stand-in.
static __device__ __align__(256) double scratch[4 * kNoAllocMaxSamples];

static std::mutex g_scratch_mutex;
static std::vector<double*> g_scratch_ptr;  // per device; nullptr until looked up

hipError_t sample_error_scratch(double** ratio) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (size_t(dev) >= g_scratch_ptr.size()) g_scratch_ptr.resize(size_t(dev) + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *ratio = g_scratch_ptr[dev];
  return hipSuccess;
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
