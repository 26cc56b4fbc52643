// Lattice constants and the per-sample / per-launch tables shared by the
// kernels and the host side of the library.
//
// Velocities are numbered in the D3Q27 order everywhere in the kernels:
// c_i in {-1,0,1}^3 with i = 9*(cx+1) + 3*(cy+1) + (cz+1); the opposite
// velocity is 26 - i. Two lattices are built on it (c_s^2 = 1/3 for both,
// with the equilibrium of eq. (equilibrium)):
//   D3Q27 (QN = 27): all 27 velocities; weights are the tensor product of the
//     1-D weights (1/6, 2/3, 1/6), i.e. 8/27 (rest), 2/27 (6 axis
//     velocities), 1/54 (12 diagonals), 1/216 (8 corners);
//   D3Q19 (QN = 19), the paper's lattice (section on the deterministic
//     scheme): the 19 velocities without the corners, weights 1/3 (rest),
//     1/18 (axis), 1/36 (diagonals).
// A lattice stores its populations in QN planes; plane_of<QN>(i) is the plane
// of velocity i (its rank among the lattice's velocities), so the opposite of
// plane k is plane QN - 1 - k.
#pragma once

#include <cstdint>

namespace mclbm {

constexpr int Q = 27;  // size of the velocity numbering (register arrays are indexed by it)
constexpr int kMaxSamples = 65536;  // samples per ensemble (tables are sized by m)

__host__ __device__ constexpr int cx(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int cy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int opposite(int i) { return 26 - i; }
__host__ __device__ constexpr int nonzeros(int i) { return (cx(i) != 0) + (cy(i) != 0) + (cz(i) != 0); }

template <int QN>
__host__ __device__ constexpr bool in_lattice(int i) {
  static_assert(QN == 27 || QN == 19, "D3Q27 or D3Q19");
  return QN == 27 || nonzeros(i) < 3;
}

template <int QN>
__host__ __device__ constexpr double weight(int i) {
  if constexpr (QN == 27)
    return nonzeros(i) == 0 ? 8.0 / 27.0 : nonzeros(i) == 1 ? 2.0 / 27.0 : nonzeros(i) == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
  else
    return nonzeros(i) == 0 ? 1.0 / 3.0 : nonzeros(i) == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
}

// storage plane of velocity i: the number of the lattice's velocities before it
template <int QN>
__host__ __device__ constexpr int plane_of(int i) {
  if constexpr (QN == 27) {
    return i;
  } else {
    // corners (nonzeros == 3) sit at 0, 2, 6, 8, 18, 20, 24, 26
    return i - ((i > 0) + (i > 2) + (i > 6) + (i > 8) + (i > 18) + (i > 20) + (i > 24));
  }
}

// velocity of storage plane k (inverse of plane_of; run time)
template <int QN>
__host__ __device__ inline int velocity_of_plane(int k) {
  int seen = 0;
  for (int i = 0; i < Q; ++i) {
    if (!in_lattice<QN>(i)) continue;
    if (seen == k) return i;
    ++seen;
  }
  return -1;
}

// Per-sample table in device memory.
struct DevSample {
  uint64_t offset;        // element offset of population plane 0 of this sample
  int32_t n;              // points per axis
  int32_t log2n;
  uint32_t pstride;       // elements from one population plane to the next (n^3 + padding)
  uint32_t pad_u32;
  double omega;           // shear relaxation frequency
  double two_over_omega;  // 2 / omega
  double kappa;           // 2 - 2 / omega
  double eps;             // 2 - omega (carries the viscosity: nu = eps / (6 - 3 eps))
  float omega_f, two_over_omega_f, kappa_f, eps_f;
  int32_t project;        // 1: the perturbation coefficients were Leray-projected
  double u0;              // Taylor-Green amplitude
  double amp;             // perturbation amplitude relative to u0
  uint64_t voffset;       // double offset of this sample's captured velocity (three planes of n^3)
};

// One run of consecutive blocks of a launch that belong to one sample.
struct Seg {
  int32_t sample;
  int32_t first_block;
  int32_t nblocks;
  int32_t parity;         // steps taken so far, modulo 2 (AA layout of the state)
};

// Reduction record layout (doubles per sample).
constexpr int kRecord = 8;  // mass, jx, jy, jz, ke, gamma_min, gamma_max, gamma_mean

}  // namespace mclbm
