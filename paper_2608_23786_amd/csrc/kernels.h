// Launch interface between the host side of the library and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lattice.h"

namespace mclbm {

// One collide-and-stream launch over the blocks described by `segs`.
struct StepLaunch {
  void* pop;                 // population storage (AA in place), or the source in push mode
  void* dst;                 // push mode: destination storage (natural layout)
  const DevSample* samples;
  const Seg* segs;
  int32_t nseg;
  int32_t total_blocks;
  int32_t block;             // threads per block (cells per block)
  int32_t xcd_remap;
  int32_t* flags;            // per-sample instability flags
  double* partials;          // record mode: kRecord doubles per block
  int32_t buffer_ok;         // buffer-resource addressing (every sample's populations span < 2 GiB)
  int32_t nontemporal;       // non-temporal loads and stores of the populations
  int32_t exact_gamma;       // 1: exact minimiser of the H-function (block 256 only)
  double* vel;               // record mode: velocity capture (DevSample::voffset), or NULL
};

enum StepKind { kStep = 0, kStepRecord = 1, kReduceOnly = 2, kPush = 3 };

// Lattice-dependent launches take the lattice q (27: D3Q27, 19: D3Q19) and the
// precision (0: double, 1: float shifted populations).
hipError_t launch_step(int q, int precision, StepKind kind, const StepLaunch& L, hipStream_t s);
// per lattice and precision (step_d3q27_f32.hip, ...)
hipError_t launch_step_d3q27_f32(StepKind kind, const StepLaunch& L, hipStream_t s);
hipError_t launch_step_d3q27_f64(StepKind kind, const StepLaunch& L, hipStream_t s);
hipError_t launch_step_d3q19_f32(StepKind kind, const StepLaunch& L, hipStream_t s);
hipError_t launch_step_d3q19_f64(StepKind kind, const StepLaunch& L, hipStream_t s);

// Records from block partials: one block per segment, writes out[sample*kRecord + k].
hipError_t launch_record_finalize(const double* partials, const Seg* segs, int32_t nseg, const DevSample* samples,
                                  double* out, hipStream_t s);

// Initial equilibrium populations of every sample in `segs` (blocks of 256 cells).
hipError_t launch_init(int q, int precision, void* pop, const DevSample* samples, const Seg* segs, int32_t nseg,
                       int32_t total_blocks, const double* ycoef, hipStream_t s);

// Density and velocity (double) of one sample; parity selects the AA layout.
hipError_t launch_moments(int q, int precision, const void* pop, const DevSample* samples, int32_t sample,
                          int32_t n, int32_t parity, double* rho, double* u, hipStream_t s);

// Unshifted populations f[q][n^3] in double, out of or into the state.
hipError_t launch_get_state(int q, int precision, const void* pop, const DevSample* samples, int32_t sample,
                            int32_t n, int32_t parity, double* f, hipStream_t s);
hipError_t launch_set_state(int q, int precision, void* pop, const DevSample* samples, int32_t sample, int32_t n,
                            int32_t parity, const double* f, hipStream_t s);
hipError_t launch_gather_cells(int q, int precision, const void* pop, const DevSample* samples, int32_t sample,
                               int32_t parity, const int64_t* cells, int32_t count, double* f, hipStream_t s);
// k: storage plane (population index in the lattice's own numbering)
hipError_t launch_poison(int q, int precision, void* pop, const DevSample* samples, int32_t sample, int32_t parity,
                         int64_t cell, int32_t k, hipStream_t s);

// Copy the state of every sample in `segs` into natural layout at dst (same offsets).
hipError_t launch_canonical_copy(int q, int precision, const void* pop, void* dst, const DevSample* samples,
                                 const Seg* segs, int32_t nseg, int32_t total_blocks, hipStream_t s);

// Adjoint vectors of one sample, lam[q][n^3] in double, into or out of the
// natural layout (no weight shift) of a buffer with the state's offsets.
hipError_t launch_put_adjoint(int q, int precision, void* dst, const DevSample* samples, int32_t sample, int32_t n,
                              const double* lam, hipStream_t s);
hipError_t launch_get_adjoint(int q, int precision, const void* src, const DevSample* samples, int32_t sample,
                              int32_t n, double* lam, hipStream_t s);

// Adjoint: seed lambda_T from the state (parity-aware), one reverse step, and the
// initial-data adjoint with its per-sample projection onto the 24 parameters.
hipError_t launch_adjoint_seed(int q, int precision, const void* pop, void* lam, const DevSample* samples,
                               const Seg* segs, int32_t nseg, int32_t total_blocks, double inv_m, hipStream_t s);
hipError_t launch_adjoint_step(int q, int precision, const void* state, const void* lam_in, void* lam_out,
                               const DevSample* samples, const Seg* segs, int32_t nseg, int32_t total_blocks,
                               int32_t buffer_ok, int32_t exact_gamma, hipStream_t s);
hipError_t launch_init_adjoint(int q, int precision, const void* lam, const DevSample* samples, const Seg* segs,
                               int32_t nseg, int32_t total_blocks, const double* ycoef, double* partials,
                               hipStream_t s);
hipError_t launch_init_adjoint_finalize(const double* partials, const Seg* segs, int32_t nseg,
                                        const DevSample* samples, const double* pmat, double* dJdY,
                                        hipStream_t s);
hipError_t launch_extract(const double* records, int32_t m, int32_t field, double* out, hipStream_t s);

// Per-sample constants of the dissipation rate (a small device table).
struct DissSample {
  double inv_u0sq;  // 1 / u0^2: KE in units of u0^2
  double dt;        // physical time of one step, (2 pi / n) * u0
  int64_t stride;   // ticks per step
};
hipError_t launch_dissipation(const double* records, const DissSample* smp, int32_t m, int32_t nrec,
                              int64_t first_tick, int32_t record_every, double eps, double* diss, double* eta,
                              hipStream_t s);
// The same from the spectra ek[nrec][count][n/2+1] of `count` samples of one
// resolution (smp points at the first of them): E = sum over kappa.
hipError_t launch_dissipation_spectra(const double* ek, int32_t n, const DissSample* smp, int32_t count,
                                      int32_t nrec, int64_t first_tick, int32_t record_every, double eps,
                                      double* diss, double* eta, hipStream_t s);

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

// Observables (observables.hip) of `count` consecutive samples sample0.. that
// share n and AA parity, in one set of launches: structure functions
// s2[count][n/2] (r = 1..n/2) and energy spectra ek[count][n/2+1]
// (kappa = 0..n/2), either may be NULL; work: observables_work_bytes(n,
// count) bytes, 256-byte aligned.
size_t observables_work_bytes(int n, int count);
hipError_t launch_observables(int q, int precision, const void* pop, const DevSample* samples, int32_t sample0,
                              int32_t count, int32_t n, int32_t parity, void* work, double* s2, double* ek,
                              hipStream_t s);
// The same observables from captured velocities (u: the capture buffer, each
// sample's three planes at its voffset).
hipError_t launch_observables_velocity(const double* u, const DevSample* samples, int32_t sample0, int32_t count,
                                       int32_t n, void* work, double* s2, double* ek, hipStream_t s);
// lattice: 27 or 19; q: common nodes per axis
hipError_t launch_point_values(int lattice, int precision, const void* pop, const DevSample* samples,
                               const Seg* segs, int32_t nseg, int q, int physical, double* out, hipStream_t s);
hipError_t launch_w1(const double* a, const double* b, int m, int q, double* col, double* out, hipStream_t s);
hipError_t launch_ensemble_moments(const double* x, int m, int k, int64_t ld, double* mean, double* sd,
                                   hipStream_t s);
hipError_t launch_compensate(const DevSample* samples, int sample0, int count, int n, const double* d,
                             const double* s2, const double* ek, double* s2c, double* ekc, hipStream_t s);
hipError_t launch_sample_error(const double* a, const double* b, int m, int q, double* ratio, double* out,
                               hipStream_t s);
// The sample error's per-sample ratios without a caller's buffer: a device
// array of the library (4 doubles per sample, at most kNoAllocMaxSamples
// samples) whose address on the current device is looked up once per device.
constexpr int kNoAllocMaxSamples = 65536;
hipError_t sample_error_scratch(double** ratio);

}  // namespace mclbm
