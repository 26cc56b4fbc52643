// The fused collide-and-stream kernel and its launch shapes. Each
// (lattice, precision) pair is instantiated in a translation unit of its
// own (step_d3q27_f32.hip, ...), which keeps the compile of the
// library parallel.
#pragma once

#include "lbm_device.h"

namespace mclbm {
namespace {

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
  double* vel;  // record ticks: the velocity of the state read, per sample at voffset (NULL: none)
};

template <int QN, typename T, int BLOCK, StepKind KIND, bool BUF, bool NT, bool EXACT = false>
__global__ void __launch_bounds__(BLOCK) kbc_step_kernel(StepArgs<T> a) {
  const int b = remap_block(blockIdx.x, a.total_blocks, a.xcd_remap);
  const Seg sg = a.segs[find_segment(a.segs, a.nseg, b)];
  const DevSample& sp = a.samples[sg.sample];
  const int l = sp.log2n;
  const Cell c = make_cell(uint32_t(b - sg.first_block) * BLOCK + threadIdx.x, l);
  using Planes = typename std::conditional<BUF, BufPlanes<T, NT, QN>, PtrPlanes<T, NT, QN>>::type;
  const Planes src(a.pop + sp.offset, sp.pstride);
  const bool odd = (KIND != kPush) && (sg.parity & 1);

  // rows longer than a wave, held whole by the block: x-shifts by lane exchange
  const uint32_t n = 1u << l;
  const bool rows = n > 64u && n <= uint32_t(BLOCK);
  __shared__ EdgeLds<T, BLOCK> edge_in, edge_out;

  T g[Q];
  if (!odd) {
    for_vel<QN>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const Slot s = aa_read_slot<i>(c, false);
      g[i] = src.load(s.vel, s.idx);
    });
  } else if (rows) {
    for_vel<QN>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      g[i] = src.load(opposite(i), neighbour_yz<i, -1>(c));
    });
    row_shift<QN, +1, BLOCK>(g, edge_in, n);
  } else {
    for_vel<QN>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      const Slot s = aa_read_slot<i>(c, true);
      g[i] = src.load(s.vel, s.idx);
    });
  }
  if constexpr (KIND == kStepRecord) {
    if (a.vel) {
      double ux, uy, uz;
      node_velocity<QN>(g, ux, uy, uz);
      double* u = a.vel + sp.voffset;
      const size_t plane = size_t(n) * n * n;
      __builtin_nontemporal_store(ux, u + c.cell);
      __builtin_nontemporal_store(uy, u + plane + c.cell);
      __builtin_nontemporal_store(uz, u + 2 * plane + c.cell);
    }
  }
  const CellResult<T> res = kbc_collide<QN, EXACT>(g, relax_of<T>(sp));
  if (res.bad) a.flags[sg.sample] = 1;

  if constexpr (KIND == kStep || KIND == kStepRecord || KIND == kPush) {
    const bool pushes = KIND == kPush || odd;
    T* const out = KIND == kPush ? a.dst : a.pop;
    const Planes dst(out + sp.offset, sp.pstride);
    if (!pushes) {
      for_vel<QN>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const Slot s = aa_write_slot<i>(c, false);
        dst.store(s.vel, s.idx, g[i]);
      });
    } else if (rows) {
      row_shift<QN, +1, BLOCK>(g, edge_out, n);
      for_vel<QN>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        dst.store(i, neighbour_yz<i, +1>(c), g[i]);
      });
    } else {
      for_vel<QN>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const Slot s = aa_write_slot<i>(c, true);
        dst.store(s.vel, s.idx, g[i]);
      });
    }
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

template <int QN, typename T, int BLOCK, StepKind KIND>
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
  a.vel = L.vel;
  const dim3 grid(L.total_blocks), blk(BLOCK);
  if (buf && L.nontemporal)
    hipLaunchKernelGGL((kbc_step_kernel<QN, T, BLOCK, KIND, true, true>), grid, blk, 0, s, a);
  else if (buf)
    hipLaunchKernelGGL((kbc_step_kernel<QN, T, BLOCK, KIND, true, false>), grid, blk, 0, s, a);
  else if (L.nontemporal)
    hipLaunchKernelGGL((kbc_step_kernel<QN, T, BLOCK, KIND, false, true>), grid, blk, 0, s, a);
  else
    hipLaunchKernelGGL((kbc_step_kernel<QN, T, BLOCK, KIND, false, false>), grid, blk, 0, s, a);
  return hipGetLastError();
}

template <int QN, typename T, StepKind KIND>
hipError_t launch_step_b(const StepLaunch& L, hipStream_t s) {
  switch (L.block) {
    case 128: return launch_step_t<QN, T, 128, KIND>(L, s);
    case 256: return launch_step_t<QN, T, 256, KIND>(L, s);
    case 512: return launch_step_t<QN, T, 512, KIND>(L, s);
    case 1024:
      if constexpr (std::is_same<T, float>::value) return launch_step_t<QN, T, 1024, KIND>(L, s);
      else return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// The exact stabiliser (eq. (kbc_entropy)) is compiled for one launch shape:
// 256 threads, non-temporal access, either addressing.
template <int QN, typename T, StepKind KIND>
hipError_t launch_step_exact(const StepLaunch& L, hipStream_t s) {
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
  a.vel = L.vel;
  if (L.block != 256) return hipErrorInvalidValue;
  if (L.buffer_ok)
    hipLaunchKernelGGL((kbc_step_kernel<QN, T, 256, KIND, true, true, true>), dim3(L.total_blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((kbc_step_kernel<QN, T, 256, KIND, false, true, true>), dim3(L.total_blocks), dim3(256), 0, s,
                       a);
  return hipGetLastError();
}

template <int QN, typename T>
hipError_t launch_step_k(StepKind kind, const StepLaunch& L, hipStream_t s) {
  if (L.exact_gamma) {
    switch (kind) {
      case kStep: return launch_step_exact<QN, T, kStep>(L, s);
      case kStepRecord: return launch_step_exact<QN, T, kStepRecord>(L, s);
      case kReduceOnly: return launch_step_exact<QN, T, kReduceOnly>(L, s);
      case kPush: return launch_step_exact<QN, T, kPush>(L, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (kind) {
    case kStep: return launch_step_b<QN, T, kStep>(L, s);
    case kStepRecord: return launch_step_b<QN, T, kStepRecord>(L, s);
    case kReduceOnly: return launch_step_b<QN, T, kReduceOnly>(L, s);
    case kPush: return launch_step_b<QN, T, kPush>(L, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace
}  // namespace mclbm
