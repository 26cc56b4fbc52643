// Host side of the C ABI declared in include/mclbm.h: context, workspace
// layout, tick scheduling of mixed-resolution ensembles, HIP graph capture,
// launch-shape autotuning, checkpoints and the adjoint driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/mclbm.h"
#include "kernels.h"
#include "lattice.h"

using namespace mclbm;

namespace {

thread_local std::string g_last_error;

mclbm_status fail(mclbm_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HIP_TRY(expr)                                                                                \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess)                                                                            \
      return fail(MCLBM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));                \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}
bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

constexpr int kMinBlock = 128;        // smallest collide-and-stream block
constexpr int kAuxBlock = 256;        // block of the auxiliary kernels
constexpr int kMaxTables = 128;       // launch tables kept in the workspace
constexpr size_t kHeaderBytes = 4096; // checkpoint header
constexpr uint64_t kCkptMagic = 0x4d434c424d434b50ull;
constexpr size_t kFwdHeaderBytes = 256;  // forward checkpoints: the token of the forward that wrote them
std::atomic<uint64_t> g_fwd_tokens{0};
constexpr int kMaxObservablesN = 512;  // the FFT passes are instantiated for n = 8..512

// Leray projection on the 24 perturbation coefficients.
// Every basis field a_i(2x) a_j(2y) a_k(2z) e_alpha is a Laplacian eigenfunction
// (eigenvalue -12), so P s = s + grad(div s) / 12 exactly, and grad div maps the
// family into itself: d/dx a_0(2x) = 2 a_1(2x), d/dx a_1(2x) = -2 a_0(2x).
// Returns P[24][24] with Y' = P Y.
std::vector<double> projection_matrix() {
  std::vector<double> P(24 * 24, 0.0);
  for (int p = 0; p < 24; ++p) {
    const int al = p / 8;
    const int idx[3] = {(p >> 2) & 1, (p >> 1) & 1, p & 1};
    for (int be = 0; be < 3; ++be) {
      int out[3] = {idx[0], idx[1], idx[2]};
      double coef;
      if (be == al) {
        coef = 1.0 - 4.0 / 12.0;  // s_alpha + d^2/dx_alpha^2 s_alpha / 12
      } else {
        const double sa = idx[al] == 0 ? 2.0 : -2.0;
        const double sb = idx[be] == 0 ? 2.0 : -2.0;
        out[al] = 1 - idx[al];
        out[be] = 1 - idx[be];
        coef = sa * sb / 12.0;
      }
      const int q = 8 * be + 4 * out[0] + 2 * out[1] + out[2];
      P[q * 24 + p] += coef;
    }
  }
  return P;
}

struct Table {
  size_t offset = 0;         // byte offset of the Seg array in the table pool
  int nseg = 0;
  int total_blocks = 0;
  std::vector<Seg> host;     // persistent host copy (source of the upload)
};

}  // namespace

struct mclbm_ctx {
  int m = 0;
  int precision = 0;
  int q = 27;                // velocities of the lattice (27 or 19)
  size_t elem = 8;
  std::vector<mclbm_sample_desc> desc;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;

  // workspace carve
  DevSample* d_samples = nullptr;
  int32_t* d_flags = nullptr;
  double* d_ycoef = nullptr;
  double* d_pmat = nullptr;
  DissSample* d_diss = nullptr;
  Seg* d_tables = nullptr;
  size_t table_pool_bytes = 0;
  double* d_partials = nullptr;
  size_t partial_blocks = 0;
  double* d_vel = nullptr;    // velocity capture of the record ticks (the caller's buffer), or NULL
  size_t vel_doubles = 0;     // 3 sum n^3: the capture buffer's length
  char* pop = nullptr;
  size_t state_bytes = 0;

  std::vector<DevSample> h_samples;
  std::vector<double> y;     // drawn or given parameters, m x 24
  std::vector<double> pmat;
  bool initialized = false;
  // bumped by every call that changes the state or its dynamics; a backward
  // sweep needs the state its forward_ckpt left (fwd_generation) and the
  // checkpoints that forward wrote (fwd_token, also in their header)
  uint64_t generation = 0;
  uint64_t fwd_generation = 0;
  uint64_t fwd_token = 0;
  int64_t tick = 0;
  std::vector<int64_t> steps;
  int max_stride = 1;

  // launch shape
  int block = 256;
  int xcd_remap = 0;
  int buffer_addr = 1;       // buffer-resource addressing where every sample fits
  int nontemporal = 1;       // non-temporal population loads and stores
  int exact_gamma = 0;       // 1: exact entropic stabiliser (256-thread blocks)

  // launch tables by key
  std::map<std::string, Table> tables;
  size_t table_next = 0;

  // graphs keyed by the tick phase
  bool use_graphs = true;
  std::map<int64_t, hipGraphExec_t> graphs;
  int64_t graph_ticks = 0;

  // launch timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;

  std::vector<char> ckpt_header;

  int64_t cells(int s) const { return int64_t(desc[s].n) * desc[s].n * desc[s].n; }
};

namespace {

void drop_graphs(mclbm_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

mclbm_status validate_desc(int32_t m, const mclbm_sample_desc* d, int32_t precision, int32_t lattice) {
  if (m < 1 || m > kMaxSamples) return fail(MCLBM_ERR_ARG, "m must be in [1, " + std::to_string(kMaxSamples) + "]");
  if (!d) return fail(MCLBM_ERR_ARG, "descriptor array is NULL");
  if (precision != MCLBM_FP64 && precision != MCLBM_FP32_SHIFTED) return fail(MCLBM_ERR_ARG, "unknown precision");
  if (lattice != MCLBM_D3Q27 && lattice != MCLBM_D3Q19) return fail(MCLBM_ERR_ARG, "lattice must be 27 or 19");
  for (int s = 0; s < m; ++s) {
    const mclbm_sample_desc& e = d[s];
    const int nmax = precision == MCLBM_FP64 ? 512 : 1024;
    if (!is_pow2(e.n) || e.n < 8 || e.n > nmax)
      return fail(MCLBM_ERR_ARG, "sample " + std::to_string(s) + ": n must be a power of two in [8, " +
                                     std::to_string(nmax) + "]");
    if (!(e.u0 > 0.0) || !(e.u0 <= 0.2)) return fail(MCLBM_ERR_ARG, "sample " + std::to_string(s) + ": u0 out of (0, 0.2]");
    if (!(e.re > 0.0) || !std::isfinite(e.re)) return fail(MCLBM_ERR_ARG, "sample " + std::to_string(s) + ": re must be > 0");
    if (!(e.amp >= 0.0) || !std::isfinite(e.amp)) return fail(MCLBM_ERR_ARG, "sample " + std::to_string(s) + ": amp must be >= 0");
    if (e.project != 0 && e.project != 1) return fail(MCLBM_ERR_ARG, "sample " + std::to_string(s) + ": project must be 0 or 1");
    if (!is_pow2(e.stride) || e.stride > 1024)
      return fail(MCLBM_ERR_ARG, "sample " + std::to_string(s) + ": stride must be a power of two <= 1024");
  }
  return MCLBM_OK;
}

// Pad after each population plane, by plane size. The q streams of a wave
// start at the same offset in q planes; how they spread over the HBM
// channels depends on the plane stride, and the best pad differs by size
// (measured with the FP32 collide-and-stream kernel on 64 x 64^3, 8 x 128^3,
// 4 x 256^3 and 1 x 512^3 for pads of 0 to 64 KiB: up to 18 % apart; the
// pads below beat 4352 bytes by 0.5 to 2 %). Other sizes take 4352 bytes
// (17 x 256), the best single choice across the four.
uint32_t plane_pad_bytes(uint64_t plane_bytes) {
  if (plane_bytes < (uint64_t(1) << 16)) return 0;
  switch (plane_bytes) {
    case uint64_t(1) << 20: return 256;    // 64^3 float
    case uint64_t(8) << 20: return 1024;   // 128^3 float
    case uint64_t(64) << 20: return 0;     // 256^3 float
    case uint64_t(512) << 20: return 1024; // 512^3 float
    default: return 4352;
  }
}

// Elements from one population plane to the next: n^3 plus the pad.
uint64_t plane_stride(int n, size_t elem) {
  const uint64_t n3 = uint64_t(n) * n * n;
  return n3 + plane_pad_bytes(n3 * elem) / elem;
}

struct Layout {
  size_t samples, flags, ycoef, pmat, diss, tables, table_bytes, partials, partial_blocks, pop, state_bytes, total;
};

Layout layout_of(int32_t m, const mclbm_sample_desc* d, int32_t precision, int32_t lattice) {
  Layout L{};
  const size_t elem = precision == MCLBM_FP64 ? 8 : 4;
  size_t off = 0;
  L.samples = off;
  off = align_up(off + sizeof(DevSample) * size_t(m));
  L.flags = off;
  off = align_up(off + sizeof(int32_t) * size_t(m));
  L.ycoef = off;
  off = align_up(off + sizeof(double) * 24 * size_t(m));
  L.pmat = off;
  off = align_up(off + sizeof(double) * 24 * 24);
  L.diss = off;
  off = align_up(off + sizeof(DissSample) * size_t(m));
  L.tables = off;
  L.table_bytes = size_t(kMaxTables) * align_up(sizeof(Seg) * m);
  off = align_up(off + L.table_bytes);
  size_t cells = 0;
  for (int s = 0; s < m; ++s) cells += size_t(d[s].n) * d[s].n * d[s].n;
  L.partial_blocks = cells / kMinBlock;
  L.partials = off;
  off = align_up(off + L.partial_blocks * kRecord * sizeof(double));
  L.pop = off;
  size_t st = 0;
  for (int s = 0; s < m; ++s) st = align_up(st + size_t(lattice) * plane_stride(d[s].n, elem) * elem);
  L.state_bytes = st;
  off += st;
  L.total = off;
  return L;
}

double omega_of(double nu);

void fill_sample(mclbm_ctx* c, int s, double nu) {
  DevSample& h = c->h_samples[s];
  const double omega = omega_of(nu);
  h.omega = omega;
  h.two_over_omega = 2.0 / omega;
  h.kappa = 2.0 - 2.0 / omega;
  h.eps = 6.0 * nu / (3.0 * nu + 0.5);  // 2 - omega = 2 - 1/(3 nu + 1/2) without cancellation
  h.omega_f = float(h.omega);
  h.eps_f = float(h.eps);
  h.two_over_omega_f = float(h.two_over_omega);
  h.kappa_f = float(h.kappa);
}

// Re = u0 L / nu with L = n / (2 pi) lattice units (the box is 2 pi reference lengths)
double lattice_nu(int32_t n, double u0, double re) { return u0 * (double(n) / (2.0 * M_PI)) / re; }
double lattice_nu(const mclbm_sample_desc& d) { return lattice_nu(d.n, d.u0, d.re); }
double omega_of(double nu) { return 1.0 / (3.0 * nu + 0.5); }  // Table 1: 2 c_s^2 / (2 nu + c_s^2), c_s^2 = 1/3

// Recycle the table pool unless `count` more tables fit: tables fetched after
// this call stay valid together (a full pool is cleared, after the stream has
// drained, only inside get_table or here).
mclbm_status reserve_tables(mclbm_ctx* c, int count) {
  const size_t slot = align_up(sizeof(Seg) * c->m);
  if (c->table_next + size_t(count) * slot > c->table_pool_bytes) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    drop_graphs(c);
    c->tables.clear();
    c->table_next = 0;
  }
  return MCLBM_OK;
}

// Launch table for the samples active at `tick` (stride divides tick), with
// their AA parities; `all` forces every sample (init, reductions, adjoint).
// The pointer stays valid until the pool is recycled: a caller that holds
// several tables at once reserves room for them first (reserve_tables).
mclbm_status get_table(mclbm_ctx* c, int64_t tick, bool all, int block, bool parity_zero, const Table** out) {
  std::string key = std::to_string(block) + (all ? "A" : "T") + (parity_zero ? "0" : "P") + ":";
  std::vector<Seg> segs;
  int first = 0;
  for (int s = 0; s < c->m; ++s) {
    const bool active = all || (tick % c->desc[s].stride == 0);
    if (!active) continue;
    Seg g;
    g.sample = s;
    g.first_block = first;
    g.nblocks = int32_t(c->cells(s) / block);
    g.parity = parity_zero ? 0 : int32_t(c->steps[s] & 1);
    first += g.nblocks;
    segs.push_back(g);
    key += std::to_string(s) + (g.parity ? "o" : "e") + ",";
  }
  auto it = c->tables.find(key);
  if (it != c->tables.end()) {
    *out = &it->second;
    return MCLBM_OK;
  }
  // pool full: wait until no launch reads a table, then start over
  mclbm_status st = reserve_tables(c, 1);
  if (st != MCLBM_OK) return st;
  const size_t slot = align_up(sizeof(Seg) * c->m);
  Table t;
  t.offset = c->table_next;
  t.nseg = int(segs.size());
  t.total_blocks = first;
  t.host = segs;
  c->table_next += slot;
  if (!segs.empty()) {
    HIP_TRY(hipMemcpy(reinterpret_cast<char*>(c->d_tables) + t.offset, t.host.data(), sizeof(Seg) * segs.size(),
                      hipMemcpyHostToDevice));
  }
  auto res = c->tables.emplace(key, std::move(t));
  *out = &res.first->second;
  return MCLBM_OK;
}

const Seg* table_ptr(mclbm_ctx* c, const Table* t) {
  return reinterpret_cast<const Seg*>(reinterpret_cast<const char*>(c->d_tables) + t->offset);
}

StepLaunch make_launch(mclbm_ctx* c, const Table* t, void* pop, void* dst) {
  StepLaunch L;
  L.pop = pop;
  L.dst = dst;
  L.samples = c->d_samples;
  L.segs = table_ptr(c, t);
  L.nseg = t->nseg;
  L.total_blocks = t->total_blocks;
  L.block = c->block;
  L.xcd_remap = c->xcd_remap;
  L.flags = c->d_flags;
  L.partials = c->d_partials;
  L.buffer_ok = c->buffer_addr;
  L.nontemporal = c->nontemporal;
  L.exact_gamma = c->exact_gamma;
  L.vel = c->d_vel;
  for (int s = 0; s < c->m; ++s)
    if (uint64_t(c->q) * c->h_samples[s].pstride * c->elem >= (uint64_t(1) << 31)) L.buffer_ok = 0;
  return L;
}

hipEvent_t next_event(mclbm_ctx* c) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->ev_pool.push_back(e);
  }
  return c->ev_pool[c->ev_used++];
}

// One tick: every active sample takes one step; optionally fused reductions.
mclbm_status run_tick(mclbm_ctx* c, double* record_out) {
  const Table* t = nullptr;
  mclbm_status st = get_table(c, c->tick, false, c->block, false, &t);
  if (st != MCLBM_OK) return st;
  if (t->nseg > 0) {
    StepLaunch L = make_launch(c, t, c->pop, nullptr);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
      e0 = next_event(c);
      e1 = next_event(c);
      if (!e0 || !e1) return fail(MCLBM_ERR_HIP, "hipEventCreate failed");
      HIP_TRY(hipEventRecord(e0, c->stream));
    }
    HIP_TRY(launch_step(c->q, c->precision, record_out ? kStepRecord : kStep, L, c->stream));
    if (c->timing) HIP_TRY(hipEventRecord(e1, c->stream));
    if (record_out)
      HIP_TRY(launch_record_finalize(c->d_partials, L.segs, t->nseg, c->d_samples, record_out, c->stream));
    for (const Seg& g : t->host) c->steps[g.sample] += 1;
  }
  c->tick += 1;
  return MCLBM_OK;
}

// Length of one graph: a whole number of periods of the parity/activity
// pattern (2 * max stride ticks), at least 32 ticks.
int64_t graph_length(const mclbm_ctx* c) {
  const int64_t period = 2 * int64_t(c->max_stride);
  return period * std::max<int64_t>(1, (32 + period - 1) / period);
}

// Graphs are used when one period needs few enough launch tables that all of
// them stay resident in the table pool while the graph exists.
bool graphs_possible(const mclbm_ctx* c) { return 2 * int64_t(c->max_stride) <= kMaxTables / 4; }

mclbm_status run_graph(mclbm_ctx* c) {
  const int64_t len = graph_length(c);
  const int64_t phase = c->tick % (2 * int64_t(c->max_stride));
  auto it = c->graphs.find(phase);
  if (it == c->graphs.end()) {
    // leave room for every table of the period so that none is evicted
    // between building the tables and capturing the launches that read them
    mclbm_status rs = reserve_tables(c, kMaxTables / 4 + 8);
    if (rs != MCLBM_OK) return rs;
    it = c->graphs.end();
    // make sure every table of the period exists before capturing
    const int64_t tick0 = c->tick;
    std::vector<int64_t> steps0 = c->steps;
    for (int64_t k = 0; k < len; ++k) {
      const Table* t = nullptr;
      mclbm_status st = get_table(c, c->tick, false, c->block, false, &t);
      if (st != MCLBM_OK) return st;
      for (const Seg& g : t->host) c->steps[g.sample] += 1;
      c->tick += 1;
    }
    c->tick = tick0;
    c->steps = steps0;
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    mclbm_status st = MCLBM_OK;
    for (int64_t k = 0; k < len && st == MCLBM_OK; ++k) st = run_tick(c, nullptr);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &graph);
    c->tick = tick0;
    c->steps = steps0;
    if (st != MCLBM_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e != hipSuccess) return fail(MCLBM_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(MCLBM_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    it = c->graphs.emplace(phase, exec).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, c->stream));
  // bookkeeping of the ticks the graph ran
  for (int64_t k = 0; k < len; ++k) {
    for (int s = 0; s < c->m; ++s)
      if (c->tick % c->desc[s].stride == 0) c->steps[s] += 1;
    c->tick += 1;
  }
  return MCLBM_OK;
}

mclbm_status run_plain_ticks(mclbm_ctx* c, int64_t ticks) {
  int64_t left = ticks;
  const int64_t len = graph_length(c);
  while (left > 0) {
    if (c->use_graphs && c->stream && !c->timing && graphs_possible(c) && left >= len) {
      mclbm_status st = run_graph(c);
      if (st != MCLBM_OK) return st;
      left -= len;
    } else {
      mclbm_status st = run_tick(c, nullptr);
      if (st != MCLBM_OK) return st;
      left -= 1;
    }
  }
  return MCLBM_OK;
}

mclbm_status check_ctx(const mclbm_ctx* c, bool need_init) {
  if (!c) return fail(MCLBM_ERR_ARG, "context is NULL");
  if (need_init && !c->initialized) return fail(MCLBM_ERR_STATE, "mclbm_init has not been called");
  return MCLBM_OK;
}

mclbm_status check_flags(mclbm_ctx* c, int32_t* first_bad) {
  std::vector<int32_t> flags(c->m);
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(flags.data(), c->d_flags, sizeof(int32_t) * c->m, hipMemcpyDeviceToHost));
  for (int s = 0; s < c->m; ++s)
    if (flags[s]) {
      if (first_bad) *first_bad = s;
      return fail(MCLBM_ERR_UNSTABLE, "sample " + std::to_string(s) + " became unstable (non-finite density or "
                                      "velocity, or a non-positive equilibrium population)");
    }
  if (first_bad) *first_bad = -1;
  return MCLBM_OK;
}

uint64_t splitmix64_next(uint64_t& state) {
  state += 0x9E3779B97F4A7C15ull;
  uint64_t z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" {

double mclbm_omega(int32_t n, double u0, double re) {
  if (n < 1 || !(u0 > 0.0) || !(re > 0.0)) return 0.0;
  return omega_of(lattice_nu(n, u0, re));
}

size_t mclbm_workspace_bytes(int32_t m, const mclbm_sample_desc* desc, int32_t precision, int32_t lattice) {
  if (validate_desc(m, desc, precision, lattice) != MCLBM_OK) return 0;
  return layout_of(m, desc, precision, lattice).total;
}

mclbm_status mclbm_create(mclbm_ctx** out, int32_t m, const mclbm_sample_desc* desc, int32_t precision,
                          int32_t lattice, void* workspace, size_t workspace_bytes, void* hip_stream) {
  if (!out) return fail(MCLBM_ERR_ARG, "out is NULL");
  *out = nullptr;
  mclbm_status st = validate_desc(m, desc, precision, lattice);
  if (st != MCLBM_OK) return st;
  const Layout L = layout_of(m, desc, precision, lattice);
  if (!workspace) return fail(MCLBM_ERR_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign) return fail(MCLBM_ERR_ARG, "workspace must be 256-byte aligned");
  if (workspace_bytes < L.total)
    return fail(MCLBM_ERR_OOM, "workspace too small: need " + std::to_string(L.total) + " bytes");

  mclbm_ctx* c = new mclbm_ctx();
  c->m = m;
  c->precision = precision;
  c->q = lattice;
  c->elem = precision == MCLBM_FP64 ? 8 : 4;
  c->desc.assign(desc, desc + m);
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->ws = static_cast<char*>(workspace);
  c->ws_bytes = workspace_bytes;
  c->d_samples = reinterpret_cast<DevSample*>(c->ws + L.samples);
  c->d_flags = reinterpret_cast<int32_t*>(c->ws + L.flags);
  c->d_ycoef = reinterpret_cast<double*>(c->ws + L.ycoef);
  c->d_pmat = reinterpret_cast<double*>(c->ws + L.pmat);
  c->d_diss = reinterpret_cast<DissSample*>(c->ws + L.diss);
  c->d_tables = reinterpret_cast<Seg*>(c->ws + L.tables);
  c->table_pool_bytes = L.table_bytes;
  c->d_partials = reinterpret_cast<double*>(c->ws + L.partials);
  c->partial_blocks = L.partial_blocks;
  c->pop = c->ws + L.pop;
  c->state_bytes = L.state_bytes;
  c->steps.assign(m, 0);
  c->y.assign(size_t(m) * 24, 0.0);
  c->pmat = projection_matrix();
  c->h_samples.resize(m);
  size_t off = 0;
  for (int s = 0; s < m; ++s) {
    DevSample& h = c->h_samples[s];
    std::memset(&h, 0, sizeof(h));
    h.offset = off / c->elem;
    h.n = desc[s].n;
    h.log2n = ilog2(desc[s].n);
    h.pstride = uint32_t(plane_stride(desc[s].n, c->elem));
    h.u0 = desc[s].u0;
    h.amp = desc[s].amp;
    h.project = desc[s].project;
    h.voffset = c->vel_doubles;
    c->vel_doubles += 3 * size_t(c->cells(s));
    fill_sample(c, s, lattice_nu(desc[s]));
    off = align_up(off + size_t(c->q) * h.pstride * c->elem);
    c->max_stride = std::max(c->max_stride, desc[s].stride);
  }
  hipError_t e = hipMemcpy(c->d_samples, c->h_samples.data(), sizeof(DevSample) * m, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_pmat, c->pmat.data(), sizeof(double) * 24 * 24, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->d_flags, 0, sizeof(int32_t) * size_t(m));
  if (e == hipSuccess) {
    std::vector<DissSample> ds(m);
    for (int s = 0; s < m; ++s) {
      ds[s].inv_u0sq = 1.0 / (desc[s].u0 * desc[s].u0);
      ds[s].dt = 2.0 * M_PI / desc[s].n * desc[s].u0;  // dx * u0 / U_c with U_c = 1
      ds[s].stride = desc[s].stride;
    }
    e = hipMemcpy(c->d_diss, ds.data(), sizeof(DissSample) * m, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    delete c;
    return fail(MCLBM_ERR_HIP, std::string("context upload: ") + hipGetErrorString(e));
  }
  c->ckpt_header.assign(kHeaderBytes, 0);
  *out = c;
  return MCLBM_OK;
}

mclbm_status mclbm_destroy(mclbm_ctx* c) {
  if (!c) return MCLBM_OK;
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
  return MCLBM_OK;
}

mclbm_status mclbm_init(mclbm_ctx* c, uint64_t seed, const double* y_host) {
  mclbm_status st = check_ctx(c, false);
  if (st != MCLBM_OK) return st;
  if (y_host) {
    for (size_t k = 0; k < size_t(c->m) * 24; ++k)
      if (!std::isfinite(y_host[k])) return fail(MCLBM_ERR_ARG, "Y contains a non-finite value");
    std::copy(y_host, y_host + size_t(c->m) * 24, c->y.begin());
  } else {
    uint64_t state = seed;
    for (size_t k = 0; k < size_t(c->m) * 24; ++k)
      c->y[k] = 2.0 * (double(splitmix64_next(state) >> 11) * 0x1.0p-53) - 1.0;
  }
  // coefficients of the (projected) perturbation per sample
  std::vector<double> yc(size_t(c->m) * 24);
  for (int s = 0; s < c->m; ++s) {
    const double* ys = &c->y[size_t(s) * 24];
    for (int q = 0; q < 24; ++q) {
      double v = ys[q];
      if (c->desc[s].project) {
        v = 0.0;
        for (int p = 0; p < 24; ++p) v += c->pmat[q * 24 + p] * ys[p];
      }
      yc[size_t(s) * 24 + q] = v;
    }
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(c->d_ycoef, yc.data(), sizeof(double) * yc.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(c->d_flags, 0, sizeof(int32_t) * size_t(c->m)));
  std::fill(c->steps.begin(), c->steps.end(), 0);
  c->tick = 0;
  const Table* t = nullptr;
  st = get_table(c, 0, true, kAuxBlock, true, &t);
  if (st != MCLBM_OK) return st;
  c->generation += 1;
  HIP_TRY(launch_init(c->q, c->precision, c->pop, c->d_samples, table_ptr(c, t), t->nseg, t->total_blocks, c->d_ycoef,
                      c->stream));
  c->initialized = true;
  return MCLBM_OK;
}

mclbm_status mclbm_get_y(const mclbm_ctx* c, double* y_host) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (!y_host) return fail(MCLBM_ERR_ARG, "y_host is NULL");
  std::memcpy(y_host, c->y.data(), sizeof(double) * c->y.size());
  return MCLBM_OK;
}

mclbm_status mclbm_set_viscosity(mclbm_ctx* c, const double* eps_host) {
  mclbm_status st = check_ctx(c, false);
  if (st != MCLBM_OK) return st;
  if (!eps_host) return fail(MCLBM_ERR_ARG, "eps_host is NULL");
  for (int s = 0; s < c->m; ++s)
    if (!(eps_host[s] > 0.0) || !std::isfinite(eps_host[s])) return fail(MCLBM_ERR_ARG, "viscosity must be > 0");
  c->generation += 1;
  for (int s = 0; s < c->m; ++s) {
    c->desc[s].re = 1.0 / eps_host[s];
    fill_sample(c, s, lattice_nu(c->desc[s]));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(c->d_samples, c->h_samples.data(), sizeof(DevSample) * c->m, hipMemcpyHostToDevice));
  return MCLBM_OK;
}

mclbm_status mclbm_step(mclbm_ctx* c, int64_t ticks, int32_t record_every, double* records_dev,
                        int64_t max_records) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (ticks < 0) return fail(MCLBM_ERR_ARG, "ticks must be >= 0");
  if (record_every < 0) return fail(MCLBM_ERR_ARG, "record_every must be >= 0");
  if (ticks > 0) c->generation += 1;
  if (record_every > 0) {
    if (!records_dev) return fail(MCLBM_ERR_ARG, "records_dev is NULL");
    for (int s = 0; s < c->m; ++s)
      if (record_every % c->desc[s].stride) return fail(MCLBM_ERR_ARG, "record_every must be a multiple of every stride");
    if (c->tick % c->max_stride) return fail(MCLBM_ERR_ARG, "recording must start on a tick where every sample steps");
    const int64_t need = (ticks + record_every - 1) / record_every;
    if (need > max_records) return fail(MCLBM_ERR_OOM, "records_dev holds " + std::to_string(max_records) +
                                                           " records, " + std::to_string(need) + " needed");
    int64_t k = 0;
    for (int64_t t = 0; t < ticks;) {
      st = run_tick(c, records_dev + size_t(k) * c->m * kRecord);
      if (st != MCLBM_OK) return st;
      ++k;
      ++t;
      const int64_t plain = std::min<int64_t>(record_every - 1, ticks - t);
      st = run_plain_ticks(c, plain);
      if (st != MCLBM_OK) return st;
      t += plain;
    }
    return MCLBM_OK;
  }
  return run_plain_ticks(c, ticks);
}

mclbm_status mclbm_moments(mclbm_ctx* c, int32_t sample, double* rho_dev, double* u_dev) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (sample < 0 || sample >= c->m) return fail(MCLBM_ERR_ARG, "sample out of range");
  HIP_TRY(launch_moments(c->q, c->precision, c->pop, c->d_samples, sample, c->desc[sample].n, int32_t(c->steps[sample] & 1),
                         rho_dev, u_dev, c->stream));
  return check_flags(c, nullptr);
}

mclbm_status mclbm_reduce(mclbm_ctx* c, double* red_dev) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (!red_dev) return fail(MCLBM_ERR_ARG, "red_dev is NULL");
  const Table* t = nullptr;
  st = get_table(c, c->tick, true, c->block, false, &t);
  if (st != MCLBM_OK) return st;
  StepLaunch L = make_launch(c, t, c->pop, nullptr);
  HIP_TRY(launch_step(c->q, c->precision, kReduceOnly, L, c->stream));
  HIP_TRY(launch_record_finalize(c->d_partials, L.segs, t->nseg, c->d_samples, red_dev, c->stream));
  return check_flags(c, nullptr);
}

mclbm_status mclbm_check(mclbm_ctx* c, int32_t* first_bad) {
  mclbm_status st = check_ctx(c, false);
  if (st != MCLBM_OK) return st;
  return check_flags(c, first_bad);
}

mclbm_status mclbm_get_state(mclbm_ctx* c, int32_t sample, double* f_dev) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (sample < 0 || sample >= c->m || !f_dev) return fail(MCLBM_ERR_ARG, "bad sample or NULL buffer");
  HIP_TRY(launch_get_state(c->q, c->precision, c->pop, c->d_samples, sample, c->desc[sample].n,
                           int32_t(c->steps[sample] & 1), f_dev, c->stream));
  return MCLBM_OK;
}

mclbm_status mclbm_set_state(mclbm_ctx* c, int32_t sample, const double* f_dev) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (sample < 0 || sample >= c->m || !f_dev) return fail(MCLBM_ERR_ARG, "bad sample or NULL buffer");
  c->generation += 1;
  HIP_TRY(launch_set_state(c->q, c->precision, c->pop, c->d_samples, sample, c->desc[sample].n,
                           int32_t(c->steps[sample] & 1), f_dev, c->stream));
  return MCLBM_OK;
}

mclbm_status mclbm_get_cells(mclbm_ctx* c, int32_t sample, const int64_t* cells_dev, int32_t count, double* f_dev) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (sample < 0 || sample >= c->m) return fail(MCLBM_ERR_ARG, "sample out of range");
  if (count < 0 || (count > 0 && (!cells_dev || !f_dev))) return fail(MCLBM_ERR_ARG, "bad cell list");
  if (count == 0) return MCLBM_OK;
  // the cell indices live on the device; validate them on a host copy
  std::vector<int64_t> h(count);
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(h.data(), cells_dev, sizeof(int64_t) * count, hipMemcpyDeviceToHost));
  for (int64_t v : h)
    if (v < 0 || v >= c->cells(sample)) return fail(MCLBM_ERR_ARG, "cell index out of range");
  HIP_TRY(launch_gather_cells(c->q, c->precision, c->pop, c->d_samples, sample, int32_t(c->steps[sample] & 1), cells_dev,
                              count, f_dev, c->stream));
  return MCLBM_OK;
}

mclbm_status mclbm_poison(mclbm_ctx* c, int32_t sample, int64_t cell, int32_t i) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (sample < 0 || sample >= c->m) return fail(MCLBM_ERR_ARG, "sample out of range");
  if (cell < 0 || cell >= c->cells(sample) || i < 0 || i >= c->q)
    return fail(MCLBM_ERR_ARG, "cell or velocity out of range");
  c->generation += 1;
  HIP_TRY(launch_poison(c->q, c->precision, c->pop, c->d_samples, sample, int32_t(c->steps[sample] & 1), cell, i, c->stream));
  return MCLBM_OK;
}

size_t mclbm_checkpoint_bytes(const mclbm_ctx* c) { return c ? kHeaderBytes + c->state_bytes : 0; }

mclbm_status mclbm_checkpoint(mclbm_ctx* c, void* dst_dev, size_t bytes) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (!dst_dev) return fail(MCLBM_ERR_ARG, "dst_dev is NULL");
  if (bytes < mclbm_checkpoint_bytes(c)) return fail(MCLBM_ERR_OOM, "checkpoint buffer too small");
  // header: magic, m, precision, lattice, tick, steps[m]
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::vector<int64_t> h(5 + c->m);
  h[0] = int64_t(kCkptMagic);
  h[1] = c->m;
  h[2] = c->precision;
  h[3] = c->q;
  h[4] = c->tick;
  for (int s = 0; s < c->m; ++s) h[5 + s] = c->steps[s];
  HIP_TRY(hipMemcpy(dst_dev, h.data(), sizeof(int64_t) * h.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpyAsync(static_cast<char*>(dst_dev) + kHeaderBytes, c->pop, c->state_bytes, hipMemcpyDeviceToDevice,
                         c->stream));
  return MCLBM_OK;
}

mclbm_status mclbm_restore(mclbm_ctx* c, const void* src_dev, size_t bytes) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (!src_dev) return fail(MCLBM_ERR_ARG, "src_dev is NULL");
  if (bytes < mclbm_checkpoint_bytes(c)) return fail(MCLBM_ERR_OOM, "checkpoint buffer too small");
  HIP_TRY(hipStreamSynchronize(c->stream));
  std::vector<int64_t> h(5 + c->m);
  HIP_TRY(hipMemcpy(h.data(), src_dev, sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost));
  if (h[0] != int64_t(kCkptMagic) || h[1] != c->m || h[2] != c->precision || h[3] != c->q)
    return fail(MCLBM_ERR_ARG, "checkpoint does not belong to this ensemble");
  c->generation += 1;
  HIP_TRY(hipMemcpyAsync(c->pop, static_cast<const char*>(src_dev) + kHeaderBytes, c->state_bytes,
                         hipMemcpyDeviceToDevice, c->stream));
  c->tick = h[4];
  for (int s = 0; s < c->m; ++s) c->steps[s] = h[5 + s];
  HIP_TRY(hipMemsetAsync(c->d_flags, 0, sizeof(int32_t) * size_t(c->m), c->stream));
  return MCLBM_OK;
}

// ------------------------------------------------------------------ adjoint
size_t mclbm_ckpt_bytes(const mclbm_ctx* c, int64_t ticks, int32_t ckpt_every) {
  if (!c || ticks < 1 || ckpt_every < 1) return 0;
  const int64_t nck = (ticks + ckpt_every - 1) / ckpt_every;
  return kFwdHeaderBytes + size_t(nck) * c->state_bytes;
}

size_t mclbm_backward_work_bytes(const mclbm_ctx* c, int32_t ckpt_every) {
  if (!c || ckpt_every < 1) return 0;
  size_t cells = 0;
  for (int s = 0; s < c->m; ++s) cells += size_t(c->cells(s));
  const size_t partials = align_up(cells / kAuxBlock * 24 * sizeof(double));
  const size_t records = align_up(size_t(c->m) * kRecord * sizeof(double));
  return size_t(ckpt_every) * c->state_bytes + 2 * c->state_bytes + partials + records;
}

static mclbm_status check_adjoint(mclbm_ctx* c, int64_t ticks, int32_t ckpt_every) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (ticks < 1 || ckpt_every < 1) return fail(MCLBM_ERR_ARG, "ticks and ckpt_every must be >= 1");
  for (int s = 0; s < c->m; ++s)
    if (c->desc[s].stride != 1) return fail(MCLBM_ERR_UNSUPPORTED, "the adjoint needs every stride to be 1");
  // The exact minimiser's derivative grows like 1/|dh| near equilibrium (its
  // change of f* does not vanish with dh), and in FP32 dh is rounding there.
  if (c->exact_gamma && c->precision != MCLBM_FP64)
    return fail(MCLBM_ERR_UNSUPPORTED, "the adjoint of the exact stabiliser is built for FP64 states");
  return MCLBM_OK;
}

mclbm_status mclbm_forward_ckpt(mclbm_ctx* c, int64_t ticks, int32_t ckpt_every, void* ckpt_dev, size_t ckpt_bytes) {
  mclbm_status st = check_adjoint(c, ticks, ckpt_every);
  if (st != MCLBM_OK) return st;
  if (c->tick != 0) return fail(MCLBM_ERR_STATE, "forward_ckpt must start from step 0 (call mclbm_init first)");
  if (!ckpt_dev || ckpt_bytes < mclbm_ckpt_bytes(c, ticks, ckpt_every))
    return fail(MCLBM_ERR_OOM, "checkpoint buffer too small");
  c->generation += 1;
  c->fwd_generation = 0;
  char* ck = static_cast<char*>(ckpt_dev) + kFwdHeaderBytes;
  for (int64_t k = 0; k * ckpt_every < ticks; ++k) {
    const Table* t = nullptr;
    st = get_table(c, c->tick, true, kAuxBlock, false, &t);
    if (st != MCLBM_OK) return st;
    HIP_TRY(launch_canonical_copy(c->q, c->precision, c->pop, ck + size_t(k) * c->state_bytes, c->d_samples,
                                  table_ptr(c, t), t->nseg, t->total_blocks, c->stream));
    st = run_plain_ticks(c, std::min<int64_t>(ckpt_every, ticks - k * ckpt_every));
    if (st != MCLBM_OK) return st;
  }
  const uint64_t token = ++g_fwd_tokens;
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(ckpt_dev, &token, sizeof(token), hipMemcpyHostToDevice));
  c->fwd_token = token;
  c->fwd_generation = c->generation;
  return MCLBM_OK;
}

mclbm_status mclbm_backward(mclbm_ctx* c, int64_t ticks, int32_t ckpt_every, const void* ckpt_dev,
                            size_t ckpt_bytes, void* work_dev, size_t work_bytes, double* dJdY_dev,
                            double* ke_dev) {
  mclbm_status st = check_adjoint(c, ticks, ckpt_every);
  if (st != MCLBM_OK) return st;
  if (c->tick != ticks) return fail(MCLBM_ERR_STATE, "backward must follow forward_ckpt over the same ticks");
  if (!ckpt_dev || ckpt_bytes < mclbm_ckpt_bytes(c, ticks, ckpt_every))
    return fail(MCLBM_ERR_OOM, "checkpoint buffer too small");
  if (!work_dev || work_bytes < mclbm_backward_work_bytes(c, ckpt_every))
    return fail(MCLBM_ERR_OOM, "backward work buffer too small");
  if (!dJdY_dev) return fail(MCLBM_ERR_ARG, "dJdY_dev is NULL");
  if (c->fwd_generation == 0 || c->generation != c->fwd_generation)
    return fail(MCLBM_ERR_STATE, "the state changed since mclbm_forward_ckpt (backward needs the state it left)");
  uint64_t token = 0;
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(&token, ckpt_dev, sizeof(token), hipMemcpyDeviceToHost));
  if (token != c->fwd_token)
    return fail(MCLBM_ERR_STATE, "the checkpoints were not written by the last mclbm_forward_ckpt of this context");

  char* w = static_cast<char*>(work_dev);
  char* seg_states = w;
  char* lam[2] = {w + size_t(ckpt_every) * c->state_bytes, w + size_t(ckpt_every + 1) * c->state_bytes};
  double* partials = reinterpret_cast<double*>(w + size_t(ckpt_every + 2) * c->state_bytes);
  size_t cells = 0;
  for (int s = 0; s < c->m; ++s) cells += size_t(c->cells(s));
  double* records = reinterpret_cast<double*>(reinterpret_cast<char*>(partials) +
                                              align_up(cells / kAuxBlock * 24 * sizeof(double)));

  if (ke_dev) {
    const Table* t = nullptr;
    st = get_table(c, c->tick, true, c->block, false, &t);
    if (st != MCLBM_OK) return st;
    StepLaunch L = make_launch(c, t, c->pop, nullptr);
    HIP_TRY(launch_step(c->q, c->precision, kReduceOnly, L, c->stream));
    HIP_TRY(launch_record_finalize(c->d_partials, L.segs, t->nseg, c->d_samples, records, c->stream));
    HIP_TRY(launch_extract(records, c->m, 4, ke_dev, c->stream));
  }

  st = reserve_tables(c, 3);       // the three tables below are held together
  if (st != MCLBM_OK) return st;
  const Table* aux = nullptr;      // every sample, live parities (seed)
  st = get_table(c, c->tick, true, kAuxBlock, false, &aux);
  if (st != MCLBM_OK) return st;
  HIP_TRY(launch_adjoint_seed(c->q, c->precision, c->pop, lam[0], c->d_samples, table_ptr(c, aux), aux->nseg,
                              aux->total_blocks, 1.0 / c->m, c->stream));
  const Table* nat = nullptr;      // every sample, natural layout
  st = get_table(c, 0, true, kAuxBlock, true, &nat);
  if (st != MCLBM_OK) return st;
  const Table* push = nullptr;     // push steps use the collide kernel's block
  st = get_table(c, 0, true, c->block, true, &push);
  if (st != MCLBM_OK) return st;

  const int32_t buffer_ok = make_launch(c, nat, c->pop, nullptr).buffer_ok;
  int cur = 0;
  const int64_t nseg = (ticks + ckpt_every - 1) / ckpt_every;
  for (int64_t k = nseg - 1; k >= 0; --k) {
    const int64_t n0 = k * ckpt_every;
    const int64_t n1 = std::min<int64_t>(ticks, n0 + ckpt_every);
    const char* ck = static_cast<const char*>(ckpt_dev) + kFwdHeaderBytes + size_t(k) * c->state_bytes;
    auto state_at = [&](int64_t n) -> const char* {
      return n == n0 ? ck : seg_states + size_t(n - n0) * c->state_bytes;
    };
    for (int64_t n = n0 + 1; n < n1; ++n) {
      StepLaunch L = make_launch(c, push, const_cast<char*>(state_at(n - 1)), const_cast<char*>(state_at(n)));
      HIP_TRY(launch_step(c->q, c->precision, kPush, L, c->stream));
    }
    for (int64_t n = n1 - 1; n >= n0; --n) {
      HIP_TRY(launch_adjoint_step(c->q, c->precision, state_at(n), lam[cur], lam[1 - cur], c->d_samples, table_ptr(c, nat),
                                  nat->nseg, nat->total_blocks, buffer_ok, c->exact_gamma, c->stream));
      cur = 1 - cur;
    }
  }
  HIP_TRY(launch_init_adjoint(c->q, c->precision, lam[cur], c->d_samples, table_ptr(c, nat), nat->nseg, nat->total_blocks,
                              c->d_ycoef, partials, c->stream));
  HIP_TRY(launch_init_adjoint_finalize(partials, table_ptr(c, nat), nat->nseg, c->d_samples, c->d_pmat, dJdY_dev,
                                       c->stream));
  return MCLBM_OK;
}

size_t mclbm_step_vjp_work_bytes(const mclbm_ctx* c) { return c ? 3 * c->state_bytes : 0; }

mclbm_status mclbm_step_vjp(mclbm_ctx* c, const double* lam_dev, double* out_dev, void* work_dev,
                            size_t work_bytes) {
  mclbm_status st = check_adjoint(c, 1, 1);
  if (st != MCLBM_OK) return st;
  if (!lam_dev || !out_dev) return fail(MCLBM_ERR_ARG, "lam_dev and out_dev must be given");
  if (!work_dev || work_bytes < mclbm_step_vjp_work_bytes(c)) return fail(MCLBM_ERR_OOM, "work buffer too small");
  char* state = static_cast<char*>(work_dev);
  char* lam_in = state + c->state_bytes;
  char* lam_out = lam_in + c->state_bytes;
  st = reserve_tables(c, 2);       // the two tables below are held together
  if (st != MCLBM_OK) return st;
  const Table* live = nullptr;     // every sample at its own parity
  st = get_table(c, c->tick, true, kAuxBlock, false, &live);
  if (st != MCLBM_OK) return st;
  const Table* nat = nullptr;      // every sample, natural layout
  st = get_table(c, 0, true, kAuxBlock, true, &nat);
  if (st != MCLBM_OK) return st;
  HIP_TRY(launch_canonical_copy(c->q, c->precision, c->pop, state, c->d_samples, table_ptr(c, live), live->nseg,
                                live->total_blocks, c->stream));
  size_t off = 0;
  for (int s = 0; s < c->m; ++s) {
    HIP_TRY(launch_put_adjoint(c->q, c->precision, lam_in, c->d_samples, s, c->desc[s].n, lam_dev + off, c->stream));
    off += size_t(c->q) * size_t(c->cells(s));
  }
  const int32_t buffer_ok = make_launch(c, nat, c->pop, nullptr).buffer_ok;
  HIP_TRY(launch_adjoint_step(c->q, c->precision, state, lam_in, lam_out, c->d_samples, table_ptr(c, nat), nat->nseg,
                              nat->total_blocks, buffer_ok, c->exact_gamma, c->stream));
  off = 0;
  for (int s = 0; s < c->m; ++s) {
    HIP_TRY(launch_get_adjoint(c->q, c->precision, lam_out, c->d_samples, s, c->desc[s].n, out_dev + off, c->stream));
    off += size_t(c->q) * size_t(c->cells(s));
  }
  return MCLBM_OK;
}

// ------------------------------------------------------------------ observables
size_t mclbm_observables_range_work_bytes(const mclbm_ctx* c, int32_t first, int32_t count) {
  if (!c || first < 0 || count < 1 || first + count > c->m || c->desc[first].n > kMaxObservablesN) return 0;
  for (int s = first + 1; s < first + count; ++s)
    if (c->desc[s].n != c->desc[first].n) return 0;
  return observables_work_bytes(c->desc[first].n, count);
}

size_t mclbm_observables_work_bytes(const mclbm_ctx* c, int32_t sample) {
  return mclbm_observables_range_work_bytes(c, sample, 1);
}

mclbm_status mclbm_observables_range(mclbm_ctx* c, int32_t first, int32_t count, double* s2_dev, double* ek_dev,
                                     void* work_dev, size_t work_bytes) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (first < 0 || count < 1 || first + count > c->m) return fail(MCLBM_ERR_ARG, "sample range out of bounds");
  const int n = c->desc[first].n;
  for (int s = first + 1; s < first + count; ++s)
    if (c->desc[s].n != n) return fail(MCLBM_ERR_ARG, "the samples of a range must share one n");
  if (n > kMaxObservablesN) return fail(MCLBM_ERR_UNSUPPORTED, "the observables are built for n <= 512");
  if (!work_dev || work_bytes < observables_work_bytes(n, count))
    return fail(MCLBM_ERR_OOM, "observables work buffer too small");
  if (reinterpret_cast<uintptr_t>(work_dev) % kAlign) return fail(MCLBM_ERR_ARG, "work_dev must be 256-byte aligned");
  // one set of launches per run of samples with the same AA parity
  const size_t per = observables_work_bytes(n, 1);
  for (int a = first; a < first + count;) {
    const int parity = int(c->steps[a] & 1);
    int b = a + 1;
    while (b < first + count && int(c->steps[b] & 1) == parity) ++b;
    const int k = a - first;
    HIP_TRY(launch_observables(c->q, c->precision, c->pop, c->d_samples, a, b - a, n, parity,
                               static_cast<char*>(work_dev) + size_t(k) * per,
                               s2_dev ? s2_dev + size_t(k) * (n / 2) : nullptr,
                               ek_dev ? ek_dev + size_t(k) * (n / 2 + 1) : nullptr, c->stream));
    a = b;
  }
  return MCLBM_OK;
}

mclbm_status mclbm_observables(mclbm_ctx* c, int32_t sample, double* s2_dev, double* ek_dev, void* work_dev,
                               size_t work_bytes) {
  return mclbm_observables_range(c, sample, 1, s2_dev, ek_dev, work_dev, work_bytes);
}

size_t mclbm_velocity_bytes(const mclbm_ctx* c) { return c ? sizeof(double) * c->vel_doubles : 0; }

mclbm_status mclbm_capture_velocity(mclbm_ctx* c, double* u_dev, size_t bytes) {
  mclbm_status st = check_ctx(c, false);
  if (st != MCLBM_OK) return st;
  if (u_dev) {
    if (bytes < sizeof(double) * c->vel_doubles) return fail(MCLBM_ERR_OOM, "velocity capture buffer too small");
    if (reinterpret_cast<uintptr_t>(u_dev) % kAlign) return fail(MCLBM_ERR_ARG, "u_dev must be 256-byte aligned");
  }
  c->d_vel = u_dev;
  return MCLBM_OK;
}

mclbm_status mclbm_observables_velocity_range(mclbm_ctx* c, int32_t first, int32_t count, const double* u_dev,
                                              double* s2_dev, double* ek_dev, void* work_dev, size_t work_bytes) {
  mclbm_status st = check_ctx(c, false);
  if (st != MCLBM_OK) return st;
  if (!u_dev) return fail(MCLBM_ERR_ARG, "u_dev is NULL");
  if (reinterpret_cast<uintptr_t>(u_dev) % kAlign) return fail(MCLBM_ERR_ARG, "u_dev must be 256-byte aligned");
  if (first < 0 || count < 1 || first + count > c->m) return fail(MCLBM_ERR_ARG, "sample range out of bounds");
  const int n = c->desc[first].n;
  for (int s = first + 1; s < first + count; ++s)
    if (c->desc[s].n != n) return fail(MCLBM_ERR_ARG, "the samples of a range must share one n");
  if (n > kMaxObservablesN) return fail(MCLBM_ERR_UNSUPPORTED, "the observables are built for n <= 512");
  if (!work_dev || work_bytes < observables_work_bytes(n, count))
    return fail(MCLBM_ERR_OOM, "observables work buffer too small");
  if (reinterpret_cast<uintptr_t>(work_dev) % kAlign) return fail(MCLBM_ERR_ARG, "work_dev must be 256-byte aligned");
  HIP_TRY(launch_observables_velocity(u_dev, c->d_samples, first, count, n, work_dev, s2_dev, ek_dev, c->stream));
  return MCLBM_OK;
}

mclbm_status mclbm_compensate(mclbm_ctx* c, int32_t first, int32_t count, const double* diss_dev,
                              const double* s2_dev, const double* ek_dev, double* s2c_dev, double* ekc_dev) {
  mclbm_status st = check_ctx(c, false);
  if (st != MCLBM_OK) return st;
  if (first < 0 || count < 1 || first + count > c->m) return fail(MCLBM_ERR_ARG, "sample range out of bounds");
  const int n = c->desc[first].n;
  for (int s = first + 1; s < first + count; ++s)
    if (c->desc[s].n != n) return fail(MCLBM_ERR_ARG, "the samples of a range must share one n");
  if (!diss_dev) return fail(MCLBM_ERR_ARG, "diss_dev is NULL");
  if (!s2_dev != !s2c_dev || !ek_dev != !ekc_dev)
    return fail(MCLBM_ERR_ARG, "an input and its compensated output must both be given or both be NULL");
  if (!s2_dev && !ek_dev) return MCLBM_OK;
  HIP_TRY(launch_compensate(c->d_samples, first, count, n, diss_dev, s2_dev, ek_dev, s2c_dev, ekc_dev, c->stream));
  return MCLBM_OK;
}

mclbm_status mclbm_point_values(mclbm_ctx* c, int32_t q, int32_t physical, double* out_dev) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (!out_dev) return fail(MCLBM_ERR_ARG, "out_dev is NULL");
  if (q < 1) return fail(MCLBM_ERR_ARG, "q must be >= 1");
  for (int s = 0; s < c->m; ++s)
    if (c->desc[s].n % q) return fail(MCLBM_ERR_ARG, "q must divide every sample's n");
  const Table* t = nullptr;
  st = get_table(c, c->tick, true, kAuxBlock, false, &t);
  if (st != MCLBM_OK) return st;
  if (physical != 0 && physical != 1) return fail(MCLBM_ERR_ARG, "physical must be 0 or 1");
  HIP_TRY(launch_point_values(c->q, c->precision, c->pop, c->d_samples, table_ptr(c, t), t->nseg, q, physical, out_dev,
                              c->stream));
  return MCLBM_OK;
}

size_t mclbm_w1_work_bytes(int32_t q) { return q > 0 ? size_t(3) * q * q * q * sizeof(double) : 0; }

mclbm_status mclbm_w1_1pt(const double* a_dev, const double* b_dev, int32_t m, int32_t q, double* out_dev,
                          void* work_dev, size_t work_bytes, void* hip_stream) {
  if (!a_dev || !b_dev || !out_dev || !work_dev) return fail(MCLBM_ERR_ARG, "NULL buffer");
  if (m < 1 || m > 4096) return fail(MCLBM_ERR_ARG, "m must be in [1, 4096]");
  if (q < 1 || q > 64) return fail(MCLBM_ERR_ARG, "q must be in [1, 64]");
  if (work_bytes < mclbm_w1_work_bytes(q)) return fail(MCLBM_ERR_OOM, "w1 work buffer too small");
  HIP_TRY(launch_w1(a_dev, b_dev, m, q, static_cast<double*>(work_dev), out_dev, static_cast<hipStream_t>(hip_stream)));
  return MCLBM_OK;
}

mclbm_status mclbm_ensemble_moments(const double* x_dev, int32_t m, int32_t k, int64_t ld, double* mean_dev,
                                    double* std_dev, void* hip_stream) {
  if (!x_dev || !mean_dev) return fail(MCLBM_ERR_ARG, "NULL buffer");
  if (k < 1 || ld < k) return fail(MCLBM_ERR_ARG, "need k >= 1 and ld >= k");
  if (m < (std_dev ? 2 : 1)) return fail(MCLBM_ERR_ARG, "the standard deviation needs m >= 2 (the mean m >= 1)");
  HIP_TRY(launch_ensemble_moments(x_dev, m, k, ld, mean_dev, std_dev, static_cast<hipStream_t>(hip_stream)));
  return MCLBM_OK;
}

size_t mclbm_sample_error_work_bytes(int32_t m) { return m > 0 ? size_t(4) * m * sizeof(double) : 0; }

mclbm_status mclbm_sample_error(const double* a_dev, const double* b_dev, int32_t m, int32_t q, double* out_dev,
                                void* work_dev, size_t work_bytes, void* hip_stream) {
  if (!a_dev || !b_dev || !out_dev || !work_dev) return fail(MCLBM_ERR_ARG, "NULL buffer");
  if (m < 1 || m > (1 << 20)) return fail(MCLBM_ERR_ARG, "m must be in [1, 2^20]");
  if (q < 1 || q > 64) return fail(MCLBM_ERR_ARG, "q must be in [1, 64]");
  if (work_bytes < mclbm_sample_error_work_bytes(m)) return fail(MCLBM_ERR_OOM, "sample error work buffer too small");
  HIP_TRY(launch_sample_error(a_dev, b_dev, m, q, static_cast<double*>(work_dev), out_dev,
                              static_cast<hipStream_t>(hip_stream)));
  return MCLBM_OK;
}

mclbm_status mclbm_sample_error_noalloc(const double* a_dev, const double* b_dev, int32_t m, int32_t q,
                                        double* out_dev, void* hip_stream) {
  if (!a_dev || !b_dev || !out_dev) return fail(MCLBM_ERR_ARG, "NULL buffer");
  if (m < 1 || m > kNoAllocMaxSamples)
    return fail(MCLBM_ERR_ARG, "m must be in [1, " + std::to_string(kNoAllocMaxSamples) +
                                   "] (the device scratch of the no-allocation variant)");
  if (q < 1 || q > 64) return fail(MCLBM_ERR_ARG, "q must be in [1, 64]");
  double* ratio = nullptr;
  HIP_TRY(sample_error_scratch(&ratio));
  HIP_TRY(launch_sample_error(a_dev, b_dev, m, q, ratio, out_dev, static_cast<hipStream_t>(hip_stream)));
  return MCLBM_OK;
}

mclbm_status mclbm_eoc_slope(const double* n, const double* d, int32_t k, double* slope) {
  if (!n || !d || !slope) return fail(MCLBM_ERR_ARG, "NULL argument");
  if (k < 2) return fail(MCLBM_ERR_ARG, "at least two resolutions are needed");
  double mx = 0.0, my = 0.0;
  for (int32_t i = 0; i < k; ++i) {
    if (!(n[i] > 0.0) || !(d[i] > 0.0) || !std::isfinite(n[i]) || !std::isfinite(d[i]))
      return fail(MCLBM_ERR_ARG, "resolutions and distances must be positive and finite");
    mx += std::log(n[i]);
    my += std::log(d[i]);
  }
  mx /= k;
  my /= k;
  double sxy = 0.0, sxx = 0.0;
  for (int32_t i = 0; i < k; ++i) {
    const double x = std::log(n[i]) - mx;
    sxy += x * (std::log(d[i]) - my);
    sxx += x * x;
  }
  if (!(sxx > 0.0)) return fail(MCLBM_ERR_ARG, "the resolutions must not all be equal");
  *slope = sxy / sxx;
  return MCLBM_OK;
}

// ------------------------------------------------------------------ launch shape
mclbm_status mclbm_set_launch(mclbm_ctx* c, int32_t block_threads, int32_t xcd_remap, int32_t buffer_addressing,
                              int32_t nontemporal) {
  mclbm_status st = check_ctx(c, false);
  if (st != MCLBM_OK) return st;
  if (block_threads != 128 && block_threads != 256 && block_threads != 512 && block_threads != 1024)
    return fail(MCLBM_ERR_ARG, "block_threads must be 128, 256, 512 or 1024");
  if (block_threads == 1024 && c->precision == MCLBM_FP64)
    return fail(MCLBM_ERR_UNSUPPORTED, "1024-thread blocks are built for the FP32 path only");
  for (int s = 0; s < c->m; ++s)
    if (c->cells(s) < block_threads) return fail(MCLBM_ERR_ARG, "block larger than a sample's lattice");
  if (c->exact_gamma && block_threads != 256)
    return fail(MCLBM_ERR_UNSUPPORTED, "the exact stabiliser runs 256-thread blocks only");
  if (xcd_remap != 0 && xcd_remap != 1) return fail(MCLBM_ERR_ARG, "xcd_remap must be 0 or 1");
  if (buffer_addressing != 0 && buffer_addressing != 1) return fail(MCLBM_ERR_ARG, "buffer_addressing must be 0 or 1");
  if (nontemporal != 0 && nontemporal != 1) return fail(MCLBM_ERR_ARG, "nontemporal must be 0 or 1");
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->block = block_threads;
  c->xcd_remap = xcd_remap;
  c->buffer_addr = buffer_addressing;
  c->nontemporal = nontemporal;
  drop_graphs(c);
  return MCLBM_OK;
}

mclbm_status mclbm_get_launch(const mclbm_ctx* c, int32_t* block_threads, int32_t* xcd_remap,
                              int32_t* buffer_addressing, int32_t* nontemporal) {
  if (!c) return fail(MCLBM_ERR_ARG, "context is NULL");
  if (block_threads) *block_threads = c->block;
  if (xcd_remap) *xcd_remap = c->xcd_remap;
  if (buffer_addressing) *buffer_addressing = c->buffer_addr;
  if (nontemporal) *nontemporal = c->nontemporal;
  return MCLBM_OK;
}

mclbm_status mclbm_autotune(mclbm_ctx* c, int32_t reps, void* scratch_dev, size_t scratch_bytes, int32_t* best_block,
                            int32_t* best_xcd, int32_t* best_buffer, int32_t* best_nt) {
  mclbm_status st = check_ctx(c, true);
  if (st != MCLBM_OK) return st;
  if (reps < 1) return fail(MCLBM_ERR_ARG, "reps must be >= 1");
  if (c->exact_gamma) return fail(MCLBM_ERR_UNSUPPORTED, "the exact stabiliser has one launch shape");
  st = mclbm_checkpoint(c, scratch_dev, scratch_bytes);
  if (st != MCLBM_OK) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(MCLBM_ERR_HIP, "hipEventCreate failed");
  }
  const bool timing0 = c->timing, graphs0 = c->use_graphs;
  const int b0 = c->block, x0 = c->xcd_remap, f0 = c->buffer_addr, n0 = c->nontemporal;
  c->use_graphs = false;
  c->timing = false;
  const int64_t per = 2 * int64_t(c->max_stride) * reps;
  // one trial: warm-up, timed ticks, then the state as it was
  auto trial = [&](float* ms) -> mclbm_status {
    mclbm_status r = run_plain_ticks(c, 2 * int64_t(c->max_stride));
    if (r != MCLBM_OK) return r;
    HIP_TRY(hipEventRecord(e0, c->stream));
    r = run_plain_ticks(c, per);
    if (r != MCLBM_OK) return r;
    HIP_TRY(hipEventRecord(e1, c->stream));
    HIP_TRY(hipEventSynchronize(e1));
    HIP_TRY(hipEventElapsedTime(ms, e0, e1));
    return mclbm_restore(c, scratch_dev, scratch_bytes);
  };
  const int blocks[4] = {128, 256, 512, 1024};
  float best = 1e30f;
  int bb = b0, bx = x0, bf = f0, bn = n0;
  struct Shape {
    float ms;
    int b, x, f, nt;
  };
  std::vector<Shape> timed;
  // buffer addressing needs every sample's populations below 2 GiB; without
  // it both settings run the same pointer kernels, so only one is timed
  bool buffer_possible = true;
  for (int s = 0; s < c->m; ++s)
    buffer_possible = buffer_possible && uint64_t(c->q) * c->h_samples[s].pstride * c->elem < (uint64_t(1) << 31);
  for (int b : blocks) {
    bool fits = !(b == 1024 && c->precision == MCLBM_FP64);
    for (int s = 0; s < c->m; ++s) fits = fits && c->cells(s) >= b;
    if (!fits) continue;
    for (int v = 0; v < 8 && st == MCLBM_OK; ++v) {
      const int x = v & 1, f = (v >> 1) & 1, nt = v >> 2;
      if (f && !buffer_possible) continue;
      c->block = b;
      c->xcd_remap = x;
      c->buffer_addr = f;
      c->nontemporal = nt;
      float ms = 0.f;
      st = trial(&ms);
      if (st == MCLBM_OK) timed.push_back({ms, b, x, f, nt});
    }
    if (st != MCLBM_OK) break;
  }
  // the three fastest shapes are timed twice more, each keeping its best
  // time, so that shapes a few per cent apart are not ranked by one trial
  std::sort(timed.begin(), timed.end(), [](const Shape& l, const Shape& r) { return l.ms < r.ms; });
  const size_t finalists = std::min<size_t>(3, timed.size());
  for (int round = 0; round < 2 && st == MCLBM_OK; ++round) {
    for (size_t k = 0; k < finalists && st == MCLBM_OK; ++k) {
      Shape& sh = timed[k];
      c->block = sh.b;
      c->xcd_remap = sh.x;
      c->buffer_addr = sh.f;
      c->nontemporal = sh.nt;
      float ms = 0.f;
      st = trial(&ms);
      if (st == MCLBM_OK) sh.ms = std::min(sh.ms, ms);
    }
  }
  for (size_t k = 0; k < finalists && st == MCLBM_OK; ++k) {
    if (timed[k].ms < best) {
      best = timed[k].ms;
      bb = timed[k].b;
      bx = timed[k].x;
      bf = timed[k].f;
      bn = timed[k].nt;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->use_graphs = graphs0;
  c->timing = timing0;
  if (st != MCLBM_OK) {
    // keep the error of the failed trial; put back the shape and the state
    const std::string err = g_last_error;
    c->block = b0;
    c->xcd_remap = x0;
    c->buffer_addr = f0;
    c->nontemporal = n0;
    drop_graphs(c);
    (void)mclbm_restore(c, scratch_dev, scratch_bytes);
    g_last_error = err;
    return st;
  }
  c->block = bb;
  c->xcd_remap = bx;
  c->buffer_addr = bf;
  c->nontemporal = bn;
  drop_graphs(c);
  if (best_block) *best_block = bb;
  if (best_xcd) *best_xcd = bx;
  if (best_buffer) *best_buffer = bf;
  if (best_nt) *best_nt = bn;
  return MCLBM_OK;  // every trial ended by restoring the state
}

mclbm_status mclbm_dissipation(mclbm_ctx* c, const double* records_dev, int32_t nrec, int64_t first_tick,
                               int32_t record_every, double* diss_dev, double* eta_dev) {
  mclbm_status st = check_ctx(c, false);
  if (st != MCLBM_OK) return st;
  if (!records_dev || !diss_dev) return fail(MCLBM_ERR_ARG, "records_dev and diss_dev must be given");
  if (nrec < 2) return fail(MCLBM_ERR_ARG, "at least two records are needed");
  if (first_tick < 0 || record_every < 1) return fail(MCLBM_ERR_ARG, "first_tick >= 0 and record_every >= 1");
  for (int s = 0; s < c->m; ++s)
    if (first_tick % c->desc[s].stride || record_every % c->desc[s].stride)
      return fail(MCLBM_ERR_ARG, "records must fall on ticks where every sample steps");
  if (eta_dev)
    for (int s = 1; s < c->m; ++s)
      if (c->desc[s].re != c->desc[0].re)
        return fail(MCLBM_ERR_ARG, "the Kolmogorov length needs one viscosity for the whole ensemble");
  HIP_TRY(launch_dissipation(records_dev, c->d_diss, c->m, nrec, first_tick, record_every, 1.0 / c->desc[0].re,
                             diss_dev, eta_dev, c->stream));
  return MCLBM_OK;
}

mclbm_status mclbm_dissipation_spectra(mclbm_ctx* c, int32_t first, int32_t count, const double* ek_dev,
                                       int32_t nrec, int64_t first_tick, int32_t record_every, double* diss_dev,
                                       double* eta_dev) {
  mclbm_status st = check_ctx(c, false);
  if (st != MCLBM_OK) return st;
  if (!ek_dev || !diss_dev) return fail(MCLBM_ERR_ARG, "ek_dev and diss_dev must be given");
  if (first < 0 || count < 1 || int64_t(first) + count > c->m)
    return fail(MCLBM_ERR_ARG, "the sample range leaves the ensemble");
  if (nrec < 2) return fail(MCLBM_ERR_ARG, "at least two saved spectra are needed");
  if (first_tick < 0 || record_every < 1) return fail(MCLBM_ERR_ARG, "first_tick >= 0 and record_every >= 1");
  const int n = c->desc[first].n;
  for (int s = first; s < first + count; ++s) {
    if (c->desc[s].n != n) return fail(MCLBM_ERR_ARG, "the samples of the range must share one resolution");
    if (first_tick % c->desc[s].stride || record_every % c->desc[s].stride)
      return fail(MCLBM_ERR_ARG, "saved times must fall on ticks where every sample of the range steps");
    if (eta_dev && c->desc[s].re != c->desc[first].re)
      return fail(MCLBM_ERR_ARG, "the Kolmogorov length needs one viscosity for the whole range");
  }
  HIP_TRY(launch_dissipation_spectra(ek_dev, n, c->d_diss + first, count, nrec, first_tick, record_every,
                                     1.0 / c->desc[first].re, diss_dev, eta_dev, c->stream));
  return MCLBM_OK;
}

mclbm_status mclbm_set_stabiliser(mclbm_ctx* c, int32_t mode) {
  mclbm_status st = check_ctx(c, false);
  if (st != MCLBM_OK) return st;
  if (mode != MCLBM_GAMMA_CLOSED_FORM && mode != MCLBM_GAMMA_EXACT)
    return fail(MCLBM_ERR_ARG, "stabiliser mode must be 0 (closed form) or 1 (exact)");
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->generation += 1;
  c->exact_gamma = mode == MCLBM_GAMMA_EXACT;
  if (c->exact_gamma) c->block = 256;  // every lattice has at least 512 nodes
  drop_graphs(c);
  return MCLBM_OK;
}

mclbm_status mclbm_use_graphs(mclbm_ctx* c, int32_t enable) {
  mclbm_status st = check_ctx(c, false);
  if (st != MCLBM_OK) return st;
  c->use_graphs = enable != 0;
  return MCLBM_OK;
}

int64_t mclbm_ticks(const mclbm_ctx* c) { return c ? c->tick : -1; }
int64_t mclbm_steps(const mclbm_ctx* c, int32_t sample) {
  return (c && sample >= 0 && sample < c->m) ? c->steps[sample] : -1;
}

mclbm_status mclbm_time_launches(mclbm_ctx* c, int32_t enable) {
  mclbm_status st = check_ctx(c, false);
  if (st != MCLBM_OK) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->timing = enable != 0;
  c->ev_used = 0;
  return MCLBM_OK;
}

mclbm_status mclbm_launch_time(mclbm_ctx* c, double* avg_ms, int64_t* launches) {
  mclbm_status st = check_ctx(c, false);
  if (st != MCLBM_OK) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  double total = 0.0;
  const size_t pairs = c->ev_used / 2;
  for (size_t k = 0; k < pairs; ++k) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev_pool[2 * k], c->ev_pool[2 * k + 1]));
    total += ms;
  }
  if (avg_ms) *avg_ms = pairs ? total / double(pairs) : 0.0;
  if (launches) *launches = int64_t(pairs);
  c->ev_used = 0;
  return MCLBM_OK;
}

mclbm_status mclbm_stream_copy(void* dst_dev, const void* src_dev, size_t bytes, void* hip_stream) {
  if (!dst_dev || !src_dev) return fail(MCLBM_ERR_ARG, "NULL buffer");
  if (bytes % 16) return fail(MCLBM_ERR_ARG, "bytes must be a multiple of 16");
  HIP_TRY(launch_stream_copy(dst_dev, src_dev, bytes, static_cast<hipStream_t>(hip_stream)));
  return MCLBM_OK;
}

const char* mclbm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
