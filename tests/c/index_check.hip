// Host-side check of the kernels' index arithmetic (compiled for the host
// only; no GPU is used): the cell decomposition and periodic neighbours of
// make_cell / neighbour on every lattice size the library accepts (8^3 to
// 1024^3, including the last nodes of a 1024^3 plane), the AA slot mapping
// of the in-place step (every slot read and written exactly once per step,
// and two steps stream every population by its velocity, once per step, on
// both lattices), the XCD block renumbering (a permutation of the blocks)
// and the segment search of the launch tables.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2608_23786_amd/csrc/lbm_device.h"

using namespace mclbm;

static int failures = 0;
#define CHECK(cond, ...)                        \
  do {                                          \
    if (!(cond)) {                              \
      if (failures < 20) {                      \
        std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
        std::fprintf(stderr, __VA_ARGS__);      \
        std::fprintf(stderr, "\n");             \
      }                                         \
      ++failures;                               \
    }                                           \
  } while (0)

static int64_t wrap(int64_t v, int64_t n) { return ((v % n) + n) % n; }

// make_cell and neighbour<i, s> against plain modular arithmetic
static void check_cell(uint32_t cell, int l) {
  const int64_t n = int64_t(1) << l;
  const int64_t x = cell % n, y = (cell / n) % n, z = cell / (n * n);
  const Cell c = make_cell(cell, l);
  CHECK(c.cell == cell, "cell %u", cell);
  static_for<0, 27>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    for (int s : {-1, +1}) {
      const int64_t want = (wrap(z + s * cz(i), n) * n + wrap(y + s * cy(i), n)) * n + wrap(x + s * cx(i), n);
      const uint32_t got = s < 0 ? neighbour<i, -1>(c) : neighbour<i, +1>(c);
      CHECK(int64_t(got) == want, "l %d cell %u velocity %d sign %d: %u != %lld", l, cell, i, s, got,
            (long long)want);
      const int64_t want_yz = (wrap(z + s * cz(i), n) * n + wrap(y + s * cy(i), n)) * n + x;
      const uint32_t got_yz = s < 0 ? neighbour_yz<i, -1>(c) : neighbour_yz<i, +1>(c);
      CHECK(int64_t(got_yz) == want_yz, "yz: l %d cell %u velocity %d", l, cell, i);
      CHECK(got < uint64_t(n) * n * n, "neighbour outside the lattice");
    }
  });
}

static void check_cells() {
  std::mt19937_64 rng(2608);
  for (int l = 3; l <= 10; ++l) {
    const uint64_t n3 = uint64_t(1) << (3 * l);
    if (l <= 5) {
      for (uint64_t k = 0; k < n3; ++k) check_cell(uint32_t(k), l);
      continue;
    }
    for (uint64_t k = 0; k < 4096; ++k) {
      check_cell(uint32_t(k), l);
      check_cell(uint32_t(n3 - 1 - k), l);             // the top of the plane
      check_cell(uint32_t(rng() % n3), l);
    }
    // rows, planes and their edges
    const uint64_t n = uint64_t(1) << l;
    for (uint64_t z : {uint64_t(0), n / 2, n - 1})
      for (uint64_t y : {uint64_t(0), n - 1})
        for (uint64_t x : {uint64_t(0), uint64_t(1), n - 2, n - 1}) check_cell(uint32_t((z * n + y) * n + x), l);
    // the largest index fits the 32-bit byte offsets of one plane (FP32 up
    // to 1024^3, FP64 up to 512^3)
    if (l == 10) CHECK((n3 - 1) * 4 < (uint64_t(1) << 32), "FP32 byte offset of the last node");
    if (l == 9) CHECK((n3 - 1) * 8 < (uint64_t(1) << 32), "FP64 byte offset of the last node");
  }
}

// AA: simulate two steps with an identity collision on tagged values through
// the kernel's slot functions and the state read-out.
template <int QN>
static void check_aa(int l) {
  const uint32_t n = 1u << l, n3 = n * n * n;
  const uint32_t pstride = n3 + 7;                     // a padded plane, as in the library
  std::vector<int64_t> pop(size_t(QN) * pstride, -1);
  // state at step 0: population i of node x carries tag(i, x)
  auto tag = [&](int i, uint32_t cell) { return int64_t(i) * n3 + cell; };
  for (uint32_t k = 0; k < n3; ++k) {
    int64_t g[Q];
    for_vel<QN>([&](auto ic) { g[decltype(ic)::value] = tag(decltype(ic)::value, k); });
    write_state<QN>(pop.data(), pstride, make_cell(k, l), false, g);
  }
  for (int step = 0; step < 2; ++step) {
    const bool odd = step & 1;
    std::vector<int> reads(size_t(QN) * pstride, 0), writes(size_t(QN) * pstride, 0);
    std::vector<int64_t> post(size_t(Q) * n3);
    for (uint32_t k = 0; k < n3; ++k) {
      const Cell c = make_cell(k, l);
      for_vel<QN>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const Slot s = aa_read_slot<i>(c, odd);
        const size_t e = size_t(plane_of<QN>(s.vel)) * pstride + s.idx;
        reads[e] += 1;
        post[size_t(i) * n3 + k] = pop[e];
      });
    }
    for (uint32_t k = 0; k < n3; ++k) {
      const Cell c = make_cell(k, l);
      for_vel<QN>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const Slot s = aa_write_slot<i>(c, odd);
        const size_t e = size_t(plane_of<QN>(s.vel)) * pstride + s.idx;
        writes[e] += 1;
        pop[e] = post[size_t(i) * n3 + k];
      });
    }
    for (int k = 0; k < QN; ++k)
      for (uint32_t e = 0; e < n3; ++e) {
        CHECK(reads[size_t(k) * pstride + e] == 1, "D3Q%d step %d: slot %d/%u read %d times", QN, step, k, e,
              reads[size_t(k) * pstride + e]);
        CHECK(writes[size_t(k) * pstride + e] == 1, "D3Q%d step %d: slot %d/%u written %d times", QN, step, k, e,
              writes[size_t(k) * pstride + e]);
      }
    // the post-stream state after step + 1 steps, read at the next parity:
    // population i of node x came from node x - (step + 1) c_i
    for (uint32_t k = 0; k < n3; ++k) {
      const Cell c = make_cell(k, l);
      int64_t g[Q];
      load_state<QN>(pop.data(), pstride, c, !odd, g);
      const int64_t x = k % n, y = (k / n) % n, z = k / (n * n);
      for_vel<QN>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const int64_t src = (wrap(z - (step + 1) * cz(i), n) * n + wrap(y - (step + 1) * cy(i), n)) * n +
                            wrap(x - (step + 1) * cx(i), n);
        CHECK(g[i] == tag(i, uint32_t(src)), "D3Q%d after %d steps: node %u velocity %d holds %lld", QN, step + 1,
              k, i, (long long)g[i]);
      });
    }
  }
  // the padding is never touched
  for (int k = 0; k < QN; ++k)
    for (uint32_t e = n3; e < pstride; ++e) CHECK(pop[size_t(k) * pstride + e] == -1, "pad slot written");
}

static void check_remap_and_segments() {
  for (int total : {1, 7, 8, 9, 64, 1000, 4096, 65536 + 5}) {
    std::vector<int> seen(total, 0);
    for (int b = 0; b < total; ++b) {
      const int r = remap_block(b, total, 1);
      CHECK(r >= 0 && r < total, "remap out of range");
      if (r >= 0 && r < total) seen[r] += 1;
      CHECK(remap_block(b, total, 0) == b, "identity without remap");
    }
    for (int v : seen) CHECK(v == 1, "remap is not a permutation of %d blocks", total);
  }
  std::mt19937 rng(19);
  for (int trial = 0; trial < 200; ++trial) {
    const int nseg = 1 + int(rng() % 300);
    std::vector<Seg> segs(nseg);
    int first = 0;
    for (int s = 0; s < nseg; ++s) {
      segs[s] = Seg{s, first, 1 + int(rng() % 50), 0};
      first += segs[s].nblocks;
    }
    for (int b = 0; b < first; ++b) {
      int want = 0;
      while (want + 1 < nseg && segs[want + 1].first_block <= b) ++want;
      CHECK(find_segment(segs.data(), nseg, b) == want, "segment of block %d", b);
    }
  }
}

int main() {
  check_cells();
  for (int l = 3; l <= 4; ++l) {
    check_aa<27>(l);
    check_aa<19>(l);
  }
  check_remap_and_segments();
  if (failures) {
    std::fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  std::printf("index arithmetic ok\n");
  return 0;
}
