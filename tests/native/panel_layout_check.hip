// Host-side check of the panel-ordered layout (csrc/panel.hpp): runs the
// layout's per-row and per-chunk steps -- the same functions the build
// kernels call -- on the CPU, over CSR matrices whose rows have their
// columns in random order, and checks the result entry by entry; then checks
// the launch shape of the product for row counts up to 1e8.  Built host-only
// (no kernel runs, no GPU needed).  Prints "OK" and exits 0 on success.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>
#include <algorithm>
#include "panel.hpp"

static int failures = 0;
#define CHECK(c, ...)                                           \
  do {                                                          \
    if (!(c)) {                                                 \
      if (failures < 20) { std::printf(__VA_ARGS__); std::printf("\n"); } \
      ++failures;                                               \
    }                                                           \
  } while (0)

static void check_layout(int rows, int cols, int maxlen, bool shuffle, unsigned seed) {
  std::mt19937_64 rng(seed);
  std::vector<int> rp(rows + 1, 0), ci;
  std::vector<double> v;
  for (int r = 0; r < rows; ++r) {
    const int len = (int)(rng() % (unsigned)(maxlen + 1));
    std::vector<int> c(len);
    for (int k = 0; k < len; ++k) c[k] = (int)(rng() % (unsigned)cols);
    if (!shuffle) std::sort(c.begin(), c.end());
    for (int k = 0; k < len; ++k) { ci.push_back(c[k]); v.push_back((double)ci.size() - 1.0); }
    rp[r + 1] = (int)ci.size();
  }
  const int nnz = rp[rows];
  const int nblk = (rows + HQ_BLOCK - 1) / HQ_BLOCK, nch = nblk * HQ_PANELS;
  std::vector<int> cnt((size_t)rows * HQ_PANELS, -7), size(nch, -7);
  std::vector<unsigned short> lrp((size_t)nch * (HQ_BLOCK + 1), 0xBEEF);
  for (int r = 0; r < rows; ++r) panel_count_row(r, cols, rp.data(), ci.data(), cnt.data());
  for (int ch = 0; ch < nch; ++ch) panel_offsets_chunk(ch, rows, cnt.data(), lrp.data(), size.data());
  std::vector<int> pp(nch + 1, 0);
  for (int ch = 0; ch < nch; ++ch) {
    CHECK(size[ch] >= 0 && size[ch] <= 65535, "chunk %d size %d", ch, size[ch]);
    pp[ch + 1] = pp[ch] + size[ch];
  }
  CHECK(pp[nch] == nnz, "chunk sizes sum to %d, nnz %d", pp[nch], nnz);
  // one guard slot on each side: a write outside [0, nnz) shows there
  std::vector<int> pci(nnz + 2, -1);
  std::vector<double> pv(nnz + 2, -1.0);
  for (int r = 0; r < rows; ++r)
    panel_scatter_row(r, cols, rp.data(), ci.data(), v.data(), pp.data(), lrp.data(), pci.data() + 1, pv.data() + 1);
  CHECK(pci[0] == -1 && pci[nnz + 1] == -1 && pv[0] == -1.0 && pv[nnz + 1] == -1.0, "write outside the arrays");
  // every original entry lands exactly once (v holds the entry's CSR position)
  std::vector<int> seen(nnz, 0);
  for (int d = 0; d < nnz; ++d) {
    const double k = pv[d + 1];
    CHECK(k >= 0.0 && k < nnz && k == (double)(int)k, "slot %d holds no entry (%g)", d, k);
    if (k >= 0.0 && k < nnz) {
      seen[(int)k] += 1;
      CHECK(pci[d + 1] == ci[(int)k], "slot %d: column %d, entry %d has %d", d, pci[d + 1], (int)k, ci[(int)k]);
    }
  }
  for (int k = 0; k < nnz; ++k) CHECK(seen[k] == 1, "entry %d written %d times", k, seen[k]);
  // every (row, panel) segment holds exactly that row's entries of that panel, in row order
  for (int r = 0; r < rows; ++r) {
    const int rb = r / HQ_BLOCK, lr = r % HQ_BLOCK;
    for (int p = 0; p < HQ_PANELS; ++p) {
      const int ch = rb * HQ_PANELS + p;
      const int b = pp[ch] + lrp[(size_t)ch * (HQ_BLOCK + 1) + lr], e = pp[ch] + lrp[(size_t)ch * (HQ_BLOCK + 1) + lr + 1];
      int d = b;
      for (int k = rp[r]; k < rp[r + 1]; ++k) {
        if (hq_panel_of(ci[k], cols) != p) continue;
        CHECK(d < e && pv[d + 1] == (double)k, "row %d panel %d: entry %d not at slot %d", r, p, k, d);
        ++d;
      }
      CHECK(d == e, "row %d panel %d: segment has %d slots, row has %d entries", r, p, e - b, d - b);
    }
  }
}

static void check_shape(long long rows, int ncu, const int per_cu[5], int min_bpb = 1) {
  const PanelShape sh = panel_launch_shape((int)rows, ncu, per_cu, min_bpb);
  CHECK(sh.bpb >= min_bpb, "rows %lld: bpb %d below %d", rows, sh.bpb, min_bpb);
  const long long nblk = (rows + HQ_BLOCK - 1) / HQ_BLOCK;
  CHECK(sh.grid >= 1 && sh.grid <= HQ_PCAP, "rows %lld: grid %d", rows, sh.grid);
  CHECK(sh.bpb >= 1 && sh.bpb <= 4, "rows %lld: bpb %d", rows, sh.bpb);
  // the kernel's loop: group g = blockIdx.x, + gridDim.x, ... while g * BPB < nblk
  std::vector<unsigned char> hit((size_t)nblk, 0);
  for (int b = 0; b < sh.grid; ++b)
    for (long long g = b; g * sh.bpb < nblk; g += sh.grid)
      for (int q = 0; q < sh.bpb; ++q)
        if (g * sh.bpb + q < nblk) hit[(size_t)(g * sh.bpb + q)] += 1;
  for (long long rb = 0; rb < nblk; ++rb) CHECK(hit[(size_t)rb] == 1, "rows %lld: row block %lld covered %d times", rows, rb, hit[(size_t)rb]);
  // resident whenever the matrix allows it: one group per workgroup
  if ((nblk + 3) / 4 <= (long long)ncu * per_cu[4] && (nblk + 3) / 4 <= HQ_PCAP)
    CHECK((long long)sh.grid * sh.bpb >= nblk, "rows %lld: fits but not one group per workgroup", rows);
}

int main() {
  // the panel layout is taken for short rows over many columns; small cases too
  check_layout(1, 7, 5, true, 1);
  check_layout(300, 1000, 12, true, 2);
  check_layout(300, 1000, 12, false, 3);
  check_layout(5000, 600000, 30, true, 4);
  check_layout(20000, 1 << 20, 10, true, 5);
  check_layout(257, 4, 40, true, 6);        // every panel one column wide, repeated columns
  const int occ_a[5] = {0, 8, 8, 6, 4}, occ_b[5] = {0, 2, 2, 1, 1};
  const long long rows[] = {1, 255, 256, 257, 1000000, 4194304, 4194305, 5000000, 20000000, 100000000};
  for (long long r : rows) {
    check_shape(r, 256, occ_a, 4);   // the prefetching epilogue's shape
    check_shape(r, 256, occ_a);
    check_shape(r, 256, occ_b);
    check_shape(r, 1, occ_b);
  }
  if (failures) { std::printf("FAILED: %d checks\n", failures); return 1; }
  std::printf("OK\n");
  return 0;
}
