// Host-side check of the column-split layout (csrc/split.hpp): runs the
// layout's per-row steps -- the same functions the build kernels call -- on
// the CPU, over CSR matrices whose rows list their columns in sorted or in
// random order (with repeats), and checks every (panel, row) segment entry by
// entry against the row's own entries in that panel, in CSR order.  Built
// host-only (no kernel runs, no GPU needed).  Prints "OK" and exits 0 on success.
#include <cstdio>
#include <random>
#include <vector>
#include <algorithm>
#include "split.hpp"

static int failures = 0;
#define CHECK(c, ...)                                           \
  do {                                                          \
    if (!(c)) {                                                 \
      if (failures < 20) { std::printf(__VA_ARGS__); std::printf("\n"); } \
      ++failures;                                               \
    }                                                           \
  } while (0)

static void check_layout(int rows, int cols, int maxlen, bool shuffle, unsigned seed, int pw) {
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
  const int np = (cols + pw - 1) / pw;
  const size_t cells = (size_t)np * rows;
  std::vector<int> cnt(cells, 0);
  for (int r = 0; r < rows; ++r) split_count_row(r, rows, pw, rp.data(), ci.data(), cnt.data());
  std::vector<int> off(cells + 1, 0);
  for (size_t c = 0; c < cells; ++c) off[c + 1] = off[c] + cnt[c];
  CHECK(off[cells] == nnz, "counts sum to %d, nnz %d", off[cells], nnz);
  // one guard slot on each side: a write outside [0, nnz) shows there
  std::vector<unsigned short> lci(nnz + 2, 0xBEEF);
  std::vector<double> sv(nnz + 2, -1.0);
  std::vector<int> cur(off.begin(), off.end() - 1);
  for (int r = 0; r < rows; ++r) split_scatter_row(r, rows, pw, rp.data(), ci.data(), v.data(), cur.data(), lci.data() + 1,
                                             sv.data() + 1);
  CHECK(lci[0] == 0xBEEF && lci[nnz + 1] == 0xBEEF, "scatter wrote outside the arrays");
  for (size_t c = 0; c < cells; ++c) CHECK(cur[c] == off[c + 1], "cell %zu: cursor %d, end %d", c, cur[c], off[c + 1]);
  for (int p = 0; p < np; ++p)
    for (int r = 0; r < rows; ++r) {
      std::vector<int> want;
      for (int k = rp[r]; k < rp[r + 1]; ++k)
        if (ci[k] / pw == p) want.push_back(k);
      const int b = off[(size_t)p * rows + r], e = off[(size_t)p * rows + r + 1];
      CHECK(e - b == (int)want.size(), "panel %d row %d: %d entries, want %zu", p, r, e - b, want.size());
      for (int q = 0; q < (int)want.size() && q < e - b; ++q) {
        const int k = want[q];
        CHECK(lci[1 + b + q] == ci[k] - p * pw && sv[1 + b + q] == v[k],
              "panel %d row %d entry %d: (%d, %g) want (%d, %g)", p, r, q, (int)lci[1 + b + q], sv[1 + b + q],
              ci[k] - p * pw, v[k]);
      }
    }
}

int main() {
  for (int pw : {HQ_SPLIT_PW, HQ_SPLIT_PW_WIDE}) {
    check_layout(1, 5000, 3000, false, 1, pw);
    check_layout(37, 20000, 2500, true, 2, pw);      // random order and repeats
    check_layout(200, 9 * pw + 17, 900, false, 3, pw);   // ragged last panel
    check_layout(300, 14337, 60, true, 4, pw);
    check_layout(5, 70000, 0, false, 5, pw);         // empty rows
    check_layout(3000, 65536 * 3, 400, true, 6, pw);
  }
  if (failures) { std::printf("%d failures\n", failures); return 1; }
  std::printf("OK\n");
  return 0;
}
