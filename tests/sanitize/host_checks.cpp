// Host code of the library under AddressSanitizer and UBSan (built and run
// by tests/test_host_sanitizers.py): the CSR checks of validate.h on valid
// and malformed batches, each in buffers of exactly its size, and the
// serving admission policy (lcemd_serve_sim) on random arrival traces.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <random>
#include <vector>

#include "lcemd.h"
#include "validate.h"

using lcemd_host::csr_check;
using lcemd_host::ptr_check;

static int failures = 0;
#define EXPECT(cond, ...)              \
  do {                                 \
    if (!(cond)) {                     \
      fprintf(stderr, __VA_ARGS__);    \
      fprintf(stderr, "\n");           \
      ++failures;                      \
    }                                  \
  } while (0)

struct Batch {
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<float> val;
};

static Batch random_batch(std::mt19937& g, int rows, int v, int maxlen) {
  Batch b;
  b.ptr.push_back(0);
  for (int r = 0; r < rows; ++r) {
    const int h = 1 + (int)(g() % (unsigned)maxlen);
    std::vector<char> used(v, 0);
    std::vector<int32_t> cs;
    while ((int)cs.size() < h) {
      const int c = (int)(g() % (unsigned)v);
      if (!used[c]) {
        used[c] = 1;
        cs.push_back(c);
      }
    }
    std::sort(cs.begin(), cs.end());
    double s = 0.0;
    std::vector<double> w(h);
    for (int i = 0; i < h; ++i) s += (w[i] = 1.0 + (g() % 1000));
    for (int i = 0; i < h; ++i) {
      b.col.push_back(cs[i]);
      b.val.push_back((float)(w[i] / s));
    }
    b.ptr.push_back((int64_t)b.col.size());
  }
  b.col.shrink_to_fit();
  b.val.shrink_to_fit();
  return b;
}

static int check(const Batch& b, int v, bool norm, int* hmax) {
  char msg[256];
  // exact-size copies: any read past a row's end or past rowptr[rows] is caught
  std::vector<int64_t> p(b.ptr);
  std::vector<int32_t> c(b.col);
  std::vector<float> w(b.val);
  return csr_check("batch", p.data(), c.data(), w.data(), (int64_t)p.size() - 1, v, norm, hmax, msg, sizeof msg);
}

int main() {
  std::mt19937 g(12345);
  // valid batches of every shape
  for (int t = 0; t < 300; ++t) {
    const int rows = 1 + (int)(g() % 20), v = 5 + (int)(g() % 200);
    const int maxlen = 1 + (int)(g() % std::min(v, 60));
    Batch b = random_batch(g, rows, v, maxlen);
    int hm = -1;
    const int rc = check(b, v, true, &hm);
    int want = 0;
    for (int r = 0; r < rows; ++r) want = std::max<int>(want, (int)(b.ptr[r + 1] - b.ptr[r]));
    EXPECT(rc == LCEMD_OK && hm == want, "valid batch %d rejected (%d) or hmax %d != %d", t, rc, hm, want);
    std::vector<int64_t> p(b.ptr);
    char msg[256];
    int hp = -1;
    EXPECT(ptr_check("p", p.data(), rows, &hp, msg, sizeof msg) == LCEMD_OK && hp == want, "ptr_check %d", t);
  }
  // malformed batches: each mistake gives its code, on buffers of exact size
  for (int t = 0; t < 300; ++t) {
    const int rows = 2 + (int)(g() % 10), v = 40;
    Batch b = random_batch(g, rows, v, 12);
    const int r = (int)(g() % (unsigned)rows);
    const int64_t a = b.ptr[r], e = b.ptr[r + 1];
    int want = LCEMD_E_BAD_CSR;
    switch (t % 9) {
      case 0: b.ptr[0] = 1; break;
      case 1: b.col[a] = v; break;                            // column out of range
      case 2: b.col[a] = -1 - (int)(g() % 5); break;          // negative column
      case 3: if (e - a >= 2) b.col[a + 1] = b.col[a]; else b.col[a] = v + 3; break;  // repeated column
      case 4: b.val[a] = std::numeric_limits<float>::quiet_NaN(); break;
      case 5: b.val[a] = 0.f; break;
      case 6: b.val[a] = -b.val[a]; break;
      case 7: b.val[a] *= 3.f; break;                         // row no longer sums to 1
      case 8: {                                                // an empty row: rowptr repeats
        Batch d;
        d.ptr = b.ptr;
        for (int q = r + 1; q <= rows; ++q) d.ptr[q] -= (e - a);
        d.col.assign(b.col.begin(), b.col.begin() + a);
        d.col.insert(d.col.end(), b.col.begin() + e, b.col.end());
        d.val.assign(b.val.begin(), b.val.begin() + a);
        d.val.insert(d.val.end(), b.val.begin() + e, b.val.end());
        b = d;
        break;
      }
    }
    int hm = 0;
    const int rc = check(b, v, true, &hm);
    EXPECT(rc == want, "malformed case %d (kind %d) gave %d", t, t % 9, rc);
  }
  {  // a row over the length limit
    Batch b;
    const int h = LCEMD_MAX_HIST + 1;
    b.ptr = {0, h};
    for (int i = 0; i < h; ++i) {
      b.col.push_back(i);
      b.val.push_back(1.f / h);
    }
    int hm = 0;
    EXPECT(check(b, h + 5, true, &hm) == LCEMD_E_CAPACITY, "long row not refused");
  }
  // serving admission on random traces
  for (int t = 0; t < 200; ++t) {
    const int nq = 1 + (int)(g() % 300);
    std::vector<double> arr(nq);
    std::vector<int32_t> words(nq);
    double clock = 0.0;
    for (int i = 0; i < nq; ++i) {
      clock += (g() % 1000) * 1e-5;
      arr[i] = clock;
      words[i] = 1 + (int)(g() % 700);
    }
    const int lanes = 1 + (int)(g() % 4), slots = 1 + (int)(g() % 16), maxw = 64 + (int)(g() % 1024);
    std::vector<int32_t> status(nq), lane(nq), launch(nq);
    std::vector<double> start(nq), finish(nq);
    const int rc = lcemd_serve_sim(nq, arr.data(), words.data(), lanes, slots, maxw, (int64_t)1 << 34, 1e6, 0.01,
                                   0.001, status.data(), lane.data(), launch.data(), start.data(), finish.data());
    EXPECT(rc >= 1, "serve_sim trace %d failed with %d", t, rc);
    if (rc < 1) continue;
    double last = -1.0;
    for (int i = 0; i < nq; ++i) {
      if (words[i] > maxw) {
        EXPECT(status[i] == LCEMD_E_CAPACITY, "trace %d: long query %d not refused", t, i);
        continue;
      }
      EXPECT(status[i] == 0 && lane[i] >= 0 && lane[i] < lanes, "trace %d query %d: status %d lane %d", t, i,
             status[i], lane[i]);
      EXPECT(start[i] >= arr[i] && finish[i] > start[i], "trace %d query %d times", t, i);
      EXPECT(start[i] >= last, "trace %d: query %d started out of order", t, i);
      last = start[i];
    }
  }
  if (failures) {
    fprintf(stderr, "%d failures\n", failures);
    return 1;
  }
  printf("host checks ok\n");
  return 0;
}
