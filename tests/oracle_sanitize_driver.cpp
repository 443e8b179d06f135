// Drives every entry point of the CPU oracle on random small graphs so that
// a build with AddressSanitizer and UndefinedBehaviorSanitizer can check it
// for out-of-bounds accesses, leaks and undefined behaviour. Host code only;
// exits 0 when every call returned its expected status.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
int32_t oracle_refine(int64_t, int64_t, const int32_t*, const int32_t*, const int32_t*, const int32_t*, int32_t,
                      int32_t, int32_t*, int64_t*, int64_t*, int32_t*, int32_t*);
int32_t oracle_signatures(int64_t, int64_t, const int32_t*, const int32_t*, const int32_t*, const int32_t*, int64_t,
                          const int32_t*, int64_t*, int32_t*);
int32_t oracle_signature_lengths(int64_t, int64_t, const int32_t*, const int32_t*, const int32_t*, const int32_t*,
                                 int64_t*);
void* oracle_state_create(int64_t, const int32_t*, int64_t, const int32_t*, const int32_t*, const int32_t*, int32_t);
void oracle_state_destroy(void*);
int64_t oracle_state_num_nodes(void*);
void oracle_state_history(void*, int32_t*);
void oracle_state_work(void*, int64_t*, int64_t*);
int32_t oracle_state_add_nodes(void*, int64_t, const int32_t*);
int32_t oracle_state_add_edges(void*, int64_t, const int32_t*, const int32_t*, const int32_t*);
int32_t oracle_state_delete_edges(void*, int64_t, const int32_t*, const int32_t*, const int32_t*);
int32_t oracle_state_delete_nodes(void*, int64_t, const int32_t*);
}

int main() {
  std::mt19937 rng(12345);
  int bad = 0;
  for (int it = 0; it < 300; ++it) {
    const int n = 1 + int(rng() % 40), m = int(rng() % 120), k = int(rng() % 6);
    std::vector<int32_t> lab(n), s(m), l(m), d(m);
    for (auto& x : lab) x = int32_t(rng() % 4);
    for (int e = 0; e < m; ++e) {
      s[e] = int32_t(rng() % n);
      l[e] = int32_t(rng() % 3);
      d[e] = int32_t(rng() % n);
    }
    std::vector<int32_t> pid(n), hist(size_t(k + 1) * n), rd(1);
    std::vector<int64_t> counts(k + 1), msi(k + 1);
    for (int32_t flags = 0; flags < 8; ++flags)
      bad += oracle_refine(n, m, lab.data(), s.data(), l.data(), d.data(), k, flags, pid.data(), counts.data(),
                           msi.data(), hist.data(), rd.data()) != 0;
    std::vector<int32_t> sample = {0, int32_t(n - 1), int32_t(n / 2)};
    std::vector<int64_t> off(4);
    bad += oracle_signatures(n, m, s.data(), l.data(), d.data(), pid.data(), 3, sample.data(), off.data(), nullptr);
    std::vector<int32_t> buf(static_cast<size_t>(off[3]) + 1);
    bad += oracle_signatures(n, m, s.data(), l.data(), d.data(), pid.data(), 3, sample.data(), off.data(), buf.data());
    std::vector<int64_t> len(n);
    bad += oracle_signature_lengths(n, m, s.data(), l.data(), d.data(), pid.data(), len.data());
    // invalid input is rejected, not read out of bounds
    std::vector<int32_t> bad_d = d;
    if (m) {
      bad_d[0] = n;
      bad += oracle_refine(n, m, lab.data(), s.data(), l.data(), bad_d.data(), k, 0, pid.data(), counts.data(),
                           msi.data(), nullptr, rd.data()) != -1;
    }
    void* st = oracle_state_create(n, lab.data(), m, s.data(), l.data(), d.data(), k);
    if (!st) {
      ++bad;
      continue;
    }
    for (int u = 0; u < 8; ++u) {
      const int64_t cur = oracle_state_num_nodes(st);
      if (cur == 0) break;
      const int kind = int(rng() % 4);
      std::vector<int32_t> a(3), b(3), c(3);
      for (int e = 0; e < 3; ++e) {
        a[e] = int32_t(rng() % cur);
        b[e] = int32_t(rng() % 3);
        c[e] = int32_t(rng() % cur);
      }
      if (kind == 0) {
        std::vector<int32_t> nl = {int32_t(rng() % 5), int32_t(rng() % 5)};
        bad += oracle_state_add_nodes(st, 2, nl.data()) != 0;
      } else if (kind == 1) {
        bad += oracle_state_add_edges(st, 3, a.data(), b.data(), c.data()) != 0;
      } else if (kind == 2) {
        bad += oracle_state_delete_edges(st, 3, a.data(), b.data(), c.data()) != 0;
      } else {
        bad += oracle_state_delete_nodes(st, 1, a.data()) != 0;
      }
      int64_t ch = 0, cg = 0;
      oracle_state_work(st, &ch, &cg);
      std::vector<int32_t> h(size_t(k + 1) * size_t(oracle_state_num_nodes(st)));
      oracle_state_history(st, h.data());
    }
    oracle_state_destroy(st);
  }
  std::printf("%s: %d failed calls\n", bad ? "FAIL" : "ok", bad);
  return bad ? 1 : 0;
}
