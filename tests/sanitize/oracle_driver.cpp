// Drives the CPU oracle's entry points on small seeded random graphs and
// motifs, for a build with AddressSanitizer and UndefinedBehaviorSanitizer:
// any invalid access or undefined operation aborts with a report.
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
void* or_graph_new(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                   const int64_t* t, int* status, int nthreads);
void or_graph_free(void* h);
void or_graph_orders(void* h, int32_t*, int32_t*, int32_t*, uint32_t*, uint32_t*);
int or_weights_class(void* h, int64_t delta, const uint8_t* cls, uint32_t*, uint32_t*,
                     uint32_t*, uint32_t*, uint64_t*, int);
int or_anchor(const uint8_t* motif, uint8_t* cls, int32_t* na, int32_t* order, int32_t* aedge);
int or_sample_cls(void*, int64_t, const uint8_t*, const uint32_t*, const uint32_t*,
                  const uint32_t*, const uint32_t*, const uint64_t*, const uint32_t*,
                  const uint8_t*, int, uint64_t, uint64_t, uint32_t, uint64_t, int32_t*, int32_t*,
                  int32_t*, uint64_t*, uint32_t*, uint64_t*, uint64_t*, double*, double*,
                  uint64_t*, int);
int or_enumerate(void*, int64_t, const uint8_t*, const uint32_t*, const uint32_t*,
                 const uint32_t*, const uint32_t*, const uint64_t*, const uint8_t*, int, uint64_t,
                 uint64_t, int32_t*, int32_t*, int32_t*, uint64_t*, uint64_t*, uint64_t*, double*,
                 double*, uint64_t*, int);
int or_brute_count(void*, const uint8_t*, int64_t, uint64_t*, int);
int or_list_lengths(void*, const uint8_t*, int64_t, int32_t, int32_t, int32_t, int64_t*);
int or_check_motif(void*, const uint8_t*, int64_t, int32_t, int32_t, int32_t, uint64_t*);
int or_list_count(const int64_t*, const int64_t*, int, uint64_t*);
void or_features(void*, int64_t, const uint32_t*, const uint32_t*, const uint32_t*,
                 const uint32_t*, double*, int);
int or_proposal_scan(void*, const uint32_t*, const uint32_t*, const uint32_t*, uint64_t*);
}

static uint64_t rng_state = 88172645463325252ull;
static uint64_t next() {  // xorshift64
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 7;
  rng_state ^= rng_state << 17;
  return rng_state;
}

int main() {
  int runs = 0;
  for (int g = 0; g < 6; ++g) {
    const int32_t n = 3 + (int32_t)(next() % 6);
    const int64_t m = 1 + (int64_t)(next() % 40);
    std::vector<int32_t> src(m), dst(m);
    std::vector<int64_t> t(m);
    for (int64_t e = 0; e < m; ++e) {
      src[e] = (int32_t)(next() % n);
      dst[e] = (int32_t)(next() % n);
      t[e] = (int64_t)(next() % 20) - 5;
    }
    int st = 0;
    void* h = or_graph_new(n, m, src.data(), dst.data(), t.data(), &st, 2);
    if (!h) return 2;
    std::vector<int32_t> o1(m), o2(m), o3(m);
    std::vector<uint32_t> f1(n + 1), f2(n + 1);
    or_graph_orders(h, o1.data(), o2.data(), o3.data(), f1.data(), f2.data());
    for (int c = 0; c < 24; ++c) {
      uint8_t cls[4];
      if (c < 16) {
        cls[0] = 1 + (c & 1); cls[1] = (c >> 1) & 1; cls[2] = 1 + ((c >> 2) & 1); cls[3] = (c >> 3) & 1;
      } else {
        const int w = c - 16;
        cls[0] = (w < 4) ? 1 + (w & 1) : 0; cls[1] = (w < 4) ? (w >> 1) & 1 : 0;
        cls[2] = (w >= 4) ? 1 + (w & 1) : 0; cls[3] = (w >= 4) ? ((w >> 1) & 1) : 0;
      }
      for (int64_t delta : {0LL, 3LL, 40LL}) {
        std::vector<uint32_t> lo1(m), a(m), lo3(m), b(m);
        std::vector<uint64_t> S(m + 1);
        or_weights_class(h, delta, cls, lo1.data(), a.data(), lo3.data(), b.data(), S.data(), 2);
        // random motifs of this class drive sampling and enumeration
        for (int tries = 0; tries < 30; ++tries) {
          uint8_t mb[34] = {0};
          const int nv = 3 + (int)(next() % 2);
          const int ne = 2 + (int)(next() % 6);
          mb[0] = (uint8_t)nv;
          mb[1] = (uint8_t)ne;
          for (int i = 0; i < ne; ++i) {
            int x = (int)(next() % nv), y = (int)(next() % nv);
            if (x == y) y = (y + 1) % nv;
            mb[2 + i] = (uint8_t)x;
            mb[18 + i] = (uint8_t)y;
          }
          uint8_t mc[4];
          int32_t na, order[3], ae[3];
          if (or_anchor(mb, mc, &na, order, ae) != 0) continue;
          uint64_t C[2];
          or_brute_count(h, mb, delta, C, 2);
          if (mc[0] != cls[0] || mc[2] != cls[2] || (mc[0] && mc[1] != cls[1]) ||
              (mc[2] && mc[3] != cls[3]))
            continue;
          const uint64_t k = 200;
          std::vector<int32_t> e1(k), e2(k), e3(k);
          std::vector<uint64_t> X(k), cnt(2), hits(1), xm(1);
          std::vector<uint32_t> P(k);
          double est[1], m2[1];
          or_sample_cls(h, delta, cls, lo1.data(), a.data(), lo3.data(), b.data(), S.data(),
                        nullptr, mb, 1, k, 7, 1, 0, e1.data(), e2.data(), e3.data(), X.data(),
                        P.data(), cnt.data(), hits.data(), est, m2, xm.data(), 2);
          const uint64_t W = S[m];
          const uint64_t cntr = W + 3;
          std::vector<int32_t> r1(cntr), r2(cntr), r3(cntr);
          std::vector<uint64_t> RX(cntr);
          or_enumerate(h, delta, cls, lo1.data(), a.data(), lo3.data(), b.data(), S.data(), mb, 1,
                       0, cntr, r1.data(), r2.data(), r3.data(), RX.data(), cnt.data(),
                       hits.data(), est, m2, xm.data(), 2);
          for (uint64_t i = 0; i < (W < 20 ? W : 20); ++i) {
            int64_t lens[16];
            uint64_t x1;
            or_list_lengths(h, mb, delta, r1[i], r2[i], r3[i], lens);
            or_check_motif(h, mb, delta, r1[i], r2[i], r3[i], &x1);
          }
          ++runs;
        }
        if (c == 0) {
          std::vector<double> F(8 * m);
          or_features(h, delta, lo1.data(), a.data(), lo3.data(), b.data(), F.data(), 2);
          std::vector<uint32_t> hq(m, 3);
          std::vector<uint64_t> Q(m + 1);
          or_proposal_scan(h, a.data(), b.data(), hq.data(), Q.data());
        }
      }
    }
    or_graph_free(h);
  }
  // ListCount on random sorted lists, including long chains past 2^64
  std::vector<int64_t> vals, off(14);
  for (int r = 0; r < 13; ++r) {
    off[r] = (int64_t)vals.size();
    for (int i = 0; i < 300; ++i) vals.push_back(r + 13 * i);
  }
  off[13] = (int64_t)vals.size();
  uint64_t X[2];
  or_list_count(vals.data(), off.data(), 13, X);
  std::printf("oracle driver: %d motif runs, big count %llu:%llu\n", runs,
              (unsigned long long)X[1], (unsigned long long)X[0]);
  return runs > 0 ? 0 : 3;
}
