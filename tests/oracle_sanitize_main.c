/* Drives the C oracle through its three entry points on random inputs, for
 * a build with AddressSanitizer and UndefinedBehaviorSanitizer (compiled by
 * tests/test_oracle_sanitized.py).  Checks, on every case:
 *   - the cell-based oracle and the all-pairs oracle give the same labels
 *     and core flags (one thread and several);
 *   - a point is core exactly when its closed eps-ball holds MinPts points
 *     or more (Definition 1), from the all-pairs neighbour count.
 * Inputs: empty and one-point sets, duplicates, every d from 1 to 8,
 * coordinates up to +-2^24, eps from 1 to beyond the data's extent, and
 * MinPts from 1 to n + 1.  Exit status 0 when every case agrees. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_dbscan_brute(const int32_t *X, int64_t n, int32_t d, int64_t eps, int64_t minpts, int32_t *labels,
                        uint8_t *core);
int oracle_dbscan(const int32_t *X, int64_t n, int32_t d, int64_t eps, int64_t minpts, int32_t *labels,
                  uint8_t *core, int32_t nthreads);
int oracle_neighbor_count_brute(const int32_t *X, int64_t n, int32_t d, int64_t eps, const int64_t *q, int64_t nq,
                                int64_t *out, int32_t nthreads);

/* splitmix64 (Steele, Lea and Flood, 2014) */
static uint64_t rng_state = 0x2210075800000001ull;
static uint64_t next_u64(void) {
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static int64_t uniform(int64_t lo, int64_t hi) { /* in [lo, hi] */
    return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1));
}

static int run_case(int c, int64_t n, int d, int64_t extent, int64_t eps, int64_t minpts) {
    int32_t *x = malloc(sizeof(int32_t) * (size_t)(n * d + 1));
    int32_t *la = malloc(sizeof(int32_t) * (size_t)(n + 1)), *lb = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *lc = malloc(sizeof(int32_t) * (size_t)(n + 1));
    uint8_t *ca = malloc((size_t)n + 1), *cb = malloc((size_t)n + 1), *cc = malloc((size_t)n + 1);
    int64_t *q = malloc(sizeof(int64_t) * (size_t)(n + 1)), *cnt = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int bad = 0;
    for (int64_t i = 0; i < n * d; ++i) x[i] = (int32_t)uniform(-extent, extent);
    for (int64_t i = 1; i < n; i += 3) /* duplicates */
        if (uniform(0, 1)) memcpy(x + i * d, x + (i - 1) * d, sizeof(int32_t) * (size_t)d);
    for (int64_t i = 0; i < n; ++i) q[i] = i;
    if (oracle_dbscan_brute(x, n, d, eps, minpts, la, ca) != 0 || oracle_dbscan(x, n, d, eps, minpts, lb, cb, 1) != 0 ||
        oracle_dbscan(x, n, d, eps, minpts, lc, cc, 3) != 0 ||
        oracle_neighbor_count_brute(x, n, d, eps, q, n, cnt, 2) != 0) {
        fprintf(stderr, "case %d: an entry point failed\n", c);
        bad = 1;
    }
    for (int64_t i = 0; i < n && !bad; ++i) {
        if (la[i] != lb[i] || la[i] != lc[i] || ca[i] != cb[i] || ca[i] != cc[i]) {
            fprintf(stderr, "case %d (n %lld d %d eps %lld minpts %lld): point %lld differs\n", c, (long long)n, d,
                    (long long)eps, (long long)minpts, (long long)i);
            bad = 1;
        } else if ((cnt[i] >= minpts) != (ca[i] != 0)) {
            fprintf(stderr, "case %d: point %lld has %lld neighbours, core %d\n", c, (long long)i,
                    (long long)cnt[i], ca[i]);
            bad = 1;
        }
    }
    free(x);
    free(la);
    free(lb);
    free(lc);
    free(ca);
    free(cb);
    free(cc);
    free(q);
    free(cnt);
    return bad;
}

int main(void) {
    int bad = 0, c = 0;
    bad |= run_case(c++, 0, 2, 10, 3, 1);
    bad |= run_case(c++, 1, 3, 10, 3, 1);
    bad |= run_case(c++, 1, 3, 10, 3, 2);
    bad |= run_case(c++, 40, 8, 1 << 24, 1 << 24, 3);  /* coordinates at the accepted bound */
    bad |= run_case(c++, 40, 1, 1 << 24, 1, 1);
    for (; c < 160; ++c) {
        const int d = (int)uniform(1, 8);
        const int64_t n = uniform(2, 450);
        const int64_t extent = uniform(1, 400);
        const int64_t eps = uniform(1, extent + 20);
        const int64_t choice[6] = {1, 2, 3, 5, n / 3 + 1, n + 1};
        bad |= run_case(c, n, d, extent, eps, choice[uniform(0, 5)]);
    }
    printf("%d cases, %s\n", c, bad ? "MISMATCH" : "all agree");
    return bad;
}
