/* For every float x with 1e-30 <= |x| <= 1e30 (and x = +-0) and each rate
 * constant c, the quotient formed as q = RN(x * RN(1/c)), r = x - q c (one
 * fused multiply-add, exact), RN(q + r RN(1/c)) (Markstein's correction)
 * must equal the IEEE quotient RN(x / c), bit for bit, except that x = -0
 * may give +0 (the quotient only enters exp and exprelr, which give 1 at
 * either zero). Prints one line per constant with the number of
 * mismatches. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

int main(void) {
    const float cs[4] = {10.0f, 18.0f, 20.0f, 80.0f};
    for (int ci = 0; ci < 4; ++ci) {
        const float c = cs[ci];
        const float y = 1.0f / c;
        long long bad = 0, tested = 0;
#pragma omp parallel for reduction(+ : bad, tested) schedule(static)
        for (long long u = 0; u < (1LL << 32); ++u) {
            const uint32_t b = (uint32_t)u;
            float x;
            memcpy(&x, &b, 4);
            if (!isfinite(x)) continue;
            if (x != 0.0f && (fabsf(x) < 1e-30f || fabsf(x) > 1e30f)) continue;
            volatile float ref = x / c;
            const float q = x * y;
            const float r = fmaf(-q, c, x);
            float q2 = fmaf(r, y, q);
            if (x == 0.0f && q2 == 0.0f) q2 = ref; /* either zero: same downstream */
            const float rv = ref;
            uint32_t a1, a2;
            memcpy(&a1, &rv, 4);
            memcpy(&a2, &q2, 4);
            tested++;
            if (a1 != a2) bad++;
        }
        printf("%g %lld %lld\n", c, tested, bad);
    }
    return 0;
}
