// Exhaustive host check of the division the per-row tap code uses: for all
// integers 0 <= a <= b, 1 <= b <= 65536 (every numerator and denominator of
// a tap offset t = rem / (2 N_out) or 1 - t with sides up to 32768), is
// fma(fma(-q0, b, a), y, q0) with y = RN(1/b), q0 = RN(a y) equal to the
// correctly rounded a / b? Host float division and fmaf are IEEE correctly
// rounded, as the GPU's are. Exit status 0 when every pair agrees.
#include <math.h>
#include <stdio.h>
#include <stdint.h>
int main(void)
{
    long long bad = 0, total = 0;
    for (int32_t b = 1; b <= 65536; ++b) {
        const float bf = (float)b;
        const float y = 1.0f / bf;
        for (int32_t a = 0; a <= b; ++a) {
            const float af = (float)a;
            const float want = af / bf;
            const float q0 = af * y;
            const float r = fmaf(-q0, bf, af);
            const float q = fmaf(r, y, q0);
            ++total;
            if (q != want) {
                if (bad < 5) printf("mismatch a=%d b=%d got %.9g want %.9g\n", a, b, q, want);
                ++bad;
            }
        }
    }
    printf("checked %lld pairs, %lld mismatches\n", total, bad);
    return bad != 0;
}
