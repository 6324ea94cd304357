// Host driver for tests/test_resid_host.py: reads lines of
// "fp32 s0 s1 s2 s3 s4 s5" (the reduced residual sums of one call) from stdin
// and prints "eps0 eps1 eps2 rel0 rel1 rel2 diverged" after each, with one
// divergence watch over the whole sequence (factor 1e6, as the library uses).
#include <cstdio>

#include "gsis_resid_host.h"

int main()
{
    gsis::DivWatch w;
    int fp32;
    double s[6];
    while (std::scanf("%d %lf %lf %lf %lf %lf %lf", &fp32, &s[0], &s[1], &s[2], &s[3], &s[4], &s[5]) == 7) {
        const gsis::ResidEval r = gsis::resid_eval(s, fp32 != 0);
        const bool d = gsis::resid_diverged(w, r, 1e6);
        std::printf("%.17g %.17g %.17g %d %d %d %d\n", r.eps[0], r.eps[1], r.eps[2], (int)r.relative[0],
                    (int)r.relative[1], (int)r.relative[2], (int)d);
    }
    return 0;
}
