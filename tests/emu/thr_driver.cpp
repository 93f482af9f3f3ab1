// Host build of the library's term thresholds (test infrastructure): reads
// lines "a b max_l retention limit" and prints the entry's two 8-bit codes
// and their decoded probabilities, from the same source the kernels use.
#include <hip/hip_runtime.h>
#include "../../paper_1310_2274_amd/csrc/ara_math.hpp"
#include <cstdio>

int main()
{
    double a, b, m, ret, lim;
    while (std::scanf("%lf %lf %lf %lf %lf", &a, &b, &m, &ret, &lim) == 5) {
        ara::EntryRec E{};
        E.a = a;
        E.b = b;
        E.lnB = a == 0.0 ? m : ara::log_beta(a, b);     // a == 0: degenerate, the loss is its mean (here m)
        E.maxl = (float)m;
        const ara::TermThr t = ara::term_thresholds(E, ret, lim);
        std::printf("%u %u %.9g %.9g\n", (unsigned)(t & 0xFFu), (unsigned)(t >> 8), (double)ara::thr_lo(t),
                    (double)ara::thr_hi(t));
    }
    return 0;
}
