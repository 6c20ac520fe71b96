// Drives the early-termination cut schedule (early_cut.h) over model degree profiles, for the host tests.
// argv: L s d step verify creep.  Model of the order-c basis of [S; -I] (2s rows, degrees summing to s (c + 1)):
// generator row i has degree min(ceil(c / 2), d) (row 0 keeps growing by one every `creep` orders past 2d
// when creep > 0), its partner row c + 1 minus that.  Prints every cut, then "conv <order>" or "none".
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "early_cut.h"

int main(int argc, char** argv) {
    if (argc != 7) return 2;
    const int64_t L = atoll(argv[1]), d = atoll(argv[3]);
    const int s = atoi(argv[2]);
    const int64_t step = atoll(argv[4]), verify = atoll(argv[5]), creep = atoll(argv[6]);
    bwr::EarlyCutState st;
    st.vstep = verify;
    int64_t c = std::min(L, std::max(step, L / 8));
    for (;;) {
        std::vector<int64_t> deg(2 * s);
        for (int i = 0; i < s; ++i) {
            int64_t p = std::min<int64_t>((c + 1) / 2, d);
            if (i == 0 && creep > 0 && c > 2 * d) p += (c - 2 * d) / creep;
            deg[i] = p;
            deg[s + i] = c + 1 - p;
        }
        printf("cut %lld\n", (long long)c);
        const bwr::EarlyCutDecision dec = bwr::early_cut_after_chunk(deg.data(), s, c, L, step, verify, &st);
        if (dec.converged) {
            printf("conv %lld\n", (long long)c);
            return 0;
        }
        if (dec.next_cut < 0) {
            printf("none\n");
            return 0;
        }
        c = dec.next_cut;
    }
}
