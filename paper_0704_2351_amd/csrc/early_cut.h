// Cut schedule of early termination (the outlook of the paper's conclusion): the decision taken after each
// chunk of the sigma-basis that runs beside the sequence.  Plain C++ with no device code, so that the host
// tests can compile it on its own.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace bwr {

struct EarlyCutState {
    int64_t prev_sum = -1;  // the generator rows' degree sum at the previous cut (-1 before the first)
    int64_t prev_cut = 0;   // order of the previous cut
    int64_t vstep = 0;      // length of the next confirming cut
};

struct EarlyCutDecision {
    bool converged = false;  // the basis of order `done` holds the generator
    int64_t next_cut = -1;   // order of the next cut (-1: none, converged or at L)
};

// deg: the 2s shifted row degrees of the order-`done` basis.  The generator rows are the s of least degree.
// Converged when their degree sum equals the previous cut's and at least `verify` orders lie between the two
// cuts.  Otherwise the next cut is `step` orders on, or only st->vstep orders on once the other rows' degrees
// exceed the generator rows' by s * verify in sum (they have taken the pivots for that long); a confirming cut
// that does not confirm doubles st->vstep, up to `step`.
inline EarlyCutDecision early_cut_after_chunk(const int64_t* deg, int s, int64_t done, int64_t L, int64_t step,
                                              int64_t verify, EarlyCutState* st) {
    std::vector<int64_t> d(deg, deg + 2 * s);
    std::sort(d.begin(), d.end());
    int64_t small = 0, all = 0;
    for (int i = 0; i < 2 * s; ++i) {
        all += d[i];
        if (i < s) small += d[i];
    }
    EarlyCutDecision out;
    if (st->prev_sum >= 0 && small == st->prev_sum && done - st->prev_cut >= verify) {
        out.converged = true;
        return out;
    }
    st->prev_sum = small;
    st->prev_cut = done;
    if (done < L) {
        const bool stalled = (all - small) - small >= (int64_t)s * verify;
        int64_t next = step;
        if (stalled) {
            next = st->vstep;
            st->vstep = std::min(step, 2 * st->vstep);
        }
        out.next_cut = std::min(L, done + next);
    }
    return out;
}

}  // namespace bwr
