// Optimal checkpointing schedule for reversing a chain of `steps` time steps
// with `snaps` stored states (Griewank and Walther's binomial checkpointing,
// the "revolve" the paper uses to bound the memory of the gradient; Section
// "Discrete adjoint wave-equation and FWI gradient").
//
// Model: state x_0 is held in a snapshot on entry; reversing step i needs
// x_i in memory; an advance x_i -> x_{i+1} costs one forward step; taking or
// restoring a snapshot costs nothing (states are buffers that are pinned or
// re-pointed, never copied). With s snapshots (x_0's included) the minimal
// number of advances for l steps is
//     t(l, s) = r l - C(s + r, r - 1),
// r the smallest integer with C(s + r, s) >= l. The schedule below splits a
// segment at the point that keeps the cost of both halves at that minimum:
//     T(l, s) = min_{0 < m < l} [ m + T(l - m, s - 1) + T(m, s) ].
#include <algorithm>
#include <cstdint>
#include <functional>
#include <limits>
#include <vector>

#include "runtime.h"

namespace wf {

namespace {

// C(n, k) saturated at ~1e18
int64_t binom_sat(int64_t n, int64_t k) {
    if (k < 0 || k > n) return 0;
    k = std::min(k, n - k);
    long double r = 1.0L;
    for (int64_t i = 1; i <= k; ++i) {
        r = r * (long double)(n - k + i) / (long double)i;
        if (r > 1e18L) return (int64_t)1e18;
    }
    return (int64_t)(r + 0.5L);
}

}  // namespace

int64_t revolve_cost(int64_t l, int s) {
    if (l < 1 || s < 1) return -1;
    if (l == 1) return 0;
    int64_t r = 1;
    while (binom_sat(s + r, s) < l) ++r;
    return r * l - binom_sat(s + r, r - 1);
}

wf_status revolve_schedule(int64_t steps, int snaps, std::vector<RevolveAction>& out) {
    out.clear();
    if (steps < 1 || snaps < 1) return fail(WF_E_ARG, "revolve needs steps >= 1 and snaps >= 1");
    // current position of the in-memory state, and which snapshot slots are used
    int64_t cur = 0;
    std::vector<int> free_slots;
    for (int i = snaps - 1; i >= 1; --i) free_slots.push_back(i);   // slot 0 holds x_0
    out.push_back({RevolveAction::TAKESHOT, 0, 0});

    // reverse steps [a, a + len), the state x_a being stored in `slot`
    std::function<void(int64_t, int64_t, int, int)> rev = [&](int64_t a, int64_t len, int s, int slot) {
        if (len == 1) {
            if (cur != a) {
                out.push_back({RevolveAction::RESTORE, a, slot});
                cur = a;
            }
            out.push_back({RevolveAction::REVERSE, a, a});
            return;
        }
        if (s == 1) {
            for (int64_t i = a + len - 1; i >= a; --i) {
                if (cur != a) out.push_back({RevolveAction::RESTORE, a, slot});
                cur = a;
                if (i > a) {
                    out.push_back({RevolveAction::ADVANCE, a, i});
                    cur = i;
                }
                out.push_back({RevolveAction::REVERSE, i, i});
            }
            return;
        }
        // choose the split m minimising m + t(len - m, s - 1) + t(m, s)
        const int64_t target = revolve_cost(len, s);
        int64_t best_m = 1, best = std::numeric_limits<int64_t>::max();
        for (int64_t m = 1; m < len; ++m) {
            const int64_t c = m + revolve_cost(len - m, s - 1) + revolve_cost(m, s);
            if (c < best) {
                best = c;
                best_m = m;
                if (c == target) break;
            }
        }
        const int64_t m = best_m;
        if (cur != a) {
            out.push_back({RevolveAction::RESTORE, a, slot});
            cur = a;
        }
        out.push_back({RevolveAction::ADVANCE, a, a + m});
        cur = a + m;
        const int ns = free_slots.back();
        free_slots.pop_back();
        out.push_back({RevolveAction::TAKESHOT, a + m, ns});
        rev(a + m, len - m, s - 1, ns);
        out.push_back({RevolveAction::FREE, a + m, ns});
        free_slots.push_back(ns);
        rev(a, m, s, slot);
    };
    rev(0, steps, std::min<int64_t>(snaps, steps), 0);
    out.push_back({RevolveAction::FREE, 0, 0});
    return WF_OK;
}

}  // namespace wf

extern "C" int64_t wf_revolve_schedule(int64_t steps, int snaps, int32_t* kind, int64_t* at,
                                       int64_t* arg, int64_t cap) {
    try {
        std::vector<wf::RevolveAction> acts;
        const wf_status st = wf::revolve_schedule(steps, snaps, acts);
        if (st != WF_OK) return st;
        const int64_t n = (int64_t)acts.size();
        if (cap > 0 && (!kind || !at || !arg)) return wf::fail(WF_E_ARG, "NULL output array");
        for (int64_t i = 0; i < std::min(n, cap); ++i) {
            kind[i] = (int32_t)acts[(size_t)i].kind;
            at[i] = acts[(size_t)i].at;
            arg[i] = acts[(size_t)i].arg;
        }
        return n;
    } catch (...) {
        return wf::fail(WF_E_NOMEM, "host allocation failed");
    }
}
