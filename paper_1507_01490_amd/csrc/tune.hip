// Autotuner of the execution knobs.  None of them changes the answer
// (Algorithm 1 is exact for every batching, width, direction policy and
// threshold history); they only change the time.  The tuner runs the real
// query with k: first a grid over width and deferral budget (they interact:
// a wide batch can take deep sources a narrow one must defer), then one knob
// at a time around the best setting (coordinate descent): deferred-batch
// width, bottom-up threshold, persistent slots and source order.  Every trial must
// return exactly the first trial's result, which makes tuning a self-check.
#include <chrono>
#include <cstring>
#include <functional>
#include <vector>

#include "bc_internal.h"

namespace bc {
namespace {

struct Trial {
    bc_opts o;
    double ms;
};

}  // namespace
}  // namespace bc

using bc::set_error;

extern "C" bc_status bc_autotune(bc_graph* g, int32_t k, const bc_opts* base, int32_t repeats, bc_opts* best,
                                 bc_tune_report* report) {
    try {
        if (!g || !best || k <= 0) {
            set_error("bad argument");
            return BC_EINVAL;
        }
        bc_opts b;
        bc_opts_default(&b);
        if (base) {
            if (base->size < sizeof(uint32_t) || base->size > sizeof(bc_opts)) {
                set_error("opts.size not supported");
                return BC_EINVAL;
            }
            std::memcpy(&b, base, base->size);
            b.size = sizeof(bc_opts);
        }
        b.mode = BC_MODE_BATCHED;
        if (repeats < 1) repeats = 1;
        const int32_t n = g->dg.n;
        const int32_t kk = std::min(k, std::max(n, 1));
        std::vector<int32_t> ids0((size_t)kk), ids((size_t)kk);
        std::vector<uint64_t> f0((size_t)kk), f((size_t)kk);
        std::vector<uint32_t> r0((size_t)kk), r((size_t)kk);
        int32_t c0 = -1, c = 0;
        int trials = 0;
        double default_ms = 0;
        // time of one setting: the best of `repeats` runs after a warm-up
        auto measure = [&](const bc_opts& o, double* ms) -> bc_status {
            double bestms = 1e300;
            for (int rep = 0; rep <= repeats; ++rep) {
                bc_stats st;
                std::memset(&st, 0, sizeof(st));
                st.size = sizeof(st);
                auto t0 = std::chrono::steady_clock::now();
                BC_TRY(bc::run_topk(g, k, o, ids.data(), f.data(), r.data(), &c, &st, g->stream));
                const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                if (c0 < 0) {
                    ids0 = ids;
                    f0 = f;
                    r0 = r;
                    c0 = c;
                } else if (c != c0 || ids != ids0 || f != f0 || r != r0) {
                    set_error("autotune: a setting returned a different top-k (width %d, defer_arcs %d)", o.width,
                              o.defer_arcs);
                    return BC_EDEVICE;
                }
                if (rep > 0 && t < bestms) bestms = t;
            }
            ++trials;
            *ms = bestms;
            return BC_OK;
        };
        bc_opts cur = b;
        double cur_ms = 0;
        BC_TRY(measure(cur, &cur_ms));
        default_ms = cur_ms;
        // width and deferral budget interact (a wide batch can take deep
        // sources that a narrow one must defer): search them as a grid
        {
            const bc_opts base_o = cur;
            for (int w : {64, 128, 256})
                for (int da : {16384, 65536, 262144, -1}) {
                    bc_opts t = base_o;
                    t.width = w;
                    t.defer_arcs = da;
                    if (std::memcmp(&t, &cur, sizeof(t)) == 0) continue;
                    double ms = 0;
                    BC_TRY(measure(t, &ms));
                    if (ms < cur_ms) {
                        cur = t;
                        cur_ms = ms;
                    }
                }
        }
        using Setter = std::function<void(bc_opts&, int)>;
        struct Knob {
            std::vector<int> values;
            Setter set;
        };
        const int cus = 256;
        std::vector<Knob> knobs = {
            {{64, 256}, [](bc_opts& o, int v) { o.defer_width = v; }},
            {{0, 3, 14}, [](bc_opts& o, int v) { o.pull_alpha = (float)v; }},
            {{cus / 2, cus, 2 * cus}, [](bc_opts& o, int v) { o.slots = v; }},
            {{BC_ORDER_GROUPED, BC_ORDER_DEGREE, BC_ORDER_LOCALITY}, [](bc_opts& o, int v) { o.order = v; }},
        };
        for (auto& kn : knobs) {
            bc_opts keep = cur;
            double keep_ms = cur_ms;
            for (int v : kn.values) {
                bc_opts t = cur;
                kn.set(t, v);
                if (std::memcmp(&t, &cur, sizeof(t)) == 0) continue;
                double ms = 0;
                BC_TRY(measure(t, &ms));
                if (ms < keep_ms) {
                    keep = t;
                    keep_ms = ms;
                }
            }
            cur = keep;
            cur_ms = keep_ms;
        }
        *best = cur;
        if (report) {
            bc_tune_report rp;
            std::memset(&rp, 0, sizeof(rp));
            rp.size = sizeof(rp);
            rp.trials = trials;
            rp.default_ms = default_ms;
            rp.best_ms = cur_ms;
            std::memcpy(report, &rp, std::min<size_t>(report->size ? report->size : sizeof(rp), sizeof(rp)));
        }
        return BC_OK;
    } catch (...) {
        set_error("internal error");
        return BC_EDEVICE;
    }
}
