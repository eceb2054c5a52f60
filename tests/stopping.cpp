// Host check of the library's convergence decision (csrc/stopping.h): one case
// per branch, each with the action the stop rules and the precision forms call
// for.  Prints "ok <cases>" or the first case that differs.
#include <cmath>
#include <cstdio>

#include "stopping.h"

using ps::CheckAction;
using ps::CheckState;

static int cases = 0;

static CheckState base()
{
    CheckState c{};
    c.stop_rule = 0;
    c.tol = 1e-8;
    c.r = 1e-3;
    c.eps = 1e-2;
    return c;
}

static const char *name(CheckAction a)
{
    switch (a) {
    case CheckAction::Continue: return "Continue";
    case CheckAction::Stop: return "Stop";
    case CheckAction::NotConverged: return "NotConverged";
    case CheckAction::Promote: return "Promote";
    case CheckAction::ToCorrection: return "ToCorrection";
    }
    return "?";
}

static bool expect(const char *what, const CheckState &c, CheckAction want)
{
    ++cases;
    const CheckAction got = ps::decide(c);
    if (got != want) {
        std::printf("%s: got %s, want %s\n", what, name(got), name(want));
        return false;
    }
    return true;
}

static bool expect_reading(const char *what, const double *h, size_t n, bool want)
{
    ++cases;
    const bool got = ps::plateau_reading(h, n);
    if (got != want) {
        std::printf("%s: reading %d, want %d\n", what, got, want);
        return false;
    }
    return true;
}

int main()
{
    bool ok = true;
    // ---- plateau reading of the residual history (K = 5: checks n-11, n-6, n-1)
    {
        double h[31];
        for (int k = 0; k < 31; ++k) h[k] = std::pow(0.9, k);
        ok &= expect_reading("ten checks are too few", h, 10, false);
        ok &= expect_reading("geometric decay to zero", h, 11, false);
        ok &= expect_reading("geometric decay to zero, late", h, 31, false);
        for (int k = 0; k < 31; ++k) h[k] = 1e-3 + 1e-3 * std::pow(0.9, k);
        ok &= expect_reading("decay onto a floor, early (limit below 0.8 r)", h, 11, false);
        ok &= expect_reading("decay onto a floor, late (limit above 0.8 r)", h, 31, true);
        for (int k = 0; k < 31; ++k) h[k] = 2e-5;
        ok &= expect_reading("flat", h, 31, true);
        for (int k = 0; k < 31; ++k) h[k] = 1e-5 * (1.0 + 0.01 * k);
        ok &= expect_reading("rising", h, 31, true);
        for (int k = 0; k < 31; ++k) h[k] = std::pow(0.9, k);
        h[30] = 1.05 * h[25];
        ok &= expect_reading("last check above the one K before", h, 31, true);
        h[30] = 0.95 * h[25];
        ok &= expect_reading("decay that slows sharply over the last K checks", h, 31, true);
    }
    // ---- FP64: the rule as written, no floor gate
    {
        CheckState c = base();
        ok &= expect("fp64 far from tol", c, CheckAction::Continue);
        c.r = 0.5e-8;
        ok &= expect("fp64 r < tol", c, CheckAction::Stop);
        c.r = 1e-8;
        ok &= expect("fp64 r == tol is not below", c, CheckAction::Continue);
        c = base();
        c.stop_rule = 1;
        c.tol = 1e-6;
        c.eps = 5e-7;
        c.near_floor = true;  // no meaning outside single precision
        c.stall = 7;
        ok &= expect("fp64 eps < tol", c, CheckAction::Stop);
        c.eps = INFINITY;
        ok &= expect("fp64 first check of a phase", c, CheckAction::Continue);
        c.budget_spent = true;
        ok &= expect("fp64 budget", c, CheckAction::NotConverged);
        c.eps = 5e-7;
        ok &= expect("fp64 meets the rule on its last sweep", c, CheckAction::Stop);
    }
    // ---- plain FP32: eps_q near the floor never stops it; the floor ends it
    {
        CheckState c = base();
        c.fp32_phase = true;
        c.stop_rule = 1;
        c.tol = 1e-6;
        c.eps = 0.0;
        c.near_floor = true;
        c.stall = 0;
        ok &= expect("fp32 eps 0 near the floor, new minimum", c, CheckAction::Continue);
        c.near_floor = false;
        ok &= expect("fp32 eps < tol away from the floor", c, CheckAction::Stop);
        c.near_floor = true;
        c.stall = 5;
        ok &= expect("fp32 floor after 5 checks without a minimum", c, CheckAction::NotConverged);
        c.stall = 1;
        c.plateau = true;
        ok &= expect("fp32 floor by the plateau test", c, CheckAction::NotConverged);
        c.plateau = false;
        c.eps = 1e-2;
        c.near_floor = false;
        c.stall = 19;
        ok &= expect("fp32 far above the floor, 19 checks", c, CheckAction::Continue);
        c.stall = 20;
        ok &= expect("fp32 20 checks without a minimum", c, CheckAction::NotConverged);
        c = base();
        c.fp32_phase = true;
        c.r = 0.5e-8;
        c.near_floor = true;
        ok &= expect("fp32 r < tol", c, CheckAction::Stop);
    }
    // ---- FP32-DC, FP32 phase
    {
        CheckState c = base();
        c.dc = true;
        c.fp32_phase = true;
        c.r = 0.5e-8;
        ok &= expect("dc r < tol: FP64 confirms", c, CheckAction::Promote);
        c.r = 1e-3;
        c.near_floor = true;
        c.stall = 5;
        ok &= expect("dc floor: correction form", c, CheckAction::ToCorrection);
        c.dc_form = 1;
        ok &= expect("dc floor, dc_form 1", c, CheckAction::Promote);
        c = base();
        c.dc = true;
        c.fp32_phase = true;
        c.stop_rule = 1;
        c.tol = 1e-6;
        c.eps = 9e-7;
        c.near_floor = true;
        c.stall = 0;
        ok &= expect("dc eps < tol near the floor, r falling", c, CheckAction::Promote);
        c.stall = 2;
        ok &= expect("dc eps < tol near the floor, no new minimum", c, CheckAction::ToCorrection);
        c.dc_form = 1;
        ok &= expect("dc the same, dc_form 1", c, CheckAction::Promote);
        c.dc_form = 0;
        c.near_floor = false;
        ok &= expect("dc eps < tol away from the floor", c, CheckAction::Promote);
        c.eps = 2e-6;
        c.near_floor = true;
        c.stall = 0;
        ok &= expect("dc eps above tol", c, CheckAction::Continue);
        c.budget_spent = true;
        ok &= expect("dc budget in the FP32 phase", c, CheckAction::NotConverged);
    }
    // ---- FP32-DC, correction form
    {
        CheckState c = base();
        c.dc = true;
        c.fp32_phase = true;
        c.delta = true;
        c.r = 0.5e-8;
        ok &= expect("correction r < tol", c, CheckAction::Stop);
        c.r = 1e-6;
        c.near_floor = true;
        c.stall = 5;
        ok &= expect("correction at its floor: FP64", c, CheckAction::Promote);
        c.stall = 0;
        ok &= expect("correction near its floor, falling", c, CheckAction::Continue);
        c = base();
        c.dc = true;
        c.fp32_phase = true;
        c.delta = true;
        c.stop_rule = 1;
        c.tol = 1e-6;
        c.eps = 5e-7;
        ok &= expect("correction eps < tol away from its floor", c, CheckAction::Stop);
        c.near_floor = true;
        ok &= expect("correction eps < tol near its floor: FP64 confirms", c, CheckAction::Promote);
        c.eps = INFINITY;
        c.near_floor = false;
        ok &= expect("correction first check", c, CheckAction::Continue);
        c.budget_spent = true;
        ok &= expect("correction budget", c, CheckAction::NotConverged);
    }
    // ---- FP32-DC after promotion: FP64 rules
    {
        CheckState c = base();
        c.dc = true;
        c.stop_rule = 1;
        c.tol = 1e-6;
        c.eps = 5e-7;
        c.near_floor = true;
        c.stall = 9;
        ok &= expect("promoted eps < tol", c, CheckAction::Stop);
        c.eps = 5e-6;
        c.stall = 30;
        ok &= expect("promoted: no floor in FP64", c, CheckAction::Continue);
    }
    // ---- invariants over every combination of flags, counts and levels
    int combos = 0;
    const int stalls[] = {0, 1, 4, 5, 19, 20};
    const double rs[] = {0.5e-8, 1e-3};                       // below / above tol 1e-8 (rule 0)
    const double epss[] = {0.0, 0.5e-6, 2e-6, INFINITY};       // against tol 1e-6 (rule 1)
    for (int bits = 0; bits < 64; ++bits)
        for (int rule = 0; rule < 2; ++rule)
            for (int form = 0; form < 2; ++form)
                for (int st : stalls)
                    for (double r : rs)
                        for (double e : epss) {
                            CheckState c{};
                            c.dc = bits & 1;
                            c.fp32_phase = bits & 2;
                            c.delta = bits & 4;
                            c.near_floor = bits & 8;
                            c.plateau = bits & 16;
                            c.budget_spent = bits & 32;
                            if (c.delta && !(c.dc && c.fp32_phase)) continue;  // no such state
                            c.stop_rule = rule;
                            c.dc_form = form;
                            c.tol = rule == 0 ? 1e-8 : 1e-6;
                            c.stall = st;
                            c.r = r;
                            c.eps = e;
                            ++combos;
                            const CheckAction a = ps::decide(c);
                            const bool rule_met = rule == 0 ? r < c.tol : e < c.tol;
                            bool good = true;
                            // a spent budget ends the solve or its phase
                            good &= !(c.budget_spent && a == CheckAction::Continue);
                            // Stop only where the rule holds; in single precision
                            // under eps_q never near the floor; never from the FP32
                            // phase of FP32-DC, which a later phase must confirm
                            if (a == CheckAction::Stop) {
                                good &= rule_met;
                                good &= !(rule == 1 && c.fp32_phase && c.near_floor);
                                good &= !(c.dc && c.fp32_phase && !c.delta);
                            }
                            // phase changes only from single precision under FP32-DC;
                            // the correction form only from the FP32 phase, dc_form 0
                            if (a == CheckAction::Promote) good &= c.dc && c.fp32_phase;
                            if (a == CheckAction::ToCorrection)
                                good &= c.dc && c.fp32_phase && !c.delta && form == 0;
                            // FP64 ignores the floor signals
                            if (!c.fp32_phase) {
                                CheckState d = c;
                                d.near_floor = !c.near_floor;
                                d.plateau = !c.plateau;
                                d.stall = c.stall == 0 ? 20 : 0;
                                good &= ps::decide(d) == a;
                            }
                            // in single precision, eps_q < tol always ends the phase
                            // under FP32-DC
                            if (c.dc && c.fp32_phase && rule == 1 && e < c.tol)
                                good &= a == CheckAction::Stop || a == CheckAction::Promote ||
                                        a == CheckAction::ToCorrection;
                            if (!good) {
                                std::printf("invariant broken: dc %d fp32 %d delta %d near %d plateau %d budget %d "
                                            "rule %d form %d stall %d r %g eps %g -> %s\n",
                                            c.dc, c.fp32_phase, c.delta, c.near_floor, c.plateau, c.budget_spent,
                                            rule, form, st, r, e, name(a));
                                ok = false;
                            }
                        }
    if (!ok) return 1;
    std::printf("ok %d %d\n", cases, combos);
    return 0;
}
