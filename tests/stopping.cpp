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

int main()
{
    bool ok = true;
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
    if (!ok) return 1;
    std::printf("ok %d\n", cases);
    return 0;
}
