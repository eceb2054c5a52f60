// What one convergence check decides for an instance: stop, go on, or end a
// single-precision phase.  Host code, free of device state, so that every
// branch can be exercised without a GPU.
//
// Stop rules (Algorithm 1 evaluates convergence every M sweeps): 0 is r < tol
// on the steady residual; 1 is the relative change of |q| between checks,
// eps_q < tol, the criterion of the paper's large-domain runs (§7.1).
#pragma once

#include <cstddef>

namespace ps {

// One reading of the FP32 floor's plateau test on a phase's residual history
// h[0..n).  With r_n ~ r_inf + C rho^n, Aitken's extrapolation of three
// residuals K checks apart estimates r_inf: the reading is a hit once most of
// the current r is that limit (above 0.8 of it), or when r did not fall over
// either K-check span.  Multi-rate decay can fool one estimate, so the engine
// asks for two consecutive hits.
inline bool plateau_reading(const double *h, size_t n, size_t K = 5)
{
    if (n < 2 * K + 1) return false;
    const double a = h[n - 1 - 2 * K], b = h[n - 1 - K], c = h[n - 1];
    if (!(b < a) || !(c < b)) return true;  // no progress over K checks
    const double d1 = b - a, d2 = c - b, den = d2 - d1;
    return den > 0 && (c - d2 * d2 / den) > 0.8 * c;
}

enum class CheckAction {
    Continue,      // sweep on
    Stop,          // status OK
    NotConverged,  // status NOT_CONVERGED: budget spent, or plain FP32 at its floor
    Promote,       // the state continues in FP64 sweeps
    ToCorrection,  // the FP32 state becomes s0 of the correction form
};

struct CheckState {
    bool dc;            // precision PM_FP32_DC
    bool fp32_phase;    // the iterate is FP32 (FP32 phase or correction form)
    bool delta;         // the correction form
    int stop_rule;      // 0: r < tol, 1: eps_q < tol
    int dc_form;        // 0: correction form after the FP32 phase, 1: promotion
    double tol;
    double r;           // this check's residual
    double eps;         // this check's eps_q (infinite at a phase's first check)
    bool near_floor;    // r within three decades of the estimated FP32 floor
    int stall;          // checks since the phase's last new minimum of r (0: this one)
    bool plateau;       // the plateau test of the phase's r history fired
    bool budget_spent;  // max_sweeps reached
};

inline CheckAction decide(const CheckState &c)
{
    // Near its floor an FP32 iterate stagnates: q stops changing and eps_q
    // reads 0 without convergence, so there eps_q does not count as meeting
    // the rule.
    const bool met = c.stop_rule == 0 ? c.r < c.tol : c.eps < c.tol && !(c.fp32_phase && c.near_floor);
    const bool eps_below = c.stop_rule == 1 && c.eps < c.tol;
    // A hand-over to FP64, which then meets the rule by itself, may also
    // follow eps_q near the floor while r still reaches a new minimum, which a
    // stagnating iterate does not (the 1536^3 packing: eps_q < 1e-6 at 40,500
    // FP32 sweeps with r = 1.5e-5, within three decades of its floor and still
    // falling 5 % per 1000 sweeps).
    const bool met_dc = met || (eps_below && c.stall == 0);
    // FP32 rounding stops the updates once dt |F| falls below half an ulp: a
    // plateau counts within three decades of that level, or after 20 checks
    // without a new minimum anywhere.
    const bool floor = c.fp32_phase && ((c.near_floor && (c.stall >= 5 || c.plateau)) || c.stall >= 20);
    if (c.dc && c.fp32_phase && c.delta) {
        // correction form: s0 + e meets the rule, or e sits at its own floor
        // (s0 + e continues in FP64).  eps_q < tol that the floor gate does
        // not count also goes on in FP64, which must meet the rule once more
        // (a 512^3 foam ended its budget in this form with eps_q = 1.6e-8 and
        // r still falling).
        if (met) return CheckAction::Stop;
        if (floor || eps_below) return CheckAction::Promote;
    } else if (c.dc && c.fp32_phase) {
        // FP32 phase: hand over once the iterate meets the rule (FP64 confirms
        // it) or sits at its floor.  eps_q < tol near the floor without a new
        // minimum of r is stagnation or a noisy but converging r (a 512^3 foam
        // along x ran 304,200 sweeps where y and z met the rule at 160,000):
        // the phase ends either way, as at the floor, and s0 + e must meet the
        // rule again.
        if (met_dc) return CheckAction::Promote;
        if (floor || eps_below) return c.dc_form == 1 ? CheckAction::Promote : CheckAction::ToCorrection;
    } else if (met) {
        return CheckAction::Stop;
    }
    if (!c.dc && floor) return CheckAction::NotConverged;  // plain FP32: its floor lies above tol
    if (c.budget_spent) return CheckAction::NotConverged;
    return CheckAction::Continue;
}

}  // namespace ps
