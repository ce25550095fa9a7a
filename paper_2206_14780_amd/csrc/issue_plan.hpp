// Host-side planning of the iteration batches of a solve (no device code:
// the host unit test compiles it alone).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "sph.h"

namespace sph {

// The fields of the solver's control block that the host polls between
// batches of iterations, in one contiguous copy: residuals, tolerances,
// states, iteration and halt.
struct CtlPoll {
    double rr[3];
    double bb[3];
    double tau2[3];
    int32_t state[3];
    int32_t iter;
    int32_t halt;
    int32_t halt_reason;
};

// How many iterations the host queues before its next poll of the control
// block.  With nothing known the batches grow 2, 4, 8 (up to kmax).  Two
// polls give each progressing component c a rate of decrease of ln(r.r) per
// iteration (the steeper of the latest interval's and the round's average,
// so that a noisy residual history errs towards short batches; a round
// after a restart starts from the rates of the round before), and from it
// the iterations m_c left to reach its tolerance.  The iteration whose
// p-update halts is then predicted at H = iter + max_c m_c (iter: the last
// p-update polled), and each batch covers half of what is left up to H.
// When every issued iteration already reaches H the host queues nothing
// until the next poll is read (unless none is in flight), so a solve that
// ends as predicted leaves no iteration issued past its halt.  The halting
// iteration itself is always issued (its p-update decides the halt), once
// per round of host-side residual checks.
class IssuePlan {
  public:
    explicit IssuePlan(int kmax) : kmax_(kmax), k_(std::min(2, kmax)) {}

    // a new round after a host-side residual check, whose control block is
    // `m` (restarted components progressing again from their true r.r): the
    // residuals start again, the rates are kept
    void restart(const CtlPoll& m) {
        k_ = std::min(2, kmax_);
        npoll_ = 0;
        have_pred_ = false;
        observe(m);
    }

    void observe(const CtlPoll& m) {
        if (m.halt) return;
        double lrr[3];
        for (int c = 0; c < 3; ++c) lrr[c] = m.rr[c] > 0.0 ? std::log(m.rr[c]) : -HUGE_VAL;
        double horizon = 0.0;
        bool known = true;
        for (int c = 0; c < 3; ++c) {
            if (m.state[c] != SPH_PROGRESSING) continue;
            if (npoll_ >= 1 && m.iter > it_last_ && m.iter > it_first_ && std::isfinite(lrr[c]) &&
                std::isfinite(lrr_last_[c]) && std::isfinite(lrr_first_[c])) {
                const double r_last = (lrr[c] - lrr_last_[c]) / (double)(m.iter - it_last_);
                const double r_avg = (lrr[c] - lrr_first_[c]) / (double)(m.iter - it_first_);
                rate_[c] = std::min(r_last, r_avg);
            }
            if (!(rate_[c] < 0.0) || !(m.tau2[c] > 0.0) || !std::isfinite(lrr[c])) {
                known = false;
                continue;
            }
            horizon = std::max(horizon, (std::log(m.tau2[c]) - lrr[c]) / rate_[c]);
        }
        if (npoll_ == 0) {
            it_first_ = m.iter;
            for (int c = 0; c < 3; ++c) lrr_first_[c] = lrr[c];
        }
        it_last_ = m.iter;
        for (int c = 0; c < 3; ++c) lrr_last_[c] = lrr[c];
        ++npoll_;
        have_pred_ = known;
        if (known) halt_pred_ = m.iter + (int32_t)std::min(std::ceil(horizon), 1.0e6);
    }

    // iterations to queue now, the first of them being `next`; 0 = wait for
    // the poll in flight
    int batch(int32_t next, bool poll_in_flight) {
        if (!have_pred_) {
            const int k = k_;
            k_ = std::min(2 * k_, kmax_);
            return k;
        }
        const int32_t reach = halt_pred_ - next + 1;  // iterations up to H
        if (reach <= 0) return poll_in_flight ? 0 : 1;
        // half the distance per batch, so that the polls close in on H; 0
        // (wait for the poll in flight) once H is the next iteration
        const int32_t k = poll_in_flight ? reach / 2 : (reach + 1) / 2;
        return std::min(k, (int32_t)kmax_);
    }

  private:
    int kmax_;
    int k_;
    int npoll_ = 0;
    bool have_pred_ = false;
    int32_t halt_pred_ = 0;
    int32_t it_first_ = 0, it_last_ = 0;
    double lrr_first_[3] = {0.0, 0.0, 0.0}, lrr_last_[3] = {0.0, 0.0, 0.0};
    double rate_[3] = {0.0, 0.0, 0.0};  // 0: none known yet
};

}  // namespace sph
