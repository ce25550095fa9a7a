// Host simulation of the solver's iteration issue loop on synthetic residual
// histories: the same decisions as the loop of sph_visc_solve (two polls in
// flight, the older one read before more is queued, IssuePlan sizing every
// batch), the device replaced by a table of r.r per iteration.  Prints one
// line per scenario: name, halting iteration H (the iteration whose p-update
// finds no component progressing), iterations issued, largest batch.
#include <array>
#include <cmath>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "issue_plan.hpp"

using sph::CtlPoll;
using sph::IssuePlan;

struct History {
    std::vector<std::array<double, 3>> rr;  // r.r after iteration j (j = 0: the start)
    double tau2[3];
};

static bool progressing(const History& h, int j, int c) { return !(h.rr[j][c] < h.tau2[c]); }

// The p-update of iteration it reads r.r of iteration it - 1 and halts when
// no component progresses.
static int halt_iter(const History& h) {
    for (int it = 1; it < (int)h.rr.size() + 1; ++it) {
        bool any = false;
        for (int c = 0; c < 3; ++c) any |= progressing(h, it - 1, c);
        if (!any) return it;
    }
    return (int)h.rr.size() + 1;
}

// The poll copied after iteration q ran: its p-update set iter = q and
// r.r of iteration q - 1, or the halt if some p-update up to q halted.
static CtlPoll poll_at(const History& h, int q, int H) {
    CtlPoll m{};
    if (q >= H) {
        m.halt = 1;
        return m;
    }
    for (int c = 0; c < 3; ++c) {
        m.rr[c] = h.rr[q - 1][c];
        m.tau2[c] = h.tau2[c];
        m.bb[c] = 1.0;
        m.state[c] = progressing(h, q - 1, c) ? SPH_PROGRESSING : SPH_CONVERGED;
    }
    m.iter = q;
    return m;
}

static void run(const char* name, const History& h, int kmax) {
    const int H = halt_iter(h);
    IssuePlan plan(kmax);
    int it = 1, pend[2], npend = 0, maxb = 0;
    const int last_it = (int)h.rr.size() + 1;
    bool halted = false;
    while (!halted) {
        const int k = it <= last_it && npend < 2 ? plan.batch(it, npend > 0) : 0;
        if (k > 0) {
            const int k1 = std::min(k, last_it - it + 1);
            it += k1;
            maxb = std::max(maxb, k1);
            pend[npend++] = it - 1;
        }
        if (npend == 2 || (npend > 0 && k == 0)) {
            const int q = pend[0];
            pend[0] = pend[1];
            --npend;
            const CtlPoll m = poll_at(h, q, H);
            if (m.halt) halted = true;
            else plan.observe(m);
        } else if (it > last_it && npend == 0) {
            halted = true;
        }
    }
    std::printf("%s %d %d %d\n", name, H, it - 1, maxb);
}

static History geometric(int n, const double (&q)[3], double drop) {
    History h;
    for (int j = 0; j < n; ++j) h.rr.push_back({std::pow(q[0], j), std::pow(q[1], j), std::pow(q[2], j)});
    for (int c = 0; c < 3; ++c) h.tau2[c] = drop;
    return h;
}

int main() {
    const double q1[3] = {0.7, 0.6, 0.75};
    run("geometric", geometric(400, q1, 1e-12), 8);
    run("geometric_kmax1", geometric(400, q1, 1e-12), 1);
    run("geometric_kmax16", geometric(400, q1, 1e-12), 16);
    const double q2[3] = {0.95, 0.95, 0.95};
    run("slow", geometric(2000, q2, 1e-12), 8);
    // a seeded noisy decay (BiCGSTAB's residual is not monotone)
    {
        std::mt19937_64 rng(7);
        std::normal_distribution<double> nd(0.0, 1.0);
        History h;
        for (int j = 0; j < 600; ++j) {
            std::array<double, 3> v;
            for (int c = 0; c < 3; ++c) v[c] = std::pow(0.8, j) * std::exp(1.5 * nd(rng));
            h.rr.push_back(v);
        }
        for (int c = 0; c < 3; ++c) h.tau2[c] = 1e-12;
        run("noisy", h, 8);
    }
    // a plateau of 30 iterations, then a geometric decay
    {
        History h;
        for (int j = 0; j < 600; ++j) {
            const double v = j < 30 ? 1.0 : std::pow(0.7, j - 30);
            h.rr.push_back({v, v, v});
        }
        for (int c = 0; c < 3; ++c) h.tau2[c] = 1e-12;
        run("plateau", h, 8);
    }
    // two components converged at the start (zero right-hand sides)
    {
        History h = geometric(400, q1, 1e-12);
        for (auto& v : h.rr) v[1] = v[2] = 0.0;
        h.tau2[1] = h.tau2[2] = 1e-300;
        run("one_component", h, 8);
    }
    // converged at the start: the first p-update halts
    {
        History h = geometric(10, q1, 10.0);
        run("converged_start", h, 8);
    }
    return 0;
}
