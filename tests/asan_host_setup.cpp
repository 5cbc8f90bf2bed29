// Host-only driver of the library's setup arithmetic (KL eigenpairs, chaos
// tables, cell coefficients, multigrid hierarchy, coarsest inverse, coupling
// plans), built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py.  It runs the host code over a spread of
// options, both discretisations, and checks a few invariants; any memory or
// undefined-behaviour error aborts the run.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../paper_1304_1755_amd/csrc/sg_internal.h"

namespace sg {
void set_error(const std::string&) {}
}  // namespace sg

int main() {
    struct Case {
        int n, m, p, coarsest, disc;
        double sigma, L;
        bool a0;
    };
    const Case cases[] = {
        {4, 0, 0, 2, SG_DISC_Q1, 0.0, 0.5, false}, {16, 2, 2, 4, SG_DISC_Q1, 0.3, 0.5, true},
        {32, 6, 4, 8, SG_DISC_Q1, 0.4, 0.5, false}, {64, 8, 3, 8, SG_DISC_Q1, 0.5, 0.25, true},
        {16, 1, 8, 2, SG_DISC_Q1, 0.2, 0.5, false}, {16, 6, 4, 4, SG_DISC_P1, 0.2, 1.0, false},
        {32, 4, 3, 4, SG_DISC_P1, 0.4, 1.0, false}, {8, 8, 1, 8, SG_DISC_Q1, 0.1, 0.5, false},
    };
    int bad = 0;
    for (const Case& cs : cases) {
        sg_options o{};
        o.n_cells = cs.n;
        o.m = cs.m;
        o.p = cs.p;
        o.sigma = cs.sigma;
        o.corr_len = cs.L;
        o.colour_mode = SG_COLOUR_FOUR;
        o.nu1 = o.nu2 = 2;
        o.coarsest_cells = cs.coarsest;
        o.discretization = cs.disc;
        std::vector<double> a0;
        if (cs.a0) {
            a0.resize((size_t)(cs.n + 1) * (cs.n + 1));
            for (size_t i = 0; i < a0.size(); ++i) a0[i] = 1.0 + 0.05 * std::sin(0.37 * (double)i);
        }
        sg::HostSetup hs;
        const int rc = sg::host_setup(o, cs.a0 ? a0.data() : nullptr, nullptr, hs);
        if (rc < 0) {
            std::printf("host_setup failed for n=%d m=%d p=%d\n", cs.n, cs.m, cs.p);
            ++bad;
            continue;
        }
        // every coupling plan the library builds
        std::vector<sg::PlanHost> plans;
        plans.push_back(sg::make_plan(hs, 0, hs.P, 0, hs.P, true, true, true));
        for (int d = 1; d <= hs.p; ++d) {
            const int lo = hs.offsets[d], Pd = hs.offsets[d + 1] - lo;
            const int plo = hs.offsets[d - 1], Pp = hs.offsets[d] - plo;
            plans.push_back(sg::make_plan(hs, plo, Pp, lo, Pd, false, false, true));
            plans.push_back(sg::make_plan(hs, lo, Pd, plo, Pp, false, true, false));
        }
        double checksum = 0.0;
        for (const sg::PlanHost& pl : plans) {
            if ((int)pl.npos.size() != pl.nslot) ++bad;
            for (int v : pl.npos)
                if (v < 0 || v > sg::kNPos) ++bad;
            for (double c : pl.xcoef) checksum += c;
            for (uint32_t w : pl.xoff) checksum += (double)(w & 0xFFFFu);
        }
        for (const auto& st : hs.mg_sten)
            for (double v : st) checksum += v;
        for (double v : hs.coarse_inv) checksum += v;
        if (!std::isfinite(checksum)) ++bad;
        std::printf("n=%d m=%d p=%d disc=%d P=%d levels=%zu plans=%zu ok\n", cs.n, cs.m, cs.p, cs.disc, hs.P,
                    hs.mg_n.size(), plans.size());
    }
    std::printf(bad ? "FAILED %d\n" : "ALL OK\n", bad);
    return bad ? 1 : 0;
}
