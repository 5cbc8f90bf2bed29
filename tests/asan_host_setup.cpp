// Host-only driver of the library's setup arithmetic (KL eigenpairs, chaos
// tables, cell coefficients, multigrid hierarchy, coarsest inverse, coupling
// plans, the coupled hierarchy of the 2x2 split), built with AddressSanitizer and UndefinedBehaviorSanitizer by
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
        // the 2x2 split (Sec. 4.2): K_k on every level, partner tables, the coarsest A_hat inverted
        const int nxc = hs.mg_n.back() - 1, Nc = nxc * nxc;
        if (hs.p >= 1 && Nc * hs.offsets[hs.p] <= sg::kSplitMaxCoarse) {
            sg::SplitHost sp;
            if (sg::split_setup(hs, sp) != SG_OK) {
                std::printf("split_setup failed for n=%d m=%d p=%d\n", cs.n, cs.m, cs.p);
                ++bad;
            } else {
                const int Pa = sp.Pa, np = sp.npart;
                // block k = 0 of every level is the K_0 hierarchy itself
                for (size_t l = 0; l < hs.mg_sten.size(); ++l)
                    for (size_t i = 0; i < hs.mg_sten[l].size(); ++i)
                        if (sp.sten[l][i] != hs.mg_sten[l][i]) { ++bad; break; }
                // G_k is symmetric: beta lists alpha with the same k and coefficient
                for (int a = 0; a < Pa; ++a)
                    for (int q = 0; q < np; ++q) {
                        const int e = sp.pidx[(size_t)a * np + q];
                        if (e < 0) continue;
                        const int b = e & 0xFFFF, k = e >> 16;
                        bool found = false;
                        for (int r = 0; r < np; ++r)
                            if (sp.pidx[(size_t)b * np + r] == (a | (k << 16)) &&
                                sp.pcoef[(size_t)b * np + r] == sp.pcoef[(size_t)a * np + q])
                                found = true;
                        if (!found || b >= Pa || k < 1 || k > hs.m) ++bad;
                    }
                // the stored inverse times the coarsest A_hat (assembled again from the tables) is I
                const int nA = Nc * Pa;
                const std::vector<double>& sc = sp.sten.back();
                double worst = 0.0;
                for (int row = 0; row < nA; ++row) {
                    const int i = row / Pa, a = row % Pa, y = i / nxc, x = i % nxc;
                    for (int col = 0; col < nA; ++col) {
                        double acc = 0.0;
                        for (int t = 0; t < 9; ++t) {  // (A inv)(row, col) = sum_j A(row, j) inv(j, col)
                            const int X = x + t % 3 - 1, Y = y + t / 3 - 1;
                            if (X < 0 || Y < 0 || X >= nxc || Y >= nxc) continue;
                            const int jn = Y * nxc + X;
                            acc += sc[(size_t)i * 9 + t] * sp.cinv[((size_t)jn * Pa + a) * nA + col];
                            for (int q = 0; q < np; ++q) {
                                const int e = sp.pidx[(size_t)a * np + q];
                                if (e < 0) continue;
                                acc += sp.pcoef[(size_t)a * np + q] * sc[((size_t)(e >> 16) * Nc + i) * 9 + t] *
                                       sp.cinv[((size_t)jn * Pa + (e & 0xFFFF)) * nA + col];
                            }
                        }
                        worst = std::fmax(worst, std::fabs(acc - (row == col ? 1.0 : 0.0)));
                    }
                }
                std::printf("  split: Pa=%d coarsest A_hat %d unknowns, inverse residual %.2e\n", Pa, nA, worst);
                if (!(worst < 1e-9)) {
                    std::printf("coarsest A_hat inverse off by %.3e\n", worst);
                    ++bad;
                }
            }
        }
        std::printf("n=%d m=%d p=%d disc=%d P=%d levels=%zu plans=%zu ok\n", cs.n, cs.m, cs.p, cs.disc, hs.P,
                    hs.mg_n.size(), plans.size());
    }
    std::printf(bad ? "FAILED %d\n" : "ALL OK\n", bad);
    return bad ? 1 : 0;
}
