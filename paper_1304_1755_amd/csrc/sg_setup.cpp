// Host-side setup: KL eigenpairs, chaos tables, cell coefficients, the
// multigrid hierarchy of K_0 and the coupling plans used by the apply kernels.
// Runs once per context, in double precision.

#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "sg_internal.h"

namespace sg {

namespace {

// ------------------------------------------------------------------ KL (Sec. 2.1)
// 1-D covariance exp(-c|s-t|) on t in [-1/2, 1/2].  Even eigenfunctions
// cos(w t) need c cos(w/2) = w sin(w/2); odd ones sin(w t) need
// w cos(w/2) = -c sin(w/2); the eigenvalue is 2c / (w^2 + c^2).  Each
// equation has exactly one root per half period; it is isolated by bisection
// down to adjacent doubles.
struct Mode1D {
    bool even;
    double w, lam, norm;
};

double even_fn(double w, double c) { return c * std::cos(0.5 * w) - w * std::sin(0.5 * w); }
double odd_fn(double w, double c) { return w * std::cos(0.5 * w) + c * std::sin(0.5 * w); }

double bisect(double (*f)(double, double), double lo, double hi, double c) {
    double flo = f(lo, c);
    for (int it = 0; it < 2000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double fm = f(mid, c);
        if (fm == 0.0) return mid;
        if ((fm > 0) == (flo > 0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
    }
    return 0.5 * (lo + hi);
}

std::vector<Mode1D> kl_1d(double corr_len, int count) {
    const double c = 1.0 / corr_len;
    const double pi = 3.14159265358979323846;
    std::vector<Mode1D> out;
    for (int j = 0; (int)out.size() < count; ++j) {
        double w = bisect(even_fn, 2 * j * pi, 2 * j * pi + pi, c);
        out.push_back({true, w, 2 * c / (w * w + c * c), std::sqrt(0.5 + std::sin(w) / (2 * w))});
        if ((int)out.size() == count) break;
        w = bisect(odd_fn, 2 * j * pi + pi, 2 * j * pi + 2 * pi, c);
        out.push_back({false, w, 2 * c / (w * w + c * c), std::sqrt(0.5 - std::sin(w) / (2 * w))});
    }
    return out;
}

double eval1d(const Mode1D& md, double t) {
    return (md.even ? std::cos(md.w * t) : std::sin(md.w * t)) / md.norm;
}

// ------------------------------------------------------------------ chaos (Sec. 2.2, 3.1)
// orthonormal Legendre recurrence: xi q_k = b_{k+1} q_{k+1} + b_k q_{k-1},
// b_k = k / sqrt(4k^2 - 1); so E[xi q_a q_{a+1}] = b_{a+1}.
double legendre_b(int k) { return k / std::sqrt(4.0 * k * k - 1.0); }

std::vector<std::vector<int>> graded_indices(int m, int p) {
    // enumerate every alpha in {0..p}^m with |alpha| <= p, then order by total
    // degree and, inside a degree, by alpha_1 descending, alpha_2 descending, ...
    std::vector<std::vector<int>> all;
    std::vector<int> a(m, 0);
    if (m == 0) {
        all.push_back({});
        return all;
    }
    while (true) {
        int s = 0;
        for (int v : a) s += v;
        if (s <= p) all.push_back(a);
        int i = 0;
        while (i < m) {
            if (++a[i] <= p) break;
            a[i] = 0;
            ++i;
        }
        if (i == m) break;
    }
    std::sort(all.begin(), all.end(), [](const std::vector<int>& x, const std::vector<int>& y) {
        int sx = 0, sy = 0;
        for (int v : x) sx += v;
        for (int v : y) sy += v;
        if (sx != sy) return sx < sy;
        return x > y;  // lexicographically larger first
    });
    return all;
}

// ------------------------------------------------------------------ dense SPD helpers
bool cholesky_inverse(std::vector<double>& A, int n) {
    // A (n x n, row-major, symmetric) -> A^{-1} via A = L L^T
    std::vector<double> L(A.size(), 0.0);
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(d > 0)) return false;
        double ljj = std::sqrt(d);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = s / ljj;
        }
    }
    std::vector<double> inv((size_t)n * n, 0.0), col(n);
    for (int c = 0; c < n; ++c) {
        for (int i = 0; i < n; ++i) {  // forward: L y = e_c
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * col[k];
            col[i] = s / L[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {  // backward: L^T x = y
            double s = col[i];
            for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * col[k];
            col[i] = s / L[(size_t)i * n + i];
        }
        for (int i = 0; i < n; ++i) inv[(size_t)i * n + c] = col[i];
    }
    A.swap(inv);
    return true;
}

// Weight of coarse node J in the interpolated value at the fine node whose
// offset from J's own fine position (2 J + 1 per axis) is (dx, dy), |dx|, |dy| <= 1.
// Bilinear: (1 - |dx|/2)(1 - |dy|/2).  Linear interpolation on the triangles
// of the south-west to north-east split (Sec. 6): the same on the grid lines;
// a fine cell centre lies on the diagonal of its coarse cell, so it takes
// 1/2 from the coarse SW and NE corners (dx = dy) and nothing from the others.
double transfer_weight(int dx, int dy, bool p1) {
    if (dx != 0 && dy != 0) return p1 ? (dx == dy ? 0.5 : 0.0) : 0.25;
    return (dx == 0 ? 1.0 : 0.5) * (dy == 0 ? 1.0 : 0.5);
}

// Galerkin coarsening P^T K P of a 9-point operator on interior nodes, with P
// the interpolation above from the (nc-1)^2 coarse to the (2nc-1)^2 fine nodes.
std::vector<double> rap(const std::vector<double>& Sf, int nf, bool p1) {
    const int nc = nf / 2, nxf = nf - 1, nxc = nc - 1;
    std::vector<double> Sc((size_t)nxc * nxc * 9, 0.0);
    for (int Y = 0; Y < nxc; ++Y)
        for (int X = 0; X < nxc; ++X) {
            double* out = &Sc[((size_t)Y * nxc + X) * 9];
            for (int ay = -1; ay <= 1; ++ay)
                for (int ax = -1; ax <= 1; ++ax) {
                    const int fx = 2 * X + 1 + ax, fy = 2 * Y + 1 + ay;  // fine node a
                    const double pa = transfer_weight(ax, ay, p1);
                    if (pa == 0.0) continue;
                    const double* st = &Sf[((size_t)fy * nxf + fx) * 9];
                    for (int ey = -1; ey <= 1; ++ey)
                        for (int ex = -1; ex <= 1; ++ex) {
                            const int bx = fx + ex, by = fy + ey;  // fine node b
                            if (bx < 0 || by < 0 || bx >= nxf || by >= nxf) continue;
                            const double kab = st[(ey + 1) * 3 + (ex + 1)];
                            if (kab == 0.0) continue;
                            // coarse neighbours J = (X + ox, Y + oy) with P(b, J) != 0
                            for (int oy = -1; oy <= 1; ++oy)
                                for (int ox = -1; ox <= 1; ++ox) {
                                    const int JX = X + ox, JY = Y + oy;
                                    if (JX < 0 || JY < 0 || JX >= nxc || JY >= nxc) continue;
                                    const int dx = bx - (2 * JX + 1), dy = by - (2 * JY + 1);
                                    if (dx < -1 || dx > 1 || dy < -1 || dy > 1) continue;
                                    const double pb = transfer_weight(dx, dy, p1);
                                    if (pb != 0.0) out[(oy + 1) * 3 + (ox + 1)] += pa * kab * pb;
                                }
                        }
                }
        }
    return Sc;
}

// The fine-grid operator K_k (k = 0..m) as 9-point stencils on the interior
// nodes, (dy, dx) row-major, node (x, y) at y*nx + x, nx = n - 1.
//   SG_DISC_Q1: node (x, y) touches cells SW (x, y), SE (x+1, y), NW (x, y+1)
//   and NE (x+1, y+1); with the coefficient c of a cell, its element matrix
//   has entries 4c/6 (own vertex), -c/6 (edge neighbour), -2c/6 (opposite
//   vertex).
//   SG_DISC_P1: the 5-point operator sum_e w_{k,e} (u_i - u_j) over the grid
//   edges, from the east and north edge weights of every grid vertex; node
//   (x, y) is vertex (x+1, y+1).
std::vector<double> fine_stencil(const HostSetup& hs, int k) {
    const int n = hs.n, nx = n - 1, m = hs.m;
    const size_t ncell = (size_t)n * n;
    std::vector<double> st((size_t)nx * nx * 9, 0.0);
    if (hs.disc != SG_DISC_P1) {
        const double* c = &hs.cellc[(size_t)k * ncell];
        for (int y = 0; y < nx; ++y)
            for (int x = 0; x < nx; ++x) {
                const double sw = c[(size_t)y * n + x], se = c[(size_t)y * n + x + 1];
                const double nw = c[(size_t)(y + 1) * n + x], ne = c[(size_t)(y + 1) * n + x + 1];
                double* s = &st[((size_t)y * nx + x) * 9];
                s[0] = -2.0 * sw / 6.0;          // (-1,-1)
                s[1] = -(sw + se) / 6.0;         // ( 0,-1)
                s[2] = -2.0 * se / 6.0;          // (+1,-1)
                s[3] = -(sw + nw) / 6.0;         // (-1, 0)
                s[4] = 4.0 * (sw + se + nw + ne) / 6.0;
                s[5] = -(se + ne) / 6.0;         // (+1, 0)
                s[6] = -2.0 * nw / 6.0;          // (-1,+1)
                s[7] = -(nw + ne) / 6.0;         // ( 0,+1)
                s[8] = -2.0 * ne / 6.0;          // (+1,+1)
            }
        return st;
    }
    const int W = 2 * (m + 1);
    auto ew = [&](int vx, int vy) { return hs.kcoef[((size_t)vy * n + vx) * W + k]; };
    auto nw = [&](int vx, int vy) { return hs.kcoef[((size_t)vy * n + vx) * W + m + 1 + k]; };
    for (int y = 0; y < nx; ++y)
        for (int x = 0; x < nx; ++x) {
            const double wE = ew(x + 1, y + 1), wW = ew(x, y + 1), wN = nw(x + 1, y + 1), wS = nw(x + 1, y);
            double* s9 = &st[((size_t)y * nx + x) * 9];
            s9[1] = -wS;
            s9[3] = -wW;
            s9[4] = wE + wW + wN + wS;
            s9[5] = -wE;
            s9[7] = -wN;
        }
    return st;
}

// f = 2 (1/2 - x^2 - y^2) on (-1/2, 1/2)^2 (Sec. 6)
double paper_load(double x, double y) { return 2.0 * (0.5 - x * x - y * y); }

}  // namespace

int host_setup(const sg_options& opt, const double* a0_nodal, const double* kl_amp, HostSetup& hs) {
    const int n = opt.n_cells, m = opt.m, p = opt.p;
    hs.n = n;
    hs.m = m;
    hs.p = p;
    hs.N = (n - 1) * (n - 1);
    hs.disc = opt.discretization;
    const bool p1 = hs.disc == SG_DISC_P1;
    // xi_k ~ U[-1, 1] (orthonormal Legendre chaos as is), or uniform with
    // variance one (Sec. 6): xi = sqrt 3 eta with eta ~ U[-1, 1] scales the
    // coupling E[xi q_a q_b] by sqrt 3
    hs.gscale = p1 ? std::sqrt(3.0) : 1.0;

    // chaos index set and degree levels
    auto idx = graded_indices(m, p);
    hs.P = (int)idx.size();
    hs.midx.assign((size_t)hs.P * m, 0);
    hs.offsets.assign(p + 2, 0);
    for (int a = 0; a < hs.P; ++a) {
        int deg = 0;
        for (int k = 0; k < m; ++k) {
            hs.midx[(size_t)a * m + k] = idx[a][k];
            deg += idx[a][k];
        }
        hs.offsets[deg + 1] = a + 1;
    }
    for (int d = 1; d <= p + 1; ++d) hs.offsets[d] = std::max(hs.offsets[d], hs.offsets[d - 1]);

    // KL modes: products of 1-D modes, the m largest products, ties by (i, j)
    hs.lambda.assign(m, 0.0);
    hs.amps.assign(m, 0.0);
    std::vector<Mode1D> m1;
    std::vector<std::pair<int, int>> pick;
    if (m > 0) {
        m1 = kl_1d(opt.corr_len, m + 1);
        struct Cand { double lam; int i, j; };
        std::vector<Cand> cand;
        for (int i = 0; i <= m; ++i)
            for (int j = 0; j <= m; ++j) cand.push_back({m1[i].lam * m1[j].lam, i, j});
        std::stable_sort(cand.begin(), cand.end(), [](const Cand& x, const Cand& y) {
            if (x.lam != y.lam) return x.lam > y.lam;
            if (x.i != y.i) return x.i < y.i;
            return x.j < y.j;
        });
        for (int k = 0; k < m; ++k) {
            pick.push_back({cand[k].i, cand[k].j});
            hs.lambda[k] = cand[k].lam;
            hs.amps[k] = kl_amp ? kl_amp[k] : std::sqrt(cand[k].lam);
        }
    }

    const double h = 1.0 / n;
    const size_t ncell = (size_t)n * n;
    hs.mg_n.clear();
    hs.mg_sten.clear();
    if (!p1) {
        // cell coefficients (midpoint rule per cell)
        hs.cellc.assign((size_t)(m + 1) * ncell, 0.0);
        hs.klcell.assign((size_t)m * ncell, 0.0);
        for (int cy = 0; cy < n; ++cy)
            for (int cx = 0; cx < n; ++cx) {
                const size_t e = (size_t)cy * n + cx;
                double a0 = 1.0;
                if (a0_nodal) {
                    const size_t v = (size_t)cy * (n + 1) + cx;
                    a0 = 0.25 * (a0_nodal[v] + a0_nodal[v + 1] + a0_nodal[v + n + 1] + a0_nodal[v + n + 2]);
                }
                hs.cellc[e] = a0;
                const double t1 = (cx + 0.5) * h - 0.5, t2 = (cy + 0.5) * h - 0.5;
                double spread = 0.0;
                for (int k = 0; k < m; ++k) {
                    const double b = eval1d(m1[pick[k].first], t1) * eval1d(m1[pick[k].second], t2);
                    hs.klcell[(size_t)k * ncell + e] = b;
                    const double ck = opt.sigma * hs.amps[k] * b;
                    hs.cellc[(size_t)(k + 1) * ncell + e] = ck;
                    spread += std::fabs(ck);
                }
                const double margin = a0 - spread;
                if (e == 0 || margin < hs.a_min_h) hs.a_min_h = margin;
            }

        hs.mg_n.push_back(n);
        hs.mg_sten.push_back(fine_stencil(hs, 0));
        hs.kcoef.assign(ncell * (m + 1), 0.0);
        for (size_t e = 0; e < ncell; ++e)
            for (int k = 0; k <= m; ++k) hs.kcoef[e * (m + 1) + k] = hs.cellc[(size_t)k * ncell + e] / 6.0;
    } else {
        // one value per triangle at its centroid: the lower triangle (SW, SE,
        // NE) of cell (cx, cy) has its centroid at (cx + 2/3, cy + 1/3) h, the
        // upper one (SW, NE, NW) at (cx + 1/3, cy + 2/3) h, measured from the
        // corner (-1/2, -1/2); a0 = 1
        const size_t ntri = 2 * ncell;
        hs.cellc.assign((size_t)(m + 1) * ntri, 0.0);
        hs.klcell.clear();
        for (int up = 0; up < 2; ++up)
            for (int cy = 0; cy < n; ++cy)
                for (int cx = 0; cx < n; ++cx) {
                    const size_t e = (size_t)up * ncell + (size_t)cy * n + cx;
                    const double t1 = (cx + (up ? 1.0 : 2.0) / 3.0) * h - 0.5;
                    const double t2 = (cy + (up ? 2.0 : 1.0) / 3.0) * h - 0.5;
                    hs.cellc[e] = 1.0;
                    double spread = 0.0;
                    for (int k = 0; k < m; ++k) {
                        const double b = eval1d(m1[pick[k].first], t1) * eval1d(m1[pick[k].second], t2);
                        const double ck = opt.sigma * hs.amps[k] * b;
                        hs.cellc[(size_t)(k + 1) * ntri + e] = ck;
                        spread += std::fabs(ck);
                    }
                    const double margin = 1.0 - hs.gscale * spread;
                    if (e == 0 || margin < hs.a_min_h) hs.a_min_h = margin;
                }
        // A right isosceles triangle couples the two ends of each leg with
        // -1/2 of its coefficient and the ends of its hypotenuse with 0, so
        // K_k is the 5-point operator sum_e w_{k,e} (u_i - u_j) over the grid
        // edges e = (i, j), w_{k,e} the mean of the coefficients of the two
        // triangles beside e (Dirichlet neighbours contribute u_j = 0).  The
        // east edge of vertex (cx, cy) borders the lower triangle of cell
        // (cx, cy) and the upper one of cell (cx, cy - 1); its north edge the
        // upper triangle of cell (cx, cy) and the lower one of cell (cx - 1, cy).
        auto tri = [&](int k, int up, int cx, int cy) -> double {
            if (cx < 0 || cy < 0 || cx >= n || cy >= n) return 0.0;
            return hs.cellc[(size_t)k * ntri + (size_t)up * ncell + (size_t)cy * n + cx];
        };
        const int W = 2 * (m + 1);
        hs.kcoef.assign(ncell * W, 0.0);
        for (int cy = 0; cy < n; ++cy)
            for (int cx = 0; cx < n; ++cx)
                for (int k = 0; k <= m; ++k) {
                    double* w = &hs.kcoef[((size_t)cy * n + cx) * W];
                    w[k] = 0.5 * (tri(k, 0, cx, cy) + tri(k, 1, cx, cy - 1));
                    w[m + 1 + k] = 0.5 * (tri(k, 1, cx, cy) + tri(k, 0, cx - 1, cy));
                }
        hs.mg_n.push_back(n);
        hs.mg_sten.push_back(fine_stencil(hs, 0));
        const int nx = n - 1;
        // load vector: f phi_i is a cubic on every triangle; the rule with the
        // centroid (weight -27/48) and the three points (3/5, 1/5, 1/5) in
        // barycentric coordinates (weights 25/48) is exact for cubics
        hs.load.assign(hs.N, 0.0);
        const double area = 0.5 * h * h;
        const double qb[4][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {0.6, 0.2, 0.2}, {0.2, 0.6, 0.2}, {0.2, 0.2, 0.6}};
        const double qw[4] = {-27.0 / 48, 25.0 / 48, 25.0 / 48, 25.0 / 48};
        for (int up = 0; up < 2; ++up)
            for (int cy = 0; cy < n; ++cy)
                for (int cx = 0; cx < n; ++cx) {
                    // corners (grid vertex coordinates): lower SW, SE, NE; upper SW, NE, NW
                    const int vx[3] = {cx, cx + 1, up ? cx : cx + 1};
                    const int vy[3] = {cy, up ? cy + 1 : cy, cy + 1};
                    double loc[3] = {0.0, 0.0, 0.0};
                    for (int q = 0; q < 4; ++q) {
                        double px = 0.0, py = 0.0;
                        for (int i = 0; i < 3; ++i) {
                            px += qb[q][i] * (vx[i] * h - 0.5);
                            py += qb[q][i] * (vy[i] * h - 0.5);
                        }
                        const double fq = qw[q] * area * paper_load(px, py);
                        for (int i = 0; i < 3; ++i) loc[i] += fq * qb[q][i];
                    }
                    for (int i = 0; i < 3; ++i)
                        if (vx[i] > 0 && vy[i] > 0 && vx[i] < n && vy[i] < n)
                            hs.load[(size_t)(vy[i] - 1) * nx + (vx[i] - 1)] += loc[i];
                }
    }
    while (hs.mg_n.back() > opt.coarsest_cells) {
        const int nf = hs.mg_n.back();
        hs.mg_sten.push_back(rap(hs.mg_sten.back(), nf, p1));
        hs.mg_n.push_back(nf / 2);
    }
    {
        const int nc = hs.mg_n.back(), nxc = nc - 1, Nc = nxc * nxc;
        const auto& st = hs.mg_sten.back();
        std::vector<double> A((size_t)Nc * Nc, 0.0);
        for (int y = 0; y < nxc; ++y)
            for (int x = 0; x < nxc; ++x)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int X = x + dx, Y = y + dy;
                        if (X < 0 || Y < 0 || X >= nxc || Y >= nxc) continue;
                        A[(size_t)(y * nxc + x) * Nc + (Y * nxc + X)] = st[((size_t)y * nxc + x) * 9 + (dy + 1) * 3 + (dx + 1)];
                    }
        if (!cholesky_inverse(A, Nc)) {
            set_error("coarsest-grid operator is not positive definite");
            return SG_EINVAL;
        }
        hs.coarse_inv.swap(A);
    }
    return hs.a_min_h > 0.0 ? SG_OK : SG_WNOTCOERCIVE;
}

int split_setup(const HostSetup& hs, SplitHost& sp) {
    const int m = hs.m, p = hs.p;
    if (p < 1) {
        set_error("split preconditioner: needs p >= 1 (A_hat holds the modes of degree <= p - 1)");
        return SG_EINVAL;
    }
    const bool p1 = hs.disc == SG_DISC_P1;
    const int Pa = hs.offsets[p], nlev = (int)hs.mg_n.size();
    const int nxc = hs.mg_n.back() - 1, Nc = nxc * nxc, nA = Nc * Pa;
    if (nA > kSplitMaxCoarse) {
        set_error("split preconditioner: the coarsest A_hat has " + std::to_string(nA) + " unknowns (limit " +
                  std::to_string(kSplitMaxCoarse) + "); use a coarser coarsest grid");
        return SG_EINVAL;
    }
    sp.Pa = Pa;
    sp.npart = 2 * std::max(m, 1);
    // K_k on every level: the fine operator, then Galerkin coarsening with the
    // transfer of the K_0 hierarchy
    sp.sten.assign(nlev, {});
    for (int k = 0; k <= m; ++k) {
        std::vector<double> s = fine_stencil(hs, k);
        for (int l = 0; l < nlev; ++l) {
            if (l > 0) s = rap(s, hs.mg_n[l - 1], p1);
            sp.sten[l].insert(sp.sten[l].end(), s.begin(), s.end());
        }
    }
    // partners inside A_hat: G_k(alpha, alpha + e_k) = gscale b_{alpha_k + 1},
    // G_k(alpha, alpha - e_k) = gscale b_{alpha_k}; G_k(alpha, alpha) = 0
    std::map<std::vector<int>, int> pos;
    for (int a = 0; a < hs.P; ++a)
        pos[std::vector<int>(hs.midx.begin() + (size_t)a * m, hs.midx.begin() + (size_t)(a + 1) * m)] = a;
    sp.pidx.assign((size_t)Pa * sp.npart, -1);
    sp.pcoef.assign((size_t)Pa * sp.npart, 0.0);
    for (int a = 0; a < Pa; ++a) {
        const std::vector<int> al(hs.midx.begin() + (size_t)a * m, hs.midx.begin() + (size_t)(a + 1) * m);
        int j = 0;
        for (int k = 0; k < m; ++k)
            for (int dir = 0; dir < 2; ++dir) {
                if (dir == 1 && al[k] == 0) continue;
                std::vector<int> b = al;
                b[k] += dir == 0 ? 1 : -1;
                const auto it = pos.find(b);
                if (it == pos.end() || it->second >= Pa) continue;
                sp.pidx[(size_t)a * sp.npart + j] = it->second | ((k + 1) << 16);
                sp.pcoef[(size_t)a * sp.npart + j] = hs.gscale * legendre_b(dir == 0 ? al[k] + 1 : al[k]);
                ++j;
            }
    }
    // the coarsest A_hat_l, node-major (row node * Pa + alpha), inverted
    std::vector<double> A((size_t)nA * nA, 0.0);
    const std::vector<double>& sc = sp.sten.back();
    for (int y = 0; y < nxc; ++y)
        for (int x = 0; x < nxc; ++x) {
            const int i = y * nxc + x;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int X = x + dx, Y = y + dy;
                    if (X < 0 || Y < 0 || X >= nxc || Y >= nxc) continue;
                    const int jn = Y * nxc + X, t = (dy + 1) * 3 + (dx + 1);
                    for (int a = 0; a < Pa; ++a) {
                        double* row = &A[((size_t)i * Pa + a) * nA + (size_t)jn * Pa];
                        row[a] += sc[(size_t)i * 9 + t];
                        for (int q = 0; q < sp.npart; ++q) {
                            const int e = sp.pidx[(size_t)a * sp.npart + q];
                            if (e < 0) continue;
                            const int b = e & 0xFFFF, k = e >> 16;
                            row[b] += sp.pcoef[(size_t)a * sp.npart + q] * sc[((size_t)k * Nc + i) * 9 + t];
                        }
                    }
                }
        }
    if (!cholesky_inverse(A, nA)) {
        set_error("split preconditioner: the coarsest A_hat is not positive definite");
        return SG_EINVAL;
    }
    sp.cinv.swap(A);
    return SG_OK;
}

PlanHost make_plan(const HostSetup& hs, int in_lo, int W_in, int out_lo, int W_out, bool self, bool up, bool down) {
    PlanHost pl;
    pl.in_lo = in_lo;
    pl.W_in = W_in;
    pl.out_lo = out_lo;
    pl.W_out = W_out;
    pl.self = self ? 1 : 0;
    pl.nslot = std::max((W_in + 63) / 64, (W_out + 63) / 64);
    if (pl.nslot < 1) pl.nslot = 1;
    const int m = hs.m, lanes = pl.nslot * 64, L = 2 * std::max(m, 1);
    std::map<std::vector<int>, int> pos;
    for (int a = 0; a < hs.P; ++a)
        pos[std::vector<int>(hs.midx.begin() + (size_t)a * m, hs.midx.begin() + (size_t)(a + 1) * m)] = a;
    // the partners of every output lane: (k, direction, input lane, coefficient key n),
    // where G_k(alpha, beta) = gscale * b_n with n = alpha_k + 1 for the up partner
    // alpha + e_k and n = alpha_k for the down partner alpha - e_k
    struct Partner {
        int k, dir, b, key;
    };
    std::vector<std::vector<Partner>> parts(lanes);
    for (int t = 0; t < W_out; ++t) {
        const int a = out_lo + t;
        std::vector<int> al(hs.midx.begin() + (size_t)a * m, hs.midx.begin() + (size_t)(a + 1) * m);
        for (int k = 0; k < m; ++k)
            for (int dir = 0; dir < 2; ++dir) {
                if ((dir == 0 && !up) || (dir == 1 && (!down || al[k] == 0))) continue;
                auto b = al;
                b[k] += dir == 0 ? 1 : -1;
                auto it = pos.find(b);
                if (it == pos.end() || it->second < in_lo || it->second >= in_lo + W_in) continue;
                parts[t].push_back({k, dir, it->second - in_lo, dir == 0 ? al[k] + 1 : al[k]});
            }
    }
    // single-partner table (the first degree level's lower coupling: e_k from the mean mode)
    {
        size_t most = 0;
        for (int t = 0; t < W_out; ++t) most = std::max(most, parts[t].size());
        if (most <= 1 && !self) {
            pl.one_partner = 1;
            pl.okb.assign(W_out, 0);  // no partner: coefficient row 0 (valid) with coefficient 0
            pl.ocoef.assign(W_out, 0.0);
            for (int t = 0; t < W_out; ++t)
                if (!parts[t].empty()) {
                    const Partner& q = parts[t][0];
                    pl.okb[t] = (q.k + 1) | (q.b << 8);
                    pl.ocoef[t] = hs.gscale * legendre_b(q.key);
                }
        }
    }
    // gradient tables: fixed positions 2k (up) and 2k+1 (down) per lane
    const uint32_t gzero = (uint32_t)(m * lanes);
    pl.off.assign((size_t)lanes * (L / 2), gzero | (gzero << 16));
    pl.coef.assign((size_t)lanes * L, 0.0);
    for (int t = 0; t < lanes; ++t)
        for (const Partner& q : parts[t]) {
            const uint32_t idx = (uint32_t)(q.k * lanes + q.b);
            uint32_t& w = pl.off[(size_t)t * (L / 2) + q.k];
            w = q.dir == 0 ? ((w & 0xFFFF0000u) | idx) : ((w & 0x0000FFFFu) | (idx << 16));
            pl.coef[(size_t)t * L + 2 * q.k + q.dir] = hs.gscale * legendre_b(q.key);
        }
    // apply tables: per slot, the positions are grouped by coefficient key
    // (ascending); a key takes as many positions as the slot's lane with the
    // most partners of that key needs
    const uint32_t xzero = (uint32_t)(std::max(m, 1) * lanes);
    pl.xoff.assign((size_t)lanes * (kNPos / 2), xzero | (xzero << 16));
    pl.xcoef.assign((size_t)pl.nslot * kNPos, 0.0);
    pl.npos.assign(pl.nslot, 0);
    for (int s = 0; s < pl.nslot; ++s) {
        std::map<int, int> width;
        for (int t = 64 * s; t < 64 * s + 64; ++t) {
            std::map<int, int> cnt;
            for (const Partner& q : parts[t]) cnt[q.key]++;
            for (const auto& kv : cnt) width[kv.first] = std::max(width[kv.first], kv.second);
        }
        std::map<int, int> start;
        int np = 0;
        for (const auto& kv : width) {
            start[kv.first] = np;
            for (int i = 0; i < kv.second && np + i < kNPos; ++i)
                pl.xcoef[(size_t)s * kNPos + np + i] = hs.gscale * legendre_b(kv.first);
            np += kv.second;
        }
        if (np > kNPos) {  // cannot happen for P <= 256 (at most 14 positions); refuse rather than truncate
            pl.npos.clear();
            return pl;
        }
        pl.npos[s] = np;
        for (int t = 64 * s; t < 64 * s + 64; ++t) {
            std::map<int, int> used;
            for (const Partner& q : parts[t]) {
                const int j = start[q.key] + used[q.key]++;
                const uint32_t idx = (uint32_t)exchange_index(m, lanes, q.k, q.b);
                uint32_t& w = pl.xoff[(size_t)t * (kNPos / 2) + j / 2];
                w = (j & 1) ? ((w & 0x0000FFFFu) | (idx << 16)) : ((w & 0xFFFF0000u) | idx);
            }
        }
    }
    return pl;
}

}  // namespace sg
