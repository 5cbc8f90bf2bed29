// C ABI of libsgbt: context setup, the operator, the block preconditioners,
// the Krylov drivers and the adjoint QoI gradient.  Host code here only
// enqueues kernels on the context's stream and runs the O(restart^2) scalar
// work of the Krylov recurrences (Hessenberg, Givens rotations).

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "sg_internal.h"
#include "sg_vec.h"

namespace sg {

namespace {
thread_local std::string g_last_error;

template <typename T>
int dalloc(sg_ctx* c, T** p, size_t count) {
    void* q = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
        return SG_ENOMEM;
    }
    c->allocations.push_back(q);
    *p = (T*)q;
    return SG_OK;
}

// free one allocation made by dalloc (no-op for null)
void dfree(sg_ctx* c, void* q) {
    if (!q) return;
    for (size_t i = 0; i < c->allocations.size(); ++i)
        if (c->allocations[i] == q) {
            c->allocations.erase(c->allocations.begin() + i);
            break;
        }
    (void)hipStreamSynchronize(c->stream);  // no queued kernel may still use it
    (void)hipFree(q);
}

template <typename T>
int upload(sg_ctx* c, T** p, const std::vector<T>& host) {
    int rc = dalloc(c, p, host.size());
    if (rc) return rc;
    SG_HIP_CHECK(hipMemcpy(*p, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice));
    return SG_OK;
}

int upload_plan(sg_ctx* c, const PlanHost& ph, Plan& pl) {
    pl.in_lo = ph.in_lo;
    pl.W_in = ph.W_in;
    pl.out_lo = ph.out_lo;
    pl.W_out = ph.W_out;
    pl.nslot = ph.nslot;
    pl.self = ph.self;
    if ((int)ph.npos.size() != ph.nslot) {
        set_error("coupling plan: more partner positions than the apply kernel holds");
        return SG_EINVAL;
    }
    pl.nblk_max = 0;
    for (int v : ph.npos) pl.nblk_max = std::max(pl.nblk_max, (v + 3) / 4);
    int rc = upload(c, &pl.d_xoff, ph.xoff);
    if (!rc) rc = upload(c, &pl.d_xcoef, ph.xcoef);
    if (!rc) rc = upload(c, &pl.d_npos, ph.npos);
    if (!rc) rc = upload(c, &pl.d_off, ph.off);
    if (!rc) rc = upload(c, &pl.d_coef, ph.coef);
    pl.one_partner = ph.one_partner;
    pl.d_okb = nullptr;
    pl.d_ocoef = nullptr;
    if (!rc && ph.one_partner) rc = upload(c, &pl.d_okb, ph.okb);
    if (!rc && ph.one_partner) rc = upload(c, &pl.d_ocoef, ph.ocoef);
    return rc;
}

size_t NP(const sg_ctx* c) { return (size_t)c->hs.N * c->hs.P; }
// stride of the Krylov basis: NP rounded up so every basis vector starts 512-byte aligned
size_t NPpad(const sg_ctx* c) { return (NP(c) + 63) / 64 * 64; }

int ensure_mg(sg_ctx* c, int is_float) {
    const int P = c->hs.P;
    for (size_t l = 0; l < c->levels.size(); ++l) {
        Level& lv = c->levels[l];
        const size_t cap = (size_t)lv.N * P;
        int rc = SG_OK;
        if (is_float && !lv.r32) {
            rc = dalloc(c, &lv.r32, cap);
            if (!rc) rc = dalloc(c, &lv.w32, cap);
            if (!rc) rc = dalloc(c, &lv.u32, cap);  // level 0: the cycle's compact iterate
            if (!rc && l > 0) rc = dalloc(c, &lv.f32, cap);
        }
        if (!is_float && !lv.r64) {
            rc = dalloc(c, &lv.r64, cap);
            if (!rc) rc = dalloc(c, &lv.w64, cap);
            if (!rc) rc = dalloc(c, &lv.u64, cap);
            if (!rc && l > 0) rc = dalloc(c, &lv.f64, cap);
        }
        if (rc) return rc;
    }
    if (!c->ws.fstage) {
        c->ws.fstage_bytes = NP(c) * sizeof(double);
        double* p = nullptr;
        int rc = dalloc(c, &p, NP(c));
        if (rc) return rc;
        c->ws.fstage = p;
    }
    return SG_OK;
}

int ensure_scalars(sg_ctx* c) {
    if (c->ws.scal) return SG_OK;
    int rc = dalloc(c, &c->ws.scal, 1024);
    if (rc) return rc;
    rc = dalloc(c, &c->ws.partial, (size_t)kRedBlocks * 256);
    if (rc) return rc;
    SG_HIP_CHECK(hipHostMalloc((void**)&c->ws.host_scal, 1024 * sizeof(double), hipHostMallocDefault));
    return SG_OK;
}

int ensure_krylov(sg_ctx* c, int restart, int z_float) {
    int rc = ensure_scalars(c);
    if (rc) return rc;
    const size_t np = NP(c);
    if (!c->ws.w) {
        rc = dalloc(c, &c->ws.w, np);
        if (rc) return rc;
    }
    // V holds restart + 1 double vectors; Z holds restart vectors of the
    // preconditioner's precision.  A larger request replaces the old buffers
    // (freed first, so growing does not strand device memory).
    if (c->ws.restart < restart) {
        dfree(c, c->ws.V);
        c->ws.V = nullptr;
        c->ws.restart = 0;
        rc = dalloc(c, &c->ws.V, (size_t)(restart + 1) * NPpad(c));
        if (rc) return rc;
        c->ws.restart = restart;
    }
    const size_t zbytes = (size_t)restart * NPpad(c) * (z_float ? sizeof(float) : sizeof(double));
    if (c->ws.z_bytes < zbytes) {
        dfree(c, c->ws.Z);
        c->ws.Z = nullptr;
        c->ws.z_bytes = 0;
        char* z = nullptr;
        rc = dalloc(c, &z, zbytes);
        if (rc) return rc;
        c->ws.Z = z;
        c->ws.z_bytes = zbytes;
    }
    c->ws.z_is_float = z_float;
    return SG_OK;
}

// ------------------------------------------------------------------ preconditioners
int precond_diag(sg_ctx* c, const double* R, void* Z, int zf) {
    const int P = c->hs.P, N = c->hs.N;
    int rc = ensure_mg(c, zf);
    if (rc) return rc;
    if (zf) {
        rc = launch_cast(c->stream, R, 0, P, c->ws.fstage, 1, P, N, P);
        if (rc) return rc;
        return launch_vcycle(c, c->ws.fstage, P, Z, P, P, 1);
    }
    return launch_vcycle(c, R, P, Z, P, P, 0);
}

int precond_tri(sg_ctx* c, const double* R, void* Z, int zf) {
    const int P = c->hs.P, N = c->hs.N, p = c->hs.p;
    const auto& off = c->hs.offsets;
    int rc = ensure_mg(c, zf);
    if (rc) return rc;
    const size_t es = zf ? sizeof(float) : sizeof(double);
    for (int d = 0; d <= p; ++d) {
        const int lo = off[d], Pd = off[d + 1] - off[d];
        if (Pd == 0) continue;
        const void* f;
        int ldf;
        if (d == 0) {
            if (zf) {
                rc = launch_cast(c->stream, R + lo, 0, P, c->ws.fstage, 1, Pd, N, Pd);
                if (rc) return rc;
                f = c->ws.fstage;
                ldf = Pd;
            } else {
                f = R + lo;
                ldf = P;
            }
        } else {
            // R_d - sum_k [G_k]_{d,d-1} (x) K_k Z_{d-1}, into the staging block
            const Plan& pl = c->plan_down[d];
            const char* zin = (const char*)Z + (size_t)pl.in_lo * es;
            rc = launch_apply(c, pl, zin, zf, R + lo, c->ws.fstage, zf, P, Pd, P);
            if (rc) return rc;
            f = c->ws.fstage;
            ldf = Pd;
        }
        rc = launch_vcycle(c, f, ldf, (char*)Z + (size_t)lo * es, P, Pd, zf);
        if (rc) return rc;
    }
    return SG_OK;
}

// Z = B_S^{-1} R: the forward sweep, then for d = p-1 .. 0
// Z_d <- Z_d - V-cycle(sum_k [G_k]_{d,d+1} (x) K_k Z_{d+1}).
int precond_sym(sg_ctx* c, const double* R, void* Z, int zf) {
    const int P = c->hs.P, N = c->hs.N, p = c->hs.p;
    const auto& off = c->hs.offsets;
    int rc = precond_tri(c, R, Z, zf);
    if (rc) return rc;
    if (!c->ws.ustage) {
        double* q = nullptr;
        if ((rc = dalloc(c, &q, NP(c)))) return rc;
        c->ws.ustage = q;
    }
    const size_t es = zf ? sizeof(float) : sizeof(double);
    for (int d = p - 1; d >= 0; --d) {
        const int lo = off[d], Pd = off[d + 1] - off[d];
        if (Pd == 0 || off[d + 2] == off[d + 1]) continue;
        const Plan& pl = c->plan_up[d];
        const char* zin = (const char*)Z + (size_t)pl.in_lo * es;
        if ((rc = launch_apply(c, pl, zin, zf, nullptr, c->ws.fstage, zf, P, Pd, P))) return rc;
        if ((rc = launch_vcycle(c, c->ws.fstage, Pd, c->ws.ustage, Pd, Pd, zf))) return rc;
        if ((rc = launch_axpy_cols(c->stream, c->ws.ustage, zf, Pd, (char*)Z + (size_t)lo * es, P, N, Pd, -1.0)))
            return rc;
    }
    return SG_OK;
}

// ------------------------------------------------------------------ the 2 x 2 split (Sec. 4.2)
// B_T = [[A_hat, 0], [W, D]] with A_hat the modes of degree <= p-1 and
// D = I (x) K_0 those of degree p: z1 = A_hat^{-1} r1 by one coupled V-cycle,
// z2 = D^{-1} (r2 - W z1) by one K_0 V-cycle per mode.  The symmetric variant
// B_S = B_T blockdiag(A_hat, D)^{-1} B_T^T then takes z1 <- z1 - A_hat^{-1} W^T z2.
int ensure_split(sg_ctx* c) {
    SplitDev& d = c->split;
    if (d.ready) return SG_OK;
    if (c->opt.colour_mode != SG_COLOUR_LEX) {
        set_error("split preconditioner: needs SG_COLOUR_LEX (point Gauss-Seidel in the natural order)");
        return SG_EINVAL;
    }
    SplitHost h;
    int rc = split_setup(c->hs, h);
    if (rc) return rc;
    if ((rc = ensure_mg(c, 0))) return rc;
    // on a failed allocation everything this call allocated is freed again, so a later call
    // starts from scratch without stranding device memory
    const size_t first = c->allocations.size();
    struct Undo {
        sg_ctx* c;
        size_t first;
        bool armed = true;
        ~Undo() {
            if (!armed) return;
            while (c->allocations.size() > first) {
                void* q = c->allocations.back();
                dfree(c, q);
            }
        }
    } undo{c, first};
    const int L = (int)c->levels.size(), p = c->hs.p;
    d.Pa = h.Pa;
    d.npart = h.npart;
    d.gmax = 0;
    for (int dd = 0; dd < p; ++dd) d.gmax = std::max(d.gmax, c->hs.offsets[dd + 1] - c->hs.offsets[dd]);
    d.sten.assign(L, nullptr);
    d.u.assign(L, nullptr);
    d.f.assign(L, nullptr);
    d.r.assign(L, nullptr);
    for (int l = 0; l < L; ++l) {
        const size_t cap = (size_t)c->levels[l].N * d.Pa;
        if ((rc = upload(c, &d.sten[l], h.sten[l]))) return rc;
        if (l > 0 && ((rc = dalloc(c, &d.u[l], cap)) || (rc = dalloc(c, &d.f[l], cap)))) return rc;
        if (l < L - 1 && (rc = dalloc(c, &d.r[l], cap))) return rc;
    }
    const size_t N0 = c->levels[0].N;
    if ((rc = upload(c, &d.pidx, h.pidx)) || (rc = upload(c, &d.pcoef, h.pcoef)) || (rc = upload(c, &d.cinv, h.cinv)) ||
        (rc = dalloc(c, &d.g, N0 * d.gmax)) || (rc = dalloc(c, &d.s1, N0 * d.Pa)) || (rc = dalloc(c, &d.s2, N0 * d.Pa)))
        return rc;
    undo.armed = false;
    d.ready = 1;
    return SG_OK;
}

// u = one V(nu1, nu2) cycle for A_hat_l u = f on level l from u = 0 (N_l x Pa
// blocks, row strides ldf, ldu): point Gauss-Seidel in the natural order of
// A_hat_l, forward before and backward after the coarse correction, the
// coarsest level solved directly
int split_cycle(sg_ctx* c, int l, const double* f, int ldf, double* u, int ldu) {
    SplitDev& d = c->split;
    const int L = (int)c->levels.size() - 1, Pa = d.Pa, N = c->levels[l].N, p = c->hs.p;
    const auto& off = c->hs.offsets;
    if (l == L) return launch_split_coarse(c, f, ldf, u, ldu);
    int rc = launch_fill(c->stream, u, 0, ldu, N, Pa);
    if (rc) return rc;
    auto sweep = [&](bool reverse) {
        for (int i = 0; i < p; ++i) {
            const int dd = reverse ? p - 1 - i : i, lo = off[dd], w = off[dd + 1] - lo;
            if (w == 0) continue;  // an empty degree level (m = 0)
            int e = launch_split_couple(c, l, u, ldu, f, ldf, d.g, w, lo, w, 0);
            if (!e) e = launch_lex_sweep(c, l, u + lo, ldu, d.g, w, w, reverse ? 1 : 0);
            if (e) return e;
        }
        return (int)SG_OK;
    };
    for (int s = 0; s < c->opt.nu1; ++s)
        if ((rc = sweep(false))) return rc;
    if ((rc = launch_split_couple(c, l, u, ldu, f, ldf, d.r[l], Pa, 0, Pa, 1))) return rc;
    if ((rc = launch_restrict_block(c, l, d.r[l], Pa, d.f[l + 1], Pa, Pa))) return rc;
    if ((rc = split_cycle(c, l + 1, d.f[l + 1], Pa, d.u[l + 1], Pa))) return rc;
    if ((rc = launch_prolong_block(c, l, d.u[l + 1], Pa, u, ldu, Pa))) return rc;
    for (int s = 0; s < c->opt.nu2; ++s)
        if ((rc = sweep(true))) return rc;
    return SG_OK;
}

int precond_split(sg_ctx* c, const double* R, double* Z, int sym) {
    int rc = ensure_split(c);
    if (rc) return rc;
    const SplitDev& d = c->split;
    const int P = c->hs.P, N = c->hs.N, p = c->hs.p, Pa = d.Pa, Pd = P - Pa;
    const auto& off = c->hs.offsets;
    if ((rc = split_cycle(c, 0, R, P, Z, P))) return rc;
    if (Pd == 0) return SG_OK;  // no modes of degree p (m = 0): B_T is A_hat alone
    // W couples degree p only with degree p-1: the lower coupling plan of the top level
    const Plan& pd = c->plan_down[p];
    if ((rc = launch_apply(c, pd, Z + pd.in_lo, 0, R + Pa, c->ws.fstage, 0, P, Pd, P))) return rc;
    if ((rc = launch_vcycle(c, c->ws.fstage, Pd, Z + Pa, P, Pd, 0))) return rc;
    if (!sym) return SG_OK;
    // W^T z2 is nonzero in degree p-1 only
    const Plan& pu = c->plan_up[p - 1];
    if ((rc = launch_fill(c->stream, d.s1, 0, Pa, N, Pa))) return rc;
    if ((rc = launch_apply(c, pu, Z + pu.in_lo, 0, nullptr, d.s1 + off[p - 1], 0, P, Pa, P))) return rc;
    if ((rc = split_cycle(c, 0, d.s1, Pa, d.s2, Pa))) return rc;
    return launch_axpy_cols(c->stream, d.s2, 0, Pa, Z, P, N, Pa, -1.0);
}

int apply_precond(sg_ctx* c, int kind, const double* R, void* Z, int zf) {
    if (kind >= 3) return precond_split(c, R, (double*)Z, kind == 4);
    if (kind == 2) return precond_sym(c, R, Z, zf);
    return kind == 1 ? precond_tri(c, R, Z, zf) : precond_diag(c, R, Z, zf);
}

// ------------------------------------------------------------------ Krylov
struct Timer {
    bool on = false;
    hipEvent_t ev[6];
    double apply = 0, prec = 0, orth = 0;
    int napply = 0, nprec = 0;
    void init(bool enable) {
        on = enable;
        if (on)
            for (auto& e : ev) (void)hipEventCreate(&e);
    }
    void rec(int i, hipStream_t s) {
        if (on) (void)hipEventRecord(ev[i], s);
    }
    void collect(bool had_prec, bool had_apply, bool had_orth) {
        if (!on) return;
        float ms;
        if (had_prec && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) { prec += ms; ++nprec; }
        if (had_apply && hipEventElapsedTime(&ms, ev[2], ev[3]) == hipSuccess) { apply += ms; ++napply; }
        if (had_orth && hipEventElapsedTime(&ms, ev[4], ev[5]) == hipSuccess) orth += ms;
    }
    void done() {
        if (on)
            for (auto& e : ev) (void)hipEventDestroy(e);
    }
};

int fetch(sg_ctx* c, const double* dsrc, int count) {
    SG_HIP_CHECK(hipMemcpyAsync(c->ws.host_scal, dsrc, count * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    SG_HIP_CHECK(hipStreamSynchronize(c->stream));
    return SG_OK;
}

// Right-preconditioned flexible GMRES(restart).  The Arnoldi basis is built
// by classical Gram-Schmidt with delayed reorthogonalization: in step j the
// candidate u = V_j left by step j-1 (orthogonalized once, not normalized)
// is preconditioned as it is (the flexible method accepts any z_j), and one
// pass of dot products [Q, u]^T [u, w] (w = A z_j) yields both the second
// orthogonalization of u and the projection of w.  The final q_j then
// replaces u, and column j-1 of the Hessenberg matrix takes the small
// correction that the second orthogonalization implies, so A Z = Q H stays
// exact; the Givens rotations for the running residual estimate use the
// uncorrected columns, and the least-squares problem at the end of a cycle
// is solved on the corrected matrix.
int fgmres(sg_ctx* c, const double* F, double* X, const sg_solve_opts& o, sg_solve_info& info, Timer& tm) {
    const size_t np = NP(c);
    const int restart = o.restart;
    const int zf = o.prec == SG_MIXED;
    // left: GMRES on M^{-1} A x = M^{-1} F (solver 4), z_j = u_j and w = M^{-1} A u_j
    const bool left = o.solver == 4;
    int rc = ensure_krylov(c, restart, zf);
    if (rc) return rc;
    if (left && !c->ws.lt && (rc = dalloc(c, &c->ws.lt, np))) return rc;
    double* scal = c->ws.scal;
    double* hs = c->ws.host_scal;
    const size_t zes = zf ? sizeof(float) : sizeof(double);
    const size_t vs = NPpad(c);
    auto Vj = [&](int j) { return c->ws.V + (size_t)j * vs; };
    auto Zj = [&](int j) { return (void*)((char*)c->ws.Z + (size_t)j * vs * zes); };

    // Without x0 the iterate stays zero until the first solution update, and
    // every return before that update writes the zeros.
    struct ZeroX {
        hipStream_t s;
        double* X;
        int np;
        bool pending;
        ~ZeroX() {
            if (pending) (void)launch_fill(s, X, 0, 1, np, 1);
        }
    } xz{c->stream, X, (int)np, !o.use_x0};
    // From X = 0 the first candidate is F itself: when F is 16-byte aligned the
    // first step reads it in place, and |F| comes from that step's dot products.
    bool u_is_F = !left && !o.use_x0 && (uintptr_t)F % 16 == 0;
    // nF normalises the stop test: |F| (right), |M^{-1} F| (left); nFt = |F|
    double nF = 0.0, beta = 0.0, nFt = 0.0;
    if (!u_is_F) {
        SG_HIP_CHECK(vec_dot(c->stream, F, F, np, c->ws.partial, scal));
        if ((rc = fetch(c, scal, 1))) return rc;
        nF = std::sqrt(hs[0]);
        if (!std::isfinite(nF)) {
            set_error("right-hand side norm is not finite");
            return SG_ENAN;
        }
        if (nF == 0.0) {
            info.rel_res_true = 0.0;
            xz.pending = true;
            return SG_OK;
        }
        nFt = nF;
        if (left) {
            // candidate V_0 = M^{-1} (F - A X)
            if ((rc = apply_precond(c, o.precond, F, Vj(0), 0))) return rc;
            SG_HIP_CHECK(vec_dot(c->stream, Vj(0), Vj(0), np, c->ws.partial, scal));
            if ((rc = fetch(c, scal, 1))) return rc;
            nF = beta = std::sqrt(hs[0]);
            if (!std::isfinite(nF) || nF == 0.0) {
                set_error("preconditioned right-hand side norm is not finite or zero");
                return std::isfinite(nF) ? SG_EBREAKDOWN : SG_ENAN;
            }
            info.rel_res_true = 1.0;
            if (o.use_x0) {
                if ((rc = launch_apply(c, c->plan_full, X, 0, F, c->ws.lt, 0, c->hs.P, c->hs.P, c->hs.P))) return rc;
                SG_HIP_CHECK(vec_dot(c->stream, c->ws.lt, c->ws.lt, np, c->ws.partial, scal));
                if ((rc = fetch(c, scal, 1))) return rc;
                info.rel_res_true = std::sqrt(hs[0]) / nFt;
                if ((rc = apply_precond(c, o.precond, c->ws.lt, Vj(0), 0))) return rc;
                SG_HIP_CHECK(vec_dot(c->stream, Vj(0), Vj(0), np, c->ws.partial, scal));
                if ((rc = fetch(c, scal, 1))) return rc;
                beta = std::sqrt(hs[0]);
            }
        } else {
            // r = F - A X, kept unnormalized as the first candidate V_0
            beta = nF;
            if (o.use_x0) {
                if ((rc = launch_apply(c, c->plan_full, X, 0, F, Vj(0), 0, c->hs.P, c->hs.P, c->hs.P))) return rc;
                SG_HIP_CHECK(vec_dot(c->stream, Vj(0), Vj(0), np, c->ws.partial, scal));
                if ((rc = fetch(c, scal, 1))) return rc;
                beta = std::sqrt(hs[0]);
            } else {
                SG_HIP_CHECK(hipMemcpyAsync(Vj(0), F, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
            }
            info.rel_res_true = beta / nF;
        }
        if (!std::isfinite(beta)) {
            set_error("initial residual is not finite");
            return SG_ENAN;
        }
        if (beta / nF < o.rtol) return SG_OK;
    }

    const int ld = restart;
    // Hc: corrected Hessenberg matrix; Hr: columns as rotated for the running estimate
    std::vector<double> Hc((size_t)(restart + 1) * ld), Hr((size_t)(restart + 1) * ld), cs(restart), sn(restart),
        g(restart + 1), y(restart), a(restart), b(restart), cc(restart);
    auto HC = [&](int i, int j) -> double& { return Hc[(size_t)i * ld + j]; };
    auto HR = [&](int i, int j) -> double& { return Hr[(size_t)i * ld + j]; };
    while (info.iters < o.max_it) {
        std::fill(Hc.begin(), Hc.end(), 0.0);
        std::fill(Hr.begin(), Hr.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k = 0;  // columns of this cycle
        for (int j = 0; j < restart; ++j) {
            const double* uj = u_is_F ? F : Vj(j);
            if (left) {
                SG_HIP_CHECK(hipMemcpyAsync(Zj(j), uj, np * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
                tm.rec(2, c->stream);
                if ((rc = launch_apply(c, c->plan_full, uj, 0, nullptr, c->ws.lt, 0, c->hs.P, c->hs.P, c->hs.P)))
                    return rc;
                tm.rec(3, c->stream);
                tm.rec(0, c->stream);
                if ((rc = apply_precond(c, o.precond, c->ws.lt, c->ws.w, 0))) return rc;
                tm.rec(1, c->stream);
            } else {
                tm.rec(0, c->stream);
                if ((rc = apply_precond(c, o.precond, uj, Zj(j), zf))) return rc;
                tm.rec(1, c->stream);
                tm.rec(2, c->stream);
                if ((rc = launch_apply(c, c->plan_full, Zj(j), zf, nullptr, c->ws.w, 0, c->hs.P, c->hs.P, c->hs.P)))
                    return rc;
                tm.rec(3, c->stream);
            }
            tm.rec(4, c->stream);
            SG_HIP_CHECK(vec_dots2(c->stream, c->ws.V, vs, j, uj, c->ws.w, np, c->ws.partial, scal));
            const int nch = j == 0 ? 1 : (j + kDc - 1) / kDc;
            if ((rc = fetch(c, scal, nch * kDcLd))) return rc;
            for (int i = 0; i < j; ++i) {
                a[i] = hs[(i / kDc) * kDcLd + (i % kDc)];
                b[i] = hs[(i / kDc) * kDcLd + kDc + (i % kDc)];
            }
            const double uu = hs[2 * kDc], uw = hs[2 * kDc + 1];
            if (u_is_F) {  // first step from X = 0: u = F, beta = |F|
                nF = beta = std::sqrt(uu);
                if (!std::isfinite(nF)) {
                    set_error("right-hand side norm is not finite");
                    return SG_ENAN;
                }
                info.rel_res_true = nF == 0.0 ? 0.0 : 1.0;
                if (nF == 0.0 || 1.0 < o.rtol) return SG_OK;
                g[0] = beta;
            }
            double nu2 = uu, ab = 0.0;
            for (int i = 0; i < j; ++i) {
                nu2 -= a[i] * a[i];
                ab += a[i] * b[i];
            }
            if (!std::isfinite(nu2) || !std::isfinite(uw) || !std::isfinite(ab)) {
                set_error("Arnoldi vector is not finite");
                return SG_ENAN;
            }
            if (!(nu2 > 0.0)) {
                // the candidate lies in the span of the basis: breakdown after column j - 1
                if (j > 0) HC(j, j - 1) = 0.0;
                break;
            }
            const double nu = std::sqrt(nu2);
            if (j > 0) {  // column j - 1: u = sum_i a_i q_i + nu q_j
                for (int i = 0; i < j; ++i) HC(i, j - 1) += a[i];
                HC(j, j - 1) = nu;
            }
            const double hjj = (uw - ab) / nu;
            for (int i = 0; i < j; ++i) {
                HC(i, j) = b[i];
                a[i] /= nu;
                cc[i] = b[i] - hjj * a[i];
            }
            HC(j, j) = hjj;
            // q_j = (u - Q a) / nu into V_j;  w' = w - Q b - hjj q_j into V_{j+1}
            SG_HIP_CHECK(vec_update2(c->stream, c->ws.V, vs, j, a.data(), cc.data(), 1.0 / nu, hjj / nu, uj, Vj(j),
                                     c->ws.w, Vj(j + 1), np, c->ws.partial, scal + 256));
            u_is_F = false;
            tm.rec(5, c->stream);
            if ((rc = fetch(c, scal + 256, 1))) return rc;
            tm.collect(true, true, true);
            const double hn = std::sqrt(hs[0]);
            if (!std::isfinite(hn)) {
                set_error("Arnoldi vector norm is not finite");
                return SG_ENAN;
            }
            HC(j + 1, j) = hn;  // provisional until the next step reorthogonalizes V_{j+1}
            // running estimate from the uncorrected column
            for (int i = 0; i <= j + 1; ++i) HR(i, j) = HC(i, j);
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * HR(i, j) + sn[i] * HR(i + 1, j);
                HR(i + 1, j) = -sn[i] * HR(i, j) + cs[i] * HR(i + 1, j);
                HR(i, j) = t;
            }
            const double den = std::hypot(HR(j, j), HR(j + 1, j));
            cs[j] = HR(j, j) / den;
            sn[j] = HR(j + 1, j) / den;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            info.iters++;
            k = j + 1;
            const double est = std::fabs(g[j + 1]) / nF;
            if (info.n_hist < 1024) info.rel_res_hist[info.n_hist++] = est;
            if (est < o.rtol || hn == 0.0 || info.iters >= o.max_it) break;
        }
        if (k == 0) {
            set_error("FGMRES breakdown in the first step");
            return SG_EBREAKDOWN;
        }
        // least squares min |beta e_0 - Hc y| by Givens rotations on the corrected columns
        std::vector<double> R((size_t)(k + 1) * k), gg(k + 1, 0.0);
        for (int i = 0; i <= k; ++i)
            for (int jj = 0; jj < k; ++jj) R[(size_t)i * k + jj] = HC(i, jj);
        gg[0] = beta;
        for (int jj = 0; jj < k; ++jj) {
            for (int i = 0; i < jj; ++i) {
                const double t = cs[i] * R[(size_t)i * k + jj] + sn[i] * R[(size_t)(i + 1) * k + jj];
                R[(size_t)(i + 1) * k + jj] = -sn[i] * R[(size_t)i * k + jj] + cs[i] * R[(size_t)(i + 1) * k + jj];
                R[(size_t)i * k + jj] = t;
            }
            const double d = std::hypot(R[(size_t)jj * k + jj], R[(size_t)(jj + 1) * k + jj]);
            cs[jj] = R[(size_t)jj * k + jj] / d;
            sn[jj] = R[(size_t)(jj + 1) * k + jj] / d;
            R[(size_t)jj * k + jj] = d;
            R[(size_t)(jj + 1) * k + jj] = 0.0;
            gg[jj + 1] = -sn[jj] * gg[jj];
            gg[jj] = cs[jj] * gg[jj];
        }
        for (int i = k - 1; i >= 0; --i) {
            double sacc = gg[i];
            for (int l = i + 1; l < k; ++l) sacc -= R[(size_t)i * k + l] * y[l];
            y[i] = sacc / R[(size_t)i * k + i];
        }
        std::memcpy(hs + 512, y.data(), k * sizeof(double));
        SG_HIP_CHECK(hipMemcpyAsync(scal + 512, hs + 512, k * sizeof(double), hipMemcpyHostToDevice, c->stream));
        SG_HIP_CHECK(vec_combine(c->stream, c->ws.Z, zf, vs, k, scal + 512, X, np, !xz.pending));
        xz.pending = false;
        if (left) {
            // true residual, then the new candidate M^{-1} (F - A X) and its norm
            if ((rc = launch_apply(c, c->plan_full, X, 0, F, c->ws.lt, 0, c->hs.P, c->hs.P, c->hs.P))) return rc;
            SG_HIP_CHECK(vec_dot(c->stream, c->ws.lt, c->ws.lt, np, c->ws.partial, scal));
            if ((rc = fetch(c, scal, 1))) return rc;
            info.rel_res_true = std::sqrt(hs[0]) / nFt;
            if ((rc = apply_precond(c, o.precond, c->ws.lt, Vj(0), 0))) return rc;
            SG_HIP_CHECK(vec_dot(c->stream, Vj(0), Vj(0), np, c->ws.partial, scal));
            if ((rc = fetch(c, scal, 1))) return rc;
            beta = std::sqrt(hs[0]);
        } else {
            if ((rc = launch_apply(c, c->plan_full, X, 0, F, Vj(0), 0, c->hs.P, c->hs.P, c->hs.P))) return rc;
            SG_HIP_CHECK(vec_dot(c->stream, Vj(0), Vj(0), np, c->ws.partial, scal));
            if ((rc = fetch(c, scal, 1))) return rc;
            beta = std::sqrt(hs[0]);
            info.rel_res_true = beta / nF;
        }
        if (!std::isfinite(beta)) {
            set_error("true residual is not finite");
            return SG_ENAN;
        }
        if (beta / nF < o.rtol) return SG_OK;
        if (info.iters >= o.max_it) break;
        info.restarts++;
    }
    set_error("FGMRES reached max_it above the tolerance");
    return SG_ENOTCONV;
}

int pcg(sg_ctx* c, const double* F, double* X, const sg_solve_opts& o, sg_solve_info& info, Timer& tm) {
    const size_t np = NP(c);
    int rc = ensure_scalars(c);
    if (rc) return rc;
    if (!c->ws.pcg && (rc = dalloc(c, &c->ws.pcg, 4 * np))) return rc;
    double *r = c->ws.pcg, *z = r + np, *p = z + np, *q = p + np;
    double* scal = c->ws.scal;
    double* hs = c->ws.host_scal;
    SG_HIP_CHECK(vec_dot(c->stream, F, F, np, c->ws.partial, scal));
    if ((rc = fetch(c, scal, 1))) return rc;
    const double nF = std::sqrt(hs[0]);
    if (nF == 0.0) return launch_fill(c->stream, X, 0, 1, (int)np, 1);
    if (!o.use_x0 && (rc = launch_fill(c->stream, X, 0, 1, (int)np, 1))) return rc;
    if ((rc = launch_apply(c, c->plan_full, X, 0, F, r, 0, c->hs.P, c->hs.P, c->hs.P))) return rc;
    SG_HIP_CHECK(vec_dot(c->stream, r, r, np, c->ws.partial, scal));
    if ((rc = fetch(c, scal, 1))) return rc;
    info.rel_res_true = std::sqrt(hs[0]) / nF;
    if (info.rel_res_true < o.rtol) return SG_OK;
    tm.rec(0, c->stream);
    if ((rc = apply_precond(c, o.precond, r, z, 0))) return rc;
    tm.rec(1, c->stream);
    SG_HIP_CHECK(vec_scale(c->stream, z, 1.0, p, np));
    SG_HIP_CHECK(vec_dot(c->stream, r, z, np, c->ws.partial, scal));
    if ((rc = fetch(c, scal, 1))) return rc;
    tm.collect(true, false, false);
    double rz = hs[0];
    while (info.iters < o.max_it) {
        tm.rec(2, c->stream);
        if ((rc = launch_apply(c, c->plan_full, p, 0, nullptr, q, 0, c->hs.P, c->hs.P, c->hs.P))) return rc;
        tm.rec(3, c->stream);
        SG_HIP_CHECK(vec_dot(c->stream, p, q, np, c->ws.partial, scal));
        if ((rc = fetch(c, scal, 1))) return rc;
        tm.collect(false, true, false);
        if (!(hs[0] > 0.0) || !std::isfinite(hs[0])) {
            set_error(std::isfinite(hs[0]) ? "PCG breakdown: (A p, p) <= 0" : "PCG curvature is not finite");
            return std::isfinite(hs[0]) ? SG_EBREAKDOWN : SG_ENAN;
        }
        const double alpha = rz / hs[0];
        SG_HIP_CHECK(vec_axpy(c->stream, alpha, p, X, np));
        SG_HIP_CHECK(vec_axpy_sq(c->stream, -alpha, q, r, np, c->ws.partial, scal));
        if ((rc = fetch(c, scal, 1))) return rc;
        info.iters++;
        const double rel = std::sqrt(hs[0]) / nF;
        if (!std::isfinite(rel)) {
            set_error("PCG residual is not finite");
            return SG_ENAN;
        }
        if (info.n_hist < 1024) info.rel_res_hist[info.n_hist++] = rel;
        if (rel < o.rtol) {
            if ((rc = launch_apply(c, c->plan_full, X, 0, F, q, 0, c->hs.P, c->hs.P, c->hs.P))) return rc;
            SG_HIP_CHECK(vec_dot(c->stream, q, q, np, c->ws.partial, scal));
            if ((rc = fetch(c, scal, 1))) return rc;
            info.rel_res_true = std::sqrt(hs[0]) / nF;
            if (info.rel_res_true < o.rtol) return SG_OK;
        }
        tm.rec(0, c->stream);
        if ((rc = apply_precond(c, o.precond, r, z, 0))) return rc;
        tm.rec(1, c->stream);
        SG_HIP_CHECK(vec_dot(c->stream, r, z, np, c->ws.partial, scal));
        if ((rc = fetch(c, scal, 1))) return rc;
        tm.collect(true, false, false);
        const double rzn = hs[0];
        SG_HIP_CHECK(vec_xpby(c->stream, z, rzn / rz, p, np));
        rz = rzn;
    }
    if ((rc = launch_apply(c, c->plan_full, X, 0, F, q, 0, c->hs.P, c->hs.P, c->hs.P))) return rc;
    SG_HIP_CHECK(vec_dot(c->stream, q, q, np, c->ws.partial, scal));
    if ((rc = fetch(c, scal, 1))) return rc;
    info.rel_res_true = std::sqrt(hs[0]) / nF;
    set_error("PCG reached max_it above the tolerance");
    return SG_ENOTCONV;
}

// GPCG[1]: p_0 = M r_0; alpha = (r, p)/(A p, p); p <- M r - ((A p, M r)/(A p, p)) p
int gpcg1(sg_ctx* c, const double* F, double* X, const sg_solve_opts& o, sg_solve_info& info, Timer& tm) {
    const size_t np = NP(c);
    int rc = ensure_scalars(c);
    if (rc) return rc;
    if (!c->ws.pcg && (rc = dalloc(c, &c->ws.pcg, 4 * np))) return rc;
    double *r = c->ws.pcg, *z = r + np, *p = z + np, *q = p + np;
    double* scal = c->ws.scal;
    double* hs = c->ws.host_scal;
    SG_HIP_CHECK(vec_dot(c->stream, F, F, np, c->ws.partial, scal));
    if ((rc = fetch(c, scal, 1))) return rc;
    const double nF = std::sqrt(hs[0]);
    if (nF == 0.0) return launch_fill(c->stream, X, 0, 1, (int)np, 1);
    if (!o.use_x0 && (rc = launch_fill(c->stream, X, 0, 1, (int)np, 1))) return rc;
    if ((rc = launch_apply(c, c->plan_full, X, 0, F, r, 0, c->hs.P, c->hs.P, c->hs.P))) return rc;
    SG_HIP_CHECK(vec_dot(c->stream, r, r, np, c->ws.partial, scal));
    if ((rc = fetch(c, scal, 1))) return rc;
    info.rel_res_true = std::sqrt(hs[0]) / nF;
    if (info.rel_res_true < o.rtol) return SG_OK;
    tm.rec(0, c->stream);
    if ((rc = apply_precond(c, o.precond, r, p, 0))) return rc;
    tm.rec(1, c->stream);
    while (info.iters < o.max_it) {
        tm.rec(2, c->stream);
        if ((rc = launch_apply(c, c->plan_full, p, 0, nullptr, q, 0, c->hs.P, c->hs.P, c->hs.P))) return rc;
        tm.rec(3, c->stream);
        SG_HIP_CHECK(vec_dot(c->stream, p, q, np, c->ws.partial, scal));
        SG_HIP_CHECK(vec_dot(c->stream, r, p, np, c->ws.partial, scal + 1));
        if ((rc = fetch(c, scal, 2))) return rc;
        tm.collect(info.iters == 0, true, false);
        if (!(hs[0] > 0.0) || !std::isfinite(hs[0])) {
            set_error(std::isfinite(hs[0]) ? "GPCG breakdown: (A p, p) <= 0" : "GPCG curvature is not finite");
            return std::isfinite(hs[0]) ? SG_EBREAKDOWN : SG_ENAN;
        }
        const double pq = hs[0], alpha = hs[1] / pq;
        SG_HIP_CHECK(vec_axpy(c->stream, alpha, p, X, np));
        SG_HIP_CHECK(vec_axpy_sq(c->stream, -alpha, q, r, np, c->ws.partial, scal));
        if ((rc = fetch(c, scal, 1))) return rc;
        info.iters++;
        const double rel = std::sqrt(hs[0]) / nF;
        if (!std::isfinite(rel)) {
            set_error("GPCG residual is not finite");
            return SG_ENAN;
        }
        if (info.n_hist < 1024) info.rel_res_hist[info.n_hist++] = rel;
        if (rel < o.rtol) {
            if ((rc = launch_apply(c, c->plan_full, X, 0, F, z, 0, c->hs.P, c->hs.P, c->hs.P))) return rc;
            SG_HIP_CHECK(vec_dot(c->stream, z, z, np, c->ws.partial, scal));
            if ((rc = fetch(c, scal, 1))) return rc;
            info.rel_res_true = std::sqrt(hs[0]) / nF;
            if (info.rel_res_true < o.rtol) return SG_OK;
        }
        tm.rec(0, c->stream);
        if ((rc = apply_precond(c, o.precond, r, z, 0))) return rc;
        tm.rec(1, c->stream);
        SG_HIP_CHECK(vec_dot(c->stream, q, z, np, c->ws.partial, scal));
        if ((rc = fetch(c, scal, 1))) return rc;
        tm.collect(true, false, false);
        SG_HIP_CHECK(vec_xpby(c->stream, z, -hs[0] / pq, p, np));
    }
    if ((rc = launch_apply(c, c->plan_full, X, 0, F, z, 0, c->hs.P, c->hs.P, c->hs.P))) return rc;
    SG_HIP_CHECK(vec_dot(c->stream, z, z, np, c->ws.partial, scal));
    if ((rc = fetch(c, scal, 1))) return rc;
    info.rel_res_true = std::sqrt(hs[0]) / nF;
    set_error("GPCG reached max_it above the tolerance");
    return SG_ENOTCONV;
}

// block Gauss-Seidel iteration x <- x + M(F - A x)
int block_gs(sg_ctx* c, const double* F, double* X, const sg_solve_opts& o, sg_solve_info& info, Timer& tm) {
    const size_t np = NP(c);
    int rc = ensure_scalars(c);
    if (rc) return rc;
    if (!c->ws.pcg && (rc = dalloc(c, &c->ws.pcg, 4 * np))) return rc;
    double *r = c->ws.pcg, *z = r + np;
    double* scal = c->ws.scal;
    double* hs = c->ws.host_scal;
    SG_HIP_CHECK(vec_dot(c->stream, F, F, np, c->ws.partial, scal));
    if ((rc = fetch(c, scal, 1))) return rc;
    const double nF = std::sqrt(hs[0]);
    if (nF == 0.0) return launch_fill(c->stream, X, 0, 1, (int)np, 1);
    if (!o.use_x0 && (rc = launch_fill(c->stream, X, 0, 1, (int)np, 1))) return rc;
    while (true) {
        tm.rec(2, c->stream);
        if ((rc = launch_apply(c, c->plan_full, X, 0, F, r, 0, c->hs.P, c->hs.P, c->hs.P))) return rc;
        tm.rec(3, c->stream);
        SG_HIP_CHECK(vec_dot(c->stream, r, r, np, c->ws.partial, scal));
        if ((rc = fetch(c, scal, 1))) return rc;
        tm.collect(false, true, false);
        const double rel = std::sqrt(hs[0]) / nF;
        info.rel_res_true = rel;
        if (!std::isfinite(rel)) {
            set_error("block Gauss-Seidel residual is not finite");
            return SG_ENAN;
        }
        if (info.n_hist < 1024) info.rel_res_hist[info.n_hist++] = rel;
        if (rel < o.rtol) return SG_OK;
        if (info.iters >= o.max_it) break;
        tm.rec(0, c->stream);
        if ((rc = apply_precond(c, o.precond, r, z, 0))) return rc;
        tm.rec(1, c->stream);
        SG_HIP_CHECK(vec_axpy(c->stream, 1.0, z, X, np));
        info.iters++;
    }
    set_error("block Gauss-Seidel reached max_it above the tolerance");
    return SG_ENOTCONV;
}

int check_opts(const sg_ctx* c, const sg_solve_opts* o) {
    if (!o) return SG_EINVAL;
    if (o->solver < 0 || o->solver > 4) return SG_EINVAL;
    if (o->precond < 0 || o->precond > 4) return SG_EINVAL;
    if (o->prec != SG_F64 && o->prec != SG_MIXED) return SG_EINVAL;
    if ((o->solver == 0 || o->solver == 4) && (o->restart < 1 || o->restart > kMaxRestart)) return SG_EINVAL;
    // PCG needs a symmetric preconditioner (B_D or a B_S); everything but
    // right-preconditioned FGMRES with the level-wise preconditioners runs in
    // double only
    if (o->solver == 1 && (o->precond == 1 || o->precond == 3)) return SG_EINVAL;
    if ((o->solver != 0 || o->precond >= 3) && o->prec != SG_F64) return SG_EINVAL;
    if (o->max_it < 1 || !(o->rtol > 0.0)) return SG_EINVAL;
    (void)c;
    return SG_OK;
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace sg

using namespace sg;

extern "C" {

const char* sg_last_error(void) { return g_last_error.c_str(); }

int sg_setup(const sg_options* opt, const double* a0_nodal, const double* kl_amp, void* hip_stream, sg_ctx** out) {
    if (!opt || !out) {
        set_error("sg_setup: null argument");
        return SG_EINVAL;
    }
    *out = nullptr;
    const int n = opt->n_cells, nc = opt->coarsest_cells;
    if (n < 4 || n > 4096 || n % 4 != 0 || opt->m < 0 || opt->m > kMaxM || opt->p < 0 || opt->p > 8 || nc < 2 ||
        nc > n || n % nc != 0 || ((n / nc) & (n / nc - 1)) != 0 || (nc - 1) * (nc - 1) > 4096 ||
        !(opt->corr_len > 0.0) || opt->nu1 < 0 || opt->nu1 > 8 || opt->nu2 < 0 || opt->nu2 > 8 ||
        (opt->colour_mode != SG_COLOUR_FOUR && opt->colour_mode != SG_COLOUR_RB && opt->colour_mode != SG_COLOUR_LEX) ||
        !std::isfinite(opt->sigma) ||
        (opt->discretization != SG_DISC_Q1 && opt->discretization != SG_DISC_P1)) {
        set_error("sg_setup: invalid options (need n % 4 == 0, n = coarsest * 2^L, m <= 8, p <= 8, ...)");
        return SG_EINVAL;
    }
    if (opt->discretization == SG_DISC_P1 && (a0_nodal || opt->colour_mode == SG_COLOUR_RB)) {
        set_error("sg_setup: SG_DISC_P1 takes a0 = 1 (a0_nodal NULL) and SG_COLOUR_FOUR or SG_COLOUR_LEX");
        return SG_EINVAL;
    }
    {
        // P = (m+p)!/(m!p!) must fit 4 slots of 64 lanes
        double Pd = 1.0;
        for (int i = 1; i <= opt->p; ++i) Pd = Pd * (opt->m + i) / i;
        if (Pd > 256.5) {
            set_error("sg_setup: P = (m+p)!/(m!p!) exceeds 256");
            return SG_EINVAL;
        }
    }
    sg_ctx* c = new sg_ctx();
    c->opt = *opt;
    c->stream = (hipStream_t)hip_stream;
    int warn = host_setup(*opt, a0_nodal, kl_amp, c->hs);
    if (warn < 0) {
        delete c;
        return warn;
    }
    int rc = SG_OK;
    auto fail = [&](int code) {
        sg_destroy(c);
        return code;
    };
    if (hipGetDevice(&c->device) != hipSuccess) {
        set_error("sg_setup: no HIP device");
        return fail(SG_EHIP);
    }
    {
        // device address of the allocation-free QoI's scratch array (once per device)
        const hipError_t e = qoi_scratch_address(c->device, &c->qoi_scratch);
        if (e != hipSuccess) {
            set_error(std::string("sg_setup: scratch address lookup failed: ") + hipGetErrorString(e));
            return fail(SG_EHIP);
        }
    }
    const HostSetup& hs = c->hs;
    const int m = hs.m, P = hs.P;
    const size_t ncell = (size_t)n * n;
    {
        if ((rc = upload(c, &c->cell64, hs.kcoef))) return fail(rc);
        if ((rc = upload(c, &c->zeros, std::vector<double>(256, 0.0)))) return fail(rc);
        if (hs.disc == SG_DISC_Q1) {
            std::vector<double> kl(ncell * std::max(m, 1));
            for (size_t e = 0; e < ncell; ++e)
                for (int k = 0; k < m; ++k) kl[e * m + k] = hs.klcell[(size_t)k * ncell + e];
            if ((rc = upload(c, &c->klcell, kl))) return fail(rc);
        } else if ((rc = upload(c, &c->load, hs.load))) {
            return fail(rc);
        }
    }
    if ((rc = upload(c, &c->kinv, hs.coarse_inv))) return fail(rc);
    c->levels.resize(hs.mg_n.size());
    for (size_t l = 0; l < hs.mg_n.size(); ++l) {
        Level& lv = c->levels[l];
        std::memset(&lv, 0, sizeof(Level));
        lv.n = hs.mg_n[l];
        lv.nx = lv.n - 1;
        lv.N = lv.nx * lv.nx;
        if ((rc = upload(c, &lv.sten64, hs.mg_sten[l]))) return fail(rc);
        std::vector<float> s32(hs.mg_sten[l].begin(), hs.mg_sten[l].end());
        if ((rc = upload(c, &lv.sten32, s32))) return fail(rc);
        std::vector<double> rd64((size_t)lv.N);
        std::vector<float> rd32((size_t)lv.N);
        for (int i = 0; i < lv.N; ++i) {
            rd64[i] = 1.0 / hs.mg_sten[l][(size_t)i * 9 + 4];
            rd32[i] = 1.0f / s32[(size_t)i * 9 + 4];
        }
        if ((rc = upload(c, &lv.rdiag64, rd64))) return fail(rc);
        if ((rc = upload(c, &lv.rdiag32, rd32))) return fail(rc);
        {
            std::vector<double> p64((size_t)lv.N * 10, 0.0);
            std::vector<float> p32((size_t)lv.N * 12, 0.0f);
            for (size_t node = 0; node < (size_t)lv.N; ++node) {
                for (int e = 0; e < 9; ++e) {
                    p64[node * 10 + e] = hs.mg_sten[l][node * 9 + e];
                    p32[node * 12 + e] = s32[node * 9 + e];
                }
                p64[node * 10 + 9] = rd64[node];
                p32[node * 12 + 9] = rd32[node];
            }
            if ((rc = upload(c, &lv.stp64, p64))) return fail(rc);
            if ((rc = upload(c, &lv.stp32, p32))) return fail(rc);
        }
        if (lv.nx <= kLdsCycleMaxNx) {
            // colour q = (x odd when q is even) + (y odd when q < 2), the order of a forward sweep
            std::vector<double> c64;
            std::vector<float> c32;
            for (int q = 0; q < 4; ++q) {
                const int px = (q & 1) ^ 1, py = (q >> 1) ^ 1;
                for (int y = py; y < lv.nx; y += 2)
                    for (int x = px; x < lv.nx; x += 2) {
                        const size_t node = (size_t)y * lv.nx + x;
                        for (int e = 0; e < 9; ++e) {
                            c64.push_back(hs.mg_sten[l][node * 9 + e]);
                            c32.push_back(s32[node * 9 + e]);
                        }
                        c64.push_back(rd64[node]);
                        c32.push_back(rd32[node]);
                        c32.push_back(0.0f);
                        c32.push_back(0.0f);
                    }
            }
            if ((rc = upload(c, &lv.cst64, c64))) return fail(rc);
            if ((rc = upload(c, &lv.cst32, c32))) return fail(rc);
        }
    }
    if ((rc = upload_plan(c, make_plan(hs, 0, P, 0, P, true, true, true), c->plan_full))) return fail(rc);
    c->plan_down.assign(hs.p + 1, Plan{});
    c->plan_up.assign(hs.p + 1, Plan{});
    for (int d = 1; d <= hs.p; ++d) {
        const int lo = hs.offsets[d], Pd = hs.offsets[d + 1] - lo;
        const int plo = hs.offsets[d - 1], Pp = hs.offsets[d] - plo;
        if ((rc = upload_plan(c, make_plan(hs, plo, Pp, lo, Pd, false, false, true), c->plan_down[d])))
            return fail(rc);
        // level d-1 outputs from level d inputs (upper coupling of the backward sweep)
        if ((rc = upload_plan(c, make_plan(hs, lo, Pd, plo, Pp, false, true, false), c->plan_up[d - 1])))
            return fail(rc);
    }
    {
        // QoI weights: exact integral of each interior hat function over
        // S = [1/4, 3/4]^2, divided by |S| (grid aligned because n % 4 == 0)
        const int nx = n - 1, a = n / 4, b = 3 * n / 4;
        const double hh = 1.0 / n;
        std::vector<double> w1(nx), wS((size_t)nx * nx);
        for (int i = 1; i <= nx; ++i) w1[i - 1] = (i > a && i < b) ? hh : ((i == a || i == b) ? 0.5 * hh : 0.0);
        for (int y = 0; y < nx; ++y)
            for (int x = 0; x < nx; ++x) wS[(size_t)y * nx + x] = w1[x] * w1[y] * 4.0;
        if ((rc = upload(c, &c->ws.wS, wS))) return fail(rc);
        std::vector<double> amps(hs.amps);
        amps.resize(std::max(m, 1), 0.0);
        double* d_amps = nullptr;
        if ((rc = upload(c, &d_amps, amps))) return fail(rc);
        c->ws.amps = d_amps;
    }
    *out = c;
    return warn;
}

int sg_query(const sg_ctx* c, int* N, int* P, int* level_offsets, int* multi_index, double* kl_lambda,
             double* a_min_h) {
    if (!c) {
        set_error("sg_query: null context");
        return SG_EINVAL;
    }
    if (N) *N = c->hs.N;
    if (P) *P = c->hs.P;
    if (level_offsets) std::memcpy(level_offsets, c->hs.offsets.data(), c->hs.offsets.size() * sizeof(int));
    if (multi_index && c->hs.m) std::memcpy(multi_index, c->hs.midx.data(), c->hs.midx.size() * sizeof(int));
    if (kl_lambda && c->hs.m) std::memcpy(kl_lambda, c->hs.lambda.data(), c->hs.m * sizeof(double));
    if (a_min_h) *a_min_h = c->hs.a_min_h;
    return SG_OK;
}

int sg_get_cell_coeffs(const sg_ctx* c, double* out) {
    if (!c || !out) {
        set_error("sg_get_cell_coeffs: null argument");
        return SG_EINVAL;
    }
    std::memcpy(out, c->hs.cellc.data(), c->hs.cellc.size() * sizeof(double));
    return SG_OK;
}

int sg_rhs(sg_ctx* c, double* F) {
    if (!c || !F) {
        set_error("sg_rhs: null argument");
        return SG_EINVAL;
    }
    if (c->hs.disc == SG_DISC_P1) {
        // column 0 of the node-major block is the precomputed load vector
        const size_t P = c->hs.P;
        SG_HIP_CHECK(hipMemsetAsync(F, 0, (size_t)c->hs.N * P * sizeof(double), c->stream));
        SG_HIP_CHECK(hipMemcpy2DAsync(F, P * sizeof(double), c->load, sizeof(double), sizeof(double), c->hs.N,
                                      hipMemcpyDeviceToDevice, c->stream));
        return SG_OK;
    }
    const double h = 1.0 / c->hs.n;
    SG_HIP_CHECK(vec_rhs(c->stream, F, c->hs.N, c->hs.P, h * h));
    return SG_OK;
}

int sg_apply(sg_ctx* c, const void* U, void* Y, int prec) {
    if (!c || !U || !Y || (prec != SG_F64 && prec != SG_MIXED)) {
        set_error("sg_apply: invalid argument");
        return SG_EINVAL;
    }
    const int P = c->hs.P;
    return launch_apply(c, c->plan_full, U, prec == SG_MIXED, nullptr, Y, 0, P, P, P);
}

int sg_residual(sg_ctx* c, const double* F, const double* U, double* R) {
    if (!c || !F || !U || !R) {
        set_error("sg_residual: null argument");
        return SG_EINVAL;
    }
    const int P = c->hs.P;
    return launch_apply(c, c->plan_full, U, 0, F, R, 0, P, P, P);
}

int sg_vcycle(sg_ctx* c, const void* f, int ldf, void* u, int ldu, int width, int prec) {
    if (!c || !f || !u || width < 1 || width > c->hs.P || ldf < width || ldu < width ||
        (prec != SG_F64 && prec != SG_F32)) {
        set_error("sg_vcycle: invalid argument");
        return SG_EINVAL;
    }
    int rc = ensure_mg(c, prec == SG_F32);
    if (rc) return rc;
    return launch_vcycle(c, f, ldf, u, ldu, width, prec == SG_F32);
}

int sg_precond_diag(sg_ctx* c, const void* R, void* Z, int prec) {
    if (!c || !R || !Z || (prec != SG_F64 && prec != SG_MIXED)) {
        set_error("sg_precond_diag: invalid argument");
        return SG_EINVAL;
    }
    return precond_diag(c, (const double*)R, Z, prec == SG_MIXED);
}

int sg_precond_tri(sg_ctx* c, const void* R, void* Z, int prec) {
    if (!c || !R || !Z || (prec != SG_F64 && prec != SG_MIXED)) {
        set_error("sg_precond_tri: invalid argument");
        return SG_EINVAL;
    }
    return precond_tri(c, (const double*)R, Z, prec == SG_MIXED);
}

int sg_precond_sym(sg_ctx* c, const void* R, void* Z, int prec) {
    if (!c || !R || !Z || (prec != SG_F64 && prec != SG_MIXED)) {
        set_error("sg_precond_sym: invalid argument");
        return SG_EINVAL;
    }
    return precond_sym(c, (const double*)R, Z, prec == SG_MIXED);
}

int sg_precond_split(sg_ctx* c, const double* R, double* Z, int symmetric) {
    if (!c || !R || !Z || (symmetric != 0 && symmetric != 1)) {
        set_error("sg_precond_split: invalid argument");
        return SG_EINVAL;
    }
    return precond_split(c, R, Z, symmetric);
}

int sg_solve(sg_ctx* c, const double* F, double* U, const sg_solve_opts* opts, sg_solve_info* info_out) {
    if (!c || !F || !U || check_opts(c, opts) != SG_OK) {
        set_error("sg_solve: invalid argument or options");
        return SG_EINVAL;
    }
    sg_solve_info info;
    std::memset(&info, 0, sizeof(info));
    Timer tm;
    tm.init(opts->timing != 0);
    // work the caller queued earlier on the stream is not part of the solve's time
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        set_error("sg_solve: stream synchronisation failed before the solve");
        tm.done();
        return SG_EHIP;
    }
    auto t0 = std::chrono::steady_clock::now();
    int rc;
    switch (opts->solver) {
        case 0:
        case 4: rc = fgmres(c, F, U, *opts, info, tm); break;
        case 1: rc = pcg(c, F, U, *opts, info, tm); break;
        case 2: rc = gpcg1(c, F, U, *opts, info, tm); break;
        default: rc = block_gs(c, F, U, *opts, info, tm); break;
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess && rc == SG_OK) {
        set_error("sg_solve: stream synchronisation failed");
        rc = SG_EHIP;
    }
    auto t1 = std::chrono::steady_clock::now();
    info.t_total_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    info.t_apply_ms = tm.apply;
    info.t_prec_ms = tm.prec;
    info.t_orth_ms = tm.orth;
    info.n_apply = tm.napply;
    info.n_prec = tm.nprec;
    info.status = rc;
    tm.done();
    if (info_out) *info_out = info;
    return rc;
}

int sg_qoi(sg_ctx* c, const double* U, double* q, double* J) {
    if (!c || !U || !J || c->hs.disc != SG_DISC_Q1) {
        set_error("sg_qoi: null argument or a discretisation other than SG_DISC_Q1");
        return SG_EINVAL;
    }
    int rc = ensure_scalars(c);
    if (rc) return rc;
    const int P = c->hs.P;
    if (!c->ws.qv && (rc = dalloc(c, &c->ws.qv, 2 * (size_t)P + 8))) return rc;
    SG_HIP_CHECK(vec_qoi(c->stream, U, c->ws.wS, c->hs.N, P, c->ws.partial, c->ws.qv, c->ws.qv + 2 * P,
                         c->ws.qv + P));
    SG_HIP_CHECK(hipMemcpyAsync(c->ws.host_scal, c->ws.qv, (2 * P + 1) * sizeof(double), hipMemcpyDeviceToHost,
                                c->stream));
    SG_HIP_CHECK(hipStreamSynchronize(c->stream));
    if (q) std::memcpy(q, c->ws.host_scal, P * sizeof(double));
    *J = c->ws.host_scal[2 * P];
    return SG_OK;
}

int sg_qoi_noalloc(sg_ctx* c, const double* U, double* q, double* J) {
    if (!c || !U || !q || !J || c->hs.disc != SG_DISC_Q1 || !c->qoi_scratch) {
        set_error("sg_qoi_noalloc: null argument or a discretisation other than SG_DISC_Q1");
        return SG_EINVAL;
    }
    const int P = c->hs.P;
    if ((size_t)kRedBlocks * P + P > kQoiScratchDoubles) {
        set_error("sg_qoi_noalloc: P = " + std::to_string(P) + " needs more than the " +
                  std::to_string(kQoiScratchDoubles) + "-double scratch array");
        return SG_EINVAL;
    }
    // partials in rows of P (every entry written before it is read), adjoint weights after them
    double* partial = c->qoi_scratch;
    double* coef = c->qoi_scratch + (size_t)kRedBlocks * P;
    SG_HIP_CHECK(vec_qoi(c->stream, U, c->ws.wS, c->hs.N, P, partial, q, J, coef));
    return SG_OK;
}

int sg_qoi_grad(sg_ctx* c, const double* U, const sg_solve_opts* opts, double* J, double* dJ_dsigma, double* dJ_damp,
                double* dJ_da0, sg_solve_info* adj_info) {
    if (!c || !U || !J || !dJ_dsigma || (!dJ_damp && c->hs.m) || !dJ_da0 || c->hs.disc != SG_DISC_Q1 ||
        check_opts(c, opts) != SG_OK) {
        set_error("sg_qoi_grad: invalid argument");
        return SG_EINVAL;
    }
    int rc = sg_qoi(c, U, nullptr, J);
    if (rc) return rc;
    const size_t np = NP(c);
    const int n = c->hs.n, m = c->hs.m, P = c->hs.P, N = c->hs.N;
    if (!c->ws.lam && (rc = dalloc(c, &c->ws.lam, np))) return rc;
    if (!c->ws.g && (rc = dalloc(c, &c->ws.g, np))) return rc;
    if (!c->ws.dc && (rc = dalloc(c, &c->ws.dc, (size_t)n * n * (m + 1) + 16 + (size_t)N))) return rc;
    SG_HIP_CHECK(vec_adj_rhs(c->stream, c->ws.wS, c->ws.qv + P, N, P, c->ws.g));
    sg_solve_opts o = *opts;
    o.use_x0 = 0;
    // a solve stopped by max_it still yields a usable adjoint; report it in the status
    const int solve_rc = sg_solve(c, c->ws.g, c->ws.lam, &o, adj_info);
    if (solve_rc < 0 && solve_rc != SG_ENOTCONV) return solve_rc;
    SG_HIP_CHECK(vec_grad_cells(c->stream, c->plan_full.nslot, U, c->ws.lam, n, P, m, c->plan_full.d_off,
                                c->plan_full.d_coef, c->ws.dc));
    double* params = c->ws.scal + 600;  // 1 + m values
    double* Tk = c->ws.scal + 700;
    double* a0 = c->ws.dc + (size_t)n * n * (m + 1) + 16;
    SG_HIP_CHECK(vec_grad_params(c->stream, c->ws.dc, c->klcell, c->ws.amps, c->opt.sigma, n, m, c->ws.partial, Tk,
                                 params, a0));
    SG_HIP_CHECK(hipMemcpyAsync(c->ws.host_scal + 600, params, (1 + m) * sizeof(double), hipMemcpyDeviceToHost,
                                c->stream));
    SG_HIP_CHECK(hipMemcpyAsync(dJ_da0, a0, (size_t)N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    SG_HIP_CHECK(hipStreamSynchronize(c->stream));
    *dJ_dsigma = c->ws.host_scal[600];
    for (int k = 0; k < m; ++k) dJ_damp[k] = c->ws.host_scal[601 + k];
    return solve_rc;
}

int sg_setup_host(const sg_options* opt, const double* a0_nodal, const double* kl_amp, double* cell_coeffs,
                  double* fine_stencil, double* level1_stencil, double* coarsest_inverse, double* kl_lambda,
                  double* a_min_h) {
    if (!opt || opt->n_cells < 4 || opt->n_cells > 4096 || opt->n_cells % 4 || opt->m < 0 || opt->m > kMaxM ||
        opt->p < 0 || opt->p > 8 || opt->coarsest_cells < 2 || opt->coarsest_cells > opt->n_cells ||
        opt->n_cells % opt->coarsest_cells || !(opt->corr_len > 0.0) ||
        (opt->discretization != SG_DISC_Q1 && opt->discretization != SG_DISC_P1) ||
        (opt->discretization == SG_DISC_P1 && a0_nodal)) {
        set_error("sg_setup_host: invalid options");
        return SG_EINVAL;
    }
    HostSetup hs;
    const int rc = host_setup(*opt, a0_nodal, kl_amp, hs);
    if (rc < 0) return rc;
    if (cell_coeffs) std::memcpy(cell_coeffs, hs.cellc.data(), hs.cellc.size() * sizeof(double));
    if (fine_stencil) std::memcpy(fine_stencil, hs.mg_sten[0].data(), hs.mg_sten[0].size() * sizeof(double));
    if (level1_stencil && hs.mg_sten.size() > 1)
        std::memcpy(level1_stencil, hs.mg_sten[1].data(), hs.mg_sten[1].size() * sizeof(double));
    if (coarsest_inverse) std::memcpy(coarsest_inverse, hs.coarse_inv.data(), hs.coarse_inv.size() * sizeof(double));
    if (kl_lambda && hs.m) std::memcpy(kl_lambda, hs.lambda.data(), hs.m * sizeof(double));
    if (a_min_h) *a_min_h = hs.a_min_h;
    return rc;
}

int sg_sync(sg_ctx* c) {
    if (!c) return SG_EINVAL;
    SG_HIP_CHECK(hipStreamSynchronize(c->stream));
    return SG_OK;
}

void sg_destroy(sg_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (void* p : c->allocations) (void)hipFree(p);
    if (c->ws.host_scal) (void)hipHostFree(c->ws.host_scal);
    delete c;
}

}  // extern "C"
