// Matrix-free stochastic Galerkin operator (Sec. 3.1, eq. (tensor-product)):
//
//     Y = sum_{k=0..m} K_k U G_k^T        (U, Y: N x P node-major)
//
// and its two relatives that share the same kernel:
//   * the true residual  Y = R - A U;
//   * the lower coupling of the block-triangular sweep (Sec. 4.2):
//       Y_d = R_d - sum_{k>=1} [G_k]_{d,d-1} (x) K_k U_{d-1}.
//
// Design (gfx950): one workgroup walks a segment of one grid row, one node
// per step; its lanes (64 per wave, up to 4 waves) hold the P chaos modes of
// that node, so every load of a node's mode vector is a contiguous, coalesced
// access and the cell coefficients c_{k,e} of the four cells around the node
// are wave-uniform scalars, loaded once and reused by all modes.
// With cell-constant coefficients, K_k u at a node is sum over the four cells
// of c_{k,e} r_e, where r_e = 4u_c - (two edge neighbours in that cell)
// - 2 (opposite corner) is the node's row of the Q1 element matrix (times 6;
// the 1/6 is folded into the coefficients).  r_e is computed once per mode
// and shared by all m+1 stencils.  The G_k coupling (alpha <-> alpha +- e_k,
// Sec. 3.2) crosses lanes: each lane writes its K_k u (k >= 1) to an LDS
// exchange buffer and reads back the entries of its coupling partners through
// precomputed index/coefficient tables held in registers.  A 3x3 window of
// mode vectors slides along the row, so each step loads one new column.

#include <type_traits>

#include "sg_internal.h"

namespace sg {

namespace {

template <typename T>
__device__ __forceinline__ double ld_as_double(const T* p) { return (double)(*p); }

template <typename T>
__device__ __forceinline__ void st_from_double(T* p, double v) { *p = (T)v; }

__device__ __forceinline__ int remap_block_xcd(int b, int nb) {
    // blocks are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous range of logical blocks so neighbouring grid rows share an L2
    const int x = b & 7, i = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + i;
}

// One block per row segment; wave s of the block owns modes [64 s, 64 s + 64)
// of every node in the segment.  Per node, every wave writes its K_k u
// (k >= 1) into a block-shared LDS exchange buffer (double-buffered by node
// parity), the block meets at one barrier, and every wave then gathers its
// coupling partners from the whole buffer.  Splitting the modes over waves
// keeps each wave's coupling tables and 3x3 window small, so several blocks
// share a CU and hide memory latency.
template <int M, int NS, typename Tin, typename Tout>
__global__ void __launch_bounds__(NS * 64)
k_sg_apply(const Tin* __restrict__ U, int ldu, const double* __restrict__ R, int ldr,
           Tout* __restrict__ Y, int ldy, const double* __restrict__ cell,
           const uint32_t* __restrict__ toff, const double* __restrict__ tcoef, int n, int W_in,
           int W_out, int self, double rsign, int seg, int nseg) {
    constexpr int MM = M > 0 ? M : 1;
    constexpr int LANES = NS * 64;
    constexpr int BUF = MM * LANES + 2;
    __shared__ double S[2][BUF];
    const int lane = threadIdx.x & 63;
    const int s = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // this wave's slot (uniform)
    const int nx = n - 1;
    const int lb = remap_block_xcd(blockIdx.x, gridDim.x);
    if (lb >= nx * nseg) return;  // whole block
    const int y = lb / nseg;
    const int x0 = (lb - y * nseg) * seg;
    const int x1 = min(x0 + seg, nx);
    const int t = s * 64 + lane;
    const bool has_out = s * 64 < W_out;  // uniform
    const bool vin = t < W_in, vout = t < W_out;

    // this lane's partners: position 2k = alpha + e_k, 2k+1 = alpha - e_k
    uint32_t off[MM];
    double ce[2 * MM];
#pragma unroll
    for (int j = 0; j < MM; ++j) {
        off[j] = M > 0 ? toff[t * MM + j] : 0u;
        ce[2 * j] = M > 0 ? tcoef[t * 2 * MM + 2 * j] : 0.0;
        ce[2 * j + 1] = M > 0 ? tcoef[t * 2 * MM + 2 * j + 1] : 0.0;
    }
    if (threadIdx.x == 0) {
        S[0][MM * LANES] = 0.0;  // shared zero entry for absent partners
        S[1][MM * LANES] = 0.0;
    }

    // Window w[row][c] of mode vectors: rows y-1, y, y+1, columns x-1, x, x+1
    // at step x.  Step x takes column x+1 (and R at x) from ring slot
    // (x - x0) mod 4, filled four steps earlier, so the loads of the walk are
    // in flight while earlier steps compute.  Load addresses are clamped into
    // the grid and the value replaced by zero outside it, so the loads need
    // no branches; the walk is unrolled by 4, which makes the slot and the
    // LDS buffer parity compile-time constants.
    constexpr int D = 4;
    const int tci = vin ? t : (W_in > 0 ? W_in - 1 : 0);
    const int tco = vout ? t : W_out - 1;
    const int ydn = y > 0 ? y - 1 : 0, yup = y + 1 < nx ? y + 1 : nx - 1;
    const bool rdn = y > 0, rup = y + 1 < nx;
    auto ldU = [&](int yy, int xc) -> Tin {
        const int xcl = min(max(xc, 0), nx - 1);
        return U[((size_t)yy * nx + xcl) * ldu + tci];
    };
    auto zU = [&](Tin v, bool rowok, int xc) -> double {
        return (rowok && vin && xc >= 0 && xc < nx) ? (double)v : 0.0;
    };
    // R is never null here (a zero vector with ldr = 0 stands in when no
    // right-hand side is given) and the output is R + rsign * (A U)
    Tin qd[D], qc[D], qu[D];
    double qr[D];
    auto issue = [&](int k, int x) {  // column x+1 and R at x, for step x
        qd[k] = ldU(ydn, x + 1);
        qc[k] = ldU(y, x + 1);
        qu[k] = ldU(yup, x + 1);
        qr[k] = R[((size_t)y * nx + min(x, nx - 1)) * ldr + tco];
    };
    double w[3][3];
    w[0][0] = zU(ldU(ydn, x0 - 1), rdn, x0 - 1);
    w[1][0] = zU(ldU(y, x0 - 1), true, x0 - 1);
    w[2][0] = zU(ldU(yup, x0 - 1), rup, x0 - 1);
    w[0][1] = zU(ldU(ydn, x0), rdn, x0);
    w[1][1] = zU(ldU(y, x0), true, x0);
    w[2][1] = zU(ldU(yup, x0), rup, x0);
#pragma unroll
    for (int k = 0; k < D; ++k) issue(k, x0 + k);

    auto step = [&](auto kstep, int x) {
        constexpr int k = decltype(kstep)::value;  // ring slot and LDS buffer parity
        double* B = S[k & 1];
        w[0][2] = zU(qd[k], rdn, x + 1);
        w[1][2] = zU(qc[k], true, x + 1);
        w[2][2] = zU(qu[k], rup, x + 1);
        const double rv = qr[k];
        issue(k, x + D);  // clamped: past the segment these loads are harmless
        double s0 = 0.0;
        {
            // four cells around the node: SW (x, y), SE (x+1, y), NW (x, y+1), NE (x+1, y+1)
            const double* cSW = cell + ((size_t)y * n + x) * (M + 1);
            const double* cSE = cSW + (M + 1);
            const double* cNW = cell + ((size_t)(y + 1) * n + x) * (M + 1);
            const double* cNE = cNW + (M + 1);
            const double uc4 = 4.0 * w[1][1];
            const double rSW = fma(-2.0, w[0][0], uc4 - (w[0][1] + w[1][0]));
            const double rSE = fma(-2.0, w[0][2], uc4 - (w[0][1] + w[1][2]));
            const double rNW = fma(-2.0, w[2][0], uc4 - (w[2][1] + w[1][0]));
            const double rNE = fma(-2.0, w[2][2], uc4 - (w[2][1] + w[1][2]));
            s0 = fma(cSW[0], rSW, fma(cSE[0], rSE, fma(cNW[0], rNW, cNE[0] * rNE)));
#pragma unroll
            for (int kk = 1; kk <= M; ++kk)
                B[(kk - 1) * LANES + t] = fma(cSW[kk], rSW, fma(cSE[kk], rSE, fma(cNW[kk], rNW, cNE[kk] * rNE)));
        }
        // LDS writes done, then the block barrier (no global-memory wait: the
        // ring loads stay in flight)
        __builtin_amdgcn_s_waitcnt(0xC07F);
        __asm__ __volatile__("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        __asm__ __volatile__("" ::: "memory");
        if (has_out) {
            double acc = self ? s0 : 0.0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                // absent partners read the shared zero entry: unconditional
                // gathers schedule better than skipping positions per wave
                acc = fma(ce[2 * j], B[off[j] & 0xFFFFu], acc);
                acc = fma(ce[2 * j + 1], B[off[j] >> 16], acc);
            }
            if (vout) {
                const size_t node = (size_t)y * nx + x;
                st_from_double(Y + node * ldy + t, fma(rsign, acc, rv));
            }
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            w[r][0] = w[r][1];
            w[r][1] = w[r][2];
        }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    for (int x = x0; x < x1; x += 4) {
        // x, x1 are uniform, so every wave of the block meets the same barriers
        step(I0{}, x);
        if (x + 1 < x1) step(I1{}, x + 1);
        if (x + 2 < x1) step(I2{}, x + 2);
        if (x + 3 < x1) step(I3{}, x + 3);
    }
}

template <typename Tin, typename Tout, int M, int NS>
hipError_t launch_t(hipStream_t st, const Plan& pl, const void* U, int ldu, const double* R, int ldr, void* Y,
                    int ldy, const double* cell, int n, double rsign) {
    const int nx = n - 1;
    const int seg = 32;
    const int nseg = (nx + seg - 1) / seg;
    const int blocks = nx * nseg;
    hipLaunchKernelGGL((k_sg_apply<M, NS, Tin, Tout>), dim3(blocks), dim3(NS * 64), 0, st,
                       (const Tin*)U, ldu, R, ldr, (Tout*)Y, ldy, cell, pl.d_off, pl.d_coef, n, pl.W_in, pl.W_out, pl.self,
                       rsign, seg, nseg);
    return hipGetLastError();
}

template <typename Tin, typename Tout, int M>
hipError_t launch_ns(hipStream_t st, const Plan& pl, const void* U, int ldu, const double* R, int ldr, void* Y,
                     int ldy, const double* cell, int n, double rsign) {
    switch (pl.nslot) {
        case 1: return launch_t<Tin, Tout, M, 1>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, rsign);
        case 2: return launch_t<Tin, Tout, M, 2>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, rsign);
        case 3: return launch_t<Tin, Tout, M, 3>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, rsign);
        case 4: return launch_t<Tin, Tout, M, 4>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, rsign);
    }
    return hipErrorInvalidValue;
}

template <typename Tin, typename Tout>
hipError_t launch_m(hipStream_t st, int m, const Plan& pl, const void* U, int ldu, const double* R, int ldr,
                    void* Y, int ldy, const double* cell, int n, double rsign) {
    switch (m) {
        case 0: return launch_ns<Tin, Tout, 0>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, rsign);
        case 1: return launch_ns<Tin, Tout, 1>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, rsign);
        case 2: return launch_ns<Tin, Tout, 2>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, rsign);
        case 3: return launch_ns<Tin, Tout, 3>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, rsign);
        case 4: return launch_ns<Tin, Tout, 4>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, rsign);
        case 5: return launch_ns<Tin, Tout, 5>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, rsign);
        case 6: return launch_ns<Tin, Tout, 6>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, rsign);
        case 7: return launch_ns<Tin, Tout, 7>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, rsign);
        case 8: return launch_ns<Tin, Tout, 8>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, rsign);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int launch_apply(sg_ctx* c, const Plan& pl, const void* U, int in_float, const double* R, void* Y, int out_float,
                 int ldu, int ldy, int ldr) {
    hipError_t e;
    const int m = c->hs.m, n = c->hs.n;
    // Y = R - A U, or Y = A U with a zero right-hand side
    const double rsign = R ? -1.0 : 1.0;
    if (!R) {
        R = c->zeros;
        ldr = 0;
    }
    if (!in_float && !out_float)
        e = launch_m<double, double>(c->stream, m, pl, U, ldu, R, ldr, Y, ldy, c->cell64, n, rsign);
    else if (in_float && !out_float)
        e = launch_m<float, double>(c->stream, m, pl, U, ldu, R, ldr, Y, ldy, c->cell64, n, rsign);
    else if (in_float && out_float)
        e = launch_m<float, float>(c->stream, m, pl, U, ldu, R, ldr, Y, ldy, c->cell64, n, rsign);
    else {
        set_error("apply: double input with float output is not provided");
        return SG_EINVAL;
    }
    if (e != hipSuccess) {
        set_error(std::string("apply launch: ") + hipGetErrorString(e));
        return SG_EHIP;
    }
    return SG_OK;
}

}  // namespace sg
