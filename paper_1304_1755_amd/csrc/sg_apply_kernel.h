// Matrix-free stochastic Galerkin operator (Sec. 3.1, eq. (tensor-product)):
//
//     Y = sum_{k=0..m} K_k U G_k^T        (U, Y: N x P node-major)
//
// and its two relatives that share the same kernel:
//   * the true residual  Y = R - A U;
//   * the lower coupling of the block-triangular sweep (Sec. 4.2):
//       Y_d = R_d - sum_{k>=1} [G_k]_{d,d-1} (x) K_k U_{d-1}.
//
// Design (gfx950): one workgroup walks a segment of a pair of grid rows,
// one node column per step; its lanes (64 per wave, up to 4 waves) hold the P
// chaos modes of those nodes, so every load of a node's mode vector is a
// contiguous, coalesced access and the element coefficients around the node
// are wave-uniform scalars, loaded once and reused by all modes.
// Bilinear elements (TRI = false): with cell-constant coefficients, K_k u at
// a node is sum over the four cells of c_{k,e} r_e, where r_e = 4u_c - (two
// edge neighbours in that cell) - 2 (opposite corner) is the node's row of
// the Q1 element matrix (times 6; the 1/6 is folded into the coefficients).
// Linear elements on the south-west to north-east split (TRI = true, Sec. 6):
// K_k u at a node is sum over its four grid edges of w_{k,e} (u_c - u_e).
// The per-node differences are computed once per mode and shared by all m+1
// stencils.  The G_k coupling (alpha <-> alpha +- e_k, Sec. 3.2) crosses
// lanes: each lane writes its K_k u (k >= 1) to an LDS exchange buffer, two k
// per 128-bit store, and reads back its coupling partners.  The partners of
// a lane are listed by the value of their coefficient G_k(alpha, beta), which
// takes only p values: inside one wavefront every list position then has one
// coefficient for all lanes, held in scalar registers, and only the partner
// indices (16 bits each) stay in vector registers.  A 3x4 window of mode
// vectors slides along the rows, so each step loads one new column.
//
// This header holds the kernel and its launchers; each discretisation is
// instantiated in a translation unit of its own.
#pragma once

#include <type_traits>
#include <utility>

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

constexpr int kApplyRows = 2;        // grid rows per workgroup
// below this many wavefronts a launch takes shorter segments (narrow coupling plans, small grids):
// a workgroup of fewer wavefronts keeps fewer loads in flight per column, so launches of at most
// three wavefronts per workgroup ask for four times as many (c4: 1.5 % faster solves, the full
// 165-mode apply 2 %; the four-wavefront apply at c3 is fastest with the lower bound)
constexpr int kMinApplyWaves = 16384;
constexpr int min_apply_waves(int ns) { return ns >= 4 ? kMinApplyWaves : 4 * kMinApplyWaves; }

template <typename F, int... J>
__device__ __forceinline__ void unroll_steps(F&& f, std::integer_sequence<int, J...>) {
    (f(std::integral_constant<int, J>{}), ...);
}

// One workgroup per segment of RW grid rows (a row pair for RW = 2); wave s
// of the workgroup owns modes [64 s, 64 s + 64) of every node in the
// segment.  Per column, every wave writes the K_k u (k >= 1) of its RW nodes
// into a block-shared LDS exchange buffer, the workgroup meets at a barrier,
// and every wave then gathers its coupling partners from the whole buffer.
// Splitting the modes over waves keeps each wave's window and partner lists
// small, so several workgroups share a CU and hide memory latency; two rows
// per workgroup share the window's middle rows and the cell row between them,
// and halve the synchronizations per node.
template <int M, int NS, int RW, typename Tin, typename Tout, bool HAS_R, bool TRI, int NB>
__global__ void __launch_bounds__(NS * 64)
k_sg_apply(const Tin* __restrict__ U, int ldu, const double* __restrict__ R, int ldr,
           Tout* __restrict__ Y, int ldy, const double* __restrict__ cell,
           const uint32_t* __restrict__ xoff, const double* __restrict__ xcoef, const int* __restrict__ npos_slot,
           int n, int W_in, int W_out, int self, const Tin* __restrict__ zin, int seg, int nseg) {
    constexpr int MM = M > 0 ? M : 1;
    constexpr int LANES = NS * 64;
    constexpr int NODE = MM * LANES + 2;  // exchange entries of one node (+ its zero entry; even: 16-byte rows)
    __shared__ __attribute__((aligned(16))) double S[RW * NODE];
    const int lane = threadIdx.x & 63;
    const int s = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // this wave's slot (uniform)
    const int nx = n - 1;
    const int lb = remap_block_xcd(blockIdx.x, gridDim.x);
    const int nrb = (nx + RW - 1) / RW;
    if (lb >= nrb * nseg) return;  // whole block
    // segment-major: the row blocks of one column segment are consecutive, so
    // the workgroups that share a halo row run at the same time on one XCD
    const int sgi = lb / nrb;
    const int yb = lb - sgi * nrb;
    const int y0 = yb * RW;
    const int x0 = sgi * seg;
    const int x1 = min(x0 + seg, nx);
    const int t = s * 64 + lane;
    const bool has_out = s * 64 < W_out;  // uniform
    const bool vin = t < W_in, vout = t < W_out;
    // this lane's partner list (16-bit exchange indices) and the slot's
    // per-position coefficients (uniform) and number of used positions
    (void)npos_slot;  // the launch picks NB >= every slot's ceil(npos / 4)
    const double* cw = xcoef + s * kNPos;
    uint32_t off[2 * NB];
#pragma unroll
    for (int j = 0; j < 2 * NB; ++j) off[j] = xoff[t * (kNPos / 2) + j];
    SG_POISON_LDS(S, RW * NODE);
    if (threadIdx.x < RW) S[threadIdx.x * NODE + MM * LANES] = 0.0;  // zero entries

    // Circular window wb[row][c] of mode vectors, rows y0-1 .. y0+RW: column
    // x of the grid lives in wb[.][(x - x0 + 1) mod C].  Step x reads columns
    // x-1, x, x+1 and issues the loads of column x+1+D, so D columns are in
    // flight while earlier steps compute; the walk is unrolled by C, which
    // makes every column role and the R slot a compile-time constant and the
    // window needs no register moves.  A neighbour outside the grid is read
    // from the zero vector zin (a wave-uniform choice of base pointer, so no
    // per-value select), and lanes past W_in read a valid column: their
    // values feed no partner.
    constexpr int C = 4;
    constexpr int D = C - 3;  // columns in flight
    constexpr int NR = RW + 2;
    const uint32_t tci = vin ? t : W_in - 1;
    const uint32_t tco = vout ? t : W_out - 1;
    Tin wb[NR][C];
    double qr[RW][D];  // R at (x, y0 + q) lives in qr[q][(x - x0) mod D]
    // row bases, computed once: the window rows y0-1 .. y0+RW (and which lie in
    // the grid), the R and Y rows of the segment's nodes
    const Tin* rowb[NR];
    bool rowin[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int yy = y0 + r - 1;
        rowin[r] = yy >= 0 && yy < nx;
        rowb[r] = U + (size_t)(rowin[r] ? yy : 0) * nx * ldu;
    }
    const double* rrow[RW];
    Tout* yrow[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
        const int yq = min(y0 + q, nx - 1);
        rrow[q] = HAS_R ? R + (size_t)yq * nx * ldr : R;
        yrow[q] = Y + (size_t)yq * nx * ldy;
    }
    // coefficient rows y0 .. y0+RW (cells, or vertices for TRI): (M+1) or 2(M+1) values per position
    const double* crow[RW + 1];
#pragma unroll
    for (int r = 0; r <= RW; ++r) crow[r] = cell + (size_t)min(y0 + r, n - 1) * n * (TRI ? 2 * (M + 1) : M + 1);
    auto load_col = [&](int c, int xc) {
        const bool colin = xc >= 0 && xc < nx;  // uniform
        const size_t xo = (size_t)(colin ? xc : 0) * ldu;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const Tin* rowp = (rowin[r] && colin) ? rowb[r] + xo : zin;
            wb[r][c] = rowp[tci];
        }
    };
    auto load_r = [&](int c, int x) {
        if (HAS_R) {
            const size_t xo = (size_t)min(x, nx - 1) * ldr;
#pragma unroll
            for (int q = 0; q < RW; ++q) qr[q][c % D] = rrow[q][xo + tco];
        }
    };
    // columns x0-1 .. x0+D and R at x0 .. x0+D-1
    load_col(0, x0 - 1);
    load_col(1, x0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
        load_col(2 + i, x0 + 1 + i);
        load_r(i, x0 + i);
    }

    auto step = [&](auto kstep, int x) {
        constexpr int j = decltype(kstep)::value;  // x - x0 mod C
        constexpr int cW = j % C, cC = (j + 1) % C, cE = (j + 2) % C, cL = (j + 2 + D) % C;
        double rv[RW];
#pragma unroll
        for (int q = 0; q < RW; ++q) rv[q] = HAS_R ? qr[q][j % D] : 0.0;
        load_col(cL, x + 1 + D);  // past the segment: zero-vector or in-grid loads, harmless
        load_r(j, x + D);         // the slot just read
        double s0[RW];
#pragma unroll
        for (int q = 0; q < RW; ++q) {
            s0[q] = 0.0;
            if (RW > 1 && y0 + q >= nx) break;  // uniform: no such row (its cells would lie outside)
            double* Bq = S + q * NODE;
            const double wS = (double)wb[q][cC];
            const double wW = (double)wb[q + 1][cW], wc = (double)wb[q + 1][cC], wE = (double)wb[q + 1][cE];
            const double wN = (double)wb[q + 2][cC];
            // K_k u of this node for k = 1..M into the exchange row, pairs of k per 128-bit store
            auto put = [&](auto stencil) {
#pragma unroll
                for (int kk = 0; kk < 2 * (M / 2); kk += 2) {
                    double2 v;
                    v.x = stencil(kk + 1);
                    v.y = stencil(kk + 2);
                    *(double2*)(Bq + exchange_index(M, LANES, kk, t)) = v;
                }
                if constexpr ((M & 1) != 0) Bq[exchange_index(M, LANES, M - 1, t)] = stencil(M);
            };
            if constexpr (TRI) {
                // node (x, y0 + q) is grid vertex (x+1, y0+q+1); 2(M+1) weights per vertex:
                // its east edges for k = 0..M, then its north edges.  West edge = east
                // edge of vertex (x, y0+q+1); south edge = north edge of vertex (x+1, y0+q).
                constexpr int CW = 2 * (M + 1);
                const double* pC = crow[q + 1] + (x + 1) * CW;
                const double* pW = pC - CW;
                const double* pS = crow[q] + (x + 1) * CW + (M + 1);
                const double* pN = pC + (M + 1);
                const double dE = wc - wE, dW = wc - wW, dN = wc - wN, dS = wc - wS;
                auto stencil = [&](int kk) { return fma(pC[kk], dE, fma(pW[kk], dW, fma(pN[kk], dN, pS[kk] * dS))); };
                s0[q] = stencil(0);
                put(stencil);
            } else {
                // node (x, y0 + q); cells SW (x, y0+q), SE (x+1, y0+q), NW (x, y0+q+1), NE (x+1, y0+q+1)
                const double wSW = (double)wb[q][cW], wSE = (double)wb[q][cE];
                const double wNW = (double)wb[q + 2][cW], wNE = (double)wb[q + 2][cE];
                const double* cSW = crow[q] + x * (M + 1);
                const double* cSE = cSW + (M + 1);
                const double* cNW = crow[q + 1] + x * (M + 1);
                const double* cNE = cNW + (M + 1);
                const double uc4 = 4.0 * wc;
                const double rSW = fma(-2.0, wSW, uc4 - (wS + wW));
                const double rSE = fma(-2.0, wSE, uc4 - (wS + wE));
                const double rNW = fma(-2.0, wNW, uc4 - (wN + wW));
                const double rNE = fma(-2.0, wNE, uc4 - (wN + wE));
                auto stencil = [&](int kk) {
                    return fma(cSW[kk], rSW, fma(cSE[kk], rSE, fma(cNW[kk], rNW, cNE[kk] * rNE)));
                };
                s0[q] = stencil(0);
                put(stencil);
            }
        }
        // LDS writes done, then the block barrier (no global-memory wait: the
        // window loads stay in flight)
        __builtin_amdgcn_s_waitcnt(0xC07F);
        __asm__ __volatile__("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        __asm__ __volatile__("" ::: "memory");
        if (has_out) {
#pragma unroll
            for (int q = 0; q < RW; ++q) {
                if (RW > 1 && y0 + q >= nx) break;  // uniform: the last row pair of an odd grid
                const double* Bq = S + q * NODE;
                double acc0 = self ? s0[q] : 0.0, acc1 = 0.0;
                // NB blocks of four positions, enough for every slot of the
                // plan; unused positions read the zero entry with coefficient 0
                // (no per-block branch: the gathers of all blocks issue together)
#pragma unroll
                for (int blk = 0; blk < NB; ++blk) {
                    const double v0 = Bq[off[2 * blk] & 0xFFFFu], v1 = Bq[off[2 * blk] >> 16];
                    const double v2 = Bq[off[2 * blk + 1] & 0xFFFFu], v3 = Bq[off[2 * blk + 1] >> 16];
                    acc0 = fma(cw[4 * blk], v0, acc0);
                    acc1 = fma(cw[4 * blk + 1], v1, acc1);
                    acc0 = fma(cw[4 * blk + 2], v2, acc0);
                    acc1 = fma(cw[4 * blk + 3], v3, acc1);
                }
                const double acc = acc0 + acc1;
                if (vout) st_from_double(yrow[q] + (size_t)x * ldy + t, HAS_R ? rv[q] - acc : acc);
            }
        }
        // every wave has gathered before the next column is written
        __builtin_amdgcn_s_waitcnt(0xC07F);
        __asm__ __volatile__("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        __asm__ __volatile__("" ::: "memory");
    };
    for (int x = x0; x < x1; x += C) {
        // x, x1 are uniform, so every wave of the block meets the same barriers
        unroll_steps(
            [&](auto kj) {
                constexpr int j = decltype(kj)::value;
                if (j == 0 || x + j < x1) step(kj, x + j);
            },
            std::make_integer_sequence<int, C>{});
    }
}

// blocks of four partner positions a kernel holds for m KL terms: enough for
// every slot of the full plan at any p with P <= 256 (at most 8, 12, 14, 12, 13,
// 11, 10, 11 positions for m = 1..8); coupling plans that need more take 4
template <int M>
constexpr int nb_for_m() { return M <= 0 ? 1 : M == 1 ? 2 : (M == 3 || M == 5) ? 4 : 3; }

template <typename Tin, typename Tout, int M, int NS, bool TRI, int NB>
hipError_t launch_t(hipStream_t st, const Plan& pl, const void* U, int ldu, const double* R, int ldr, void* Y,
                    int ldy, const double* cell, int n, const void* zin) {
    constexpr int RW = kApplyRows;
    const int nx = n - 1;
    // 32-node segments; on small grids shorter ones, down to 8, so that the launch still has
    // enough wavefronts to cover the chip (each segment's walk is sequential)
    int seg = 32;
    while (seg > 8 && (long)((nx + RW - 1) / RW) * ((nx + seg - 1) / seg) * NS < min_apply_waves(NS)) seg >>= 1;
    const int nseg = (nx + seg - 1) / seg;
    const int blocks = (nx + RW - 1) / RW * nseg;
    if (R)
        hipLaunchKernelGGL((k_sg_apply<M, NS, RW, Tin, Tout, true, TRI, NB>), dim3(blocks), dim3(NS * 64), 0, st,
                           (const Tin*)U, ldu, R, ldr, (Tout*)Y, ldy, cell, pl.d_xoff, pl.d_xcoef, pl.d_npos, n, pl.W_in,
                           pl.W_out, pl.self, (const Tin*)zin, seg, nseg);
    else
        hipLaunchKernelGGL((k_sg_apply<M, NS, RW, Tin, Tout, false, TRI, NB>), dim3(blocks), dim3(NS * 64), 0, st,
                           (const Tin*)U, ldu, R, ldr, (Tout*)Y, ldy, cell, pl.d_xoff, pl.d_xcoef, pl.d_npos, n, pl.W_in,
                           pl.W_out, pl.self, (const Tin*)zin, seg, nseg);
    return hipGetLastError();
}

template <typename Tin, typename Tout, int M, bool TRI, int NB>
hipError_t launch_nb(hipStream_t st, const Plan& pl, const void* U, int ldu, const double* R, int ldr, void* Y,
                     int ldy, const double* cell, int n, const void* zin) {
    switch (pl.nslot) {
        case 1: return launch_t<Tin, Tout, M, 1, TRI, NB>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
        case 2: return launch_t<Tin, Tout, M, 2, TRI, NB>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
        case 3: return launch_t<Tin, Tout, M, 3, TRI, NB>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
        case 4: return launch_t<Tin, Tout, M, 4, TRI, NB>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
    }
    return hipErrorInvalidValue;
}

template <typename Tin, typename Tout, int M, bool TRI>
hipError_t launch_ns(hipStream_t st, const Plan& pl, const void* U, int ldu, const double* R, int ldr, void* Y,
                     int ldy, const double* cell, int n, const void* zin) {
    constexpr int NB = nb_for_m<M>();
    if (pl.nblk_max <= NB) return launch_nb<Tin, Tout, M, TRI, NB>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
    if constexpr (NB < kNPos / 4)
        return launch_nb<Tin, Tout, M, TRI, kNPos / 4>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
    return hipErrorInvalidValue;
}

template <typename Tin, typename Tout, bool TRI>
hipError_t launch_m(hipStream_t st, int m, const Plan& pl, const void* U, int ldu, const double* R, int ldr,
                    void* Y, int ldy, const double* cell, int n, const void* zin) {
    switch (m) {
        case 0: return launch_ns<Tin, Tout, 0, TRI>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
        case 1: return launch_ns<Tin, Tout, 1, TRI>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
        case 2: return launch_ns<Tin, Tout, 2, TRI>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
        case 3: return launch_ns<Tin, Tout, 3, TRI>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
        case 4: return launch_ns<Tin, Tout, 4, TRI>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
        case 5: return launch_ns<Tin, Tout, 5, TRI>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
        case 6: return launch_ns<Tin, Tout, 6, TRI>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
        case 7: return launch_ns<Tin, Tout, 7, TRI>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
        case 8: return launch_ns<Tin, Tout, 8, TRI>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n, zin);
    }
    return hipErrorInvalidValue;
}

// Y = R - A U, or Y = A U when R is null, for one discretisation
template <bool TRI>
int launch_apply_disc(sg_ctx* c, const Plan& pl, const void* U, int in_float, const double* R, void* Y,
                      int out_float, int ldu, int ldy, int ldr) {
    hipError_t e;
    const int m = c->hs.m, n = c->hs.n;
    const void* zin = c->zeros;  // the zero neighbour outside the grid
    if (!in_float && !out_float)
        e = launch_m<double, double, TRI>(c->stream, m, pl, U, ldu, R, ldr, Y, ldy, c->cell64, n, zin);
    else if (in_float && !out_float)
        e = launch_m<float, double, TRI>(c->stream, m, pl, U, ldu, R, ldr, Y, ldy, c->cell64, n, zin);
    else if (in_float && out_float)
        e = launch_m<float, float, TRI>(c->stream, m, pl, U, ldu, R, ldr, Y, ldy, c->cell64, n, zin);
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

}  // namespace

}  // namespace sg
