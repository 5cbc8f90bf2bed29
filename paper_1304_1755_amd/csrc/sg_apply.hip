// Matrix-free stochastic Galerkin operator (Sec. 3.1, eq. (tensor-product)):
//
//     Y = sum_{k=0..m} K_k U G_k^T        (U, Y: N x P node-major)
//
// and its two relatives that share the same kernel:
//   * the true residual  Y = R - A U;
//   * the lower coupling of the block-triangular sweep (Sec. 4.2):
//       Y_d = R_d - sum_{k>=1} [G_k]_{d,d-1} (x) K_k U_{d-1}.
//
// Design (gfx950): one wavefront walks a segment of one grid row, one node
// per step; its 64 lanes (times up to 4 slots) hold the P chaos modes of that
// node, so every load of a node's mode vector is a contiguous, coalesced
// 512-byte access and the cell coefficients c_{k,e} of the four cells around
// the node are wave-uniform scalars, loaded once and reused by all modes.
// With cell-constant coefficients, K_k u at a node is sum over the four cells
// of c_{k,e} r_e, where r_e = 4u_c - (two edge neighbours in that cell)
// - 2 (opposite corner) is the node's row of the Q1 element matrix (times 6;
// the 1/6 is folded into the coefficients).  r_e is computed once per mode
// and shared by all m+1 stencils.  The G_k coupling (alpha <-> alpha +- e_k,
// Sec. 3.2) crosses lanes: each lane writes its K_k u (k >= 1) to a per-wave
// LDS buffer and reads back the entries of its coupling partners through
// precomputed index/coefficient tables held in registers.  A 3x3 window of
// mode vectors slides along the row, so each step loads one new column.

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

template <int M, int NS, typename Tin, typename Tout>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
k_sg_apply(const Tin* __restrict__ U, int ldu, const double* __restrict__ R, int ldr,
           Tout* __restrict__ Y, int ldy, const double* __restrict__ cell,
           const uint32_t* __restrict__ toff, const double* __restrict__ tcoef, int n, int W_in,
           int W_out, int self, int seg, int nseg) {
    constexpr int MM = M > 0 ? M : 1;
    constexpr int LANES = NS * 64;
    constexpr int WBUF = MM * LANES + 2;
    extern __shared__ double lds_raw[];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    double* S = lds_raw + wv * WBUF;
    const int nx = n - 1;
    const int lb = remap_block_xcd(blockIdx.x, gridDim.x);
    const int gw = lb * (blockDim.x >> 6) + wv;
    if (gw >= nx * nseg) return;  // whole wave
    const int y = gw / nseg;
    const int x0 = (gw - y * nseg) * seg;
    const int x1 = min(x0 + seg, nx);

    // coupling tables of this lane's output modes
    uint32_t off[NS][MM];
    double cu[NS][MM], cd[NS][MM];
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int k = 0; k < MM; ++k) {
            const int t = (s * 64 + lane) * MM + k;
            off[s][k] = M > 0 ? toff[t] : 0u;
            cu[s][k] = M > 0 ? tcoef[2 * t] : 0.0;
            cd[s][k] = M > 0 ? tcoef[2 * t + 1] : 0.0;
        }
    if (lane == 0) S[MM * LANES] = 0.0;  // shared zero entry for absent partners

    bool vin[NS], vout[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        vin[s] = s * 64 + lane < W_in;
        vout[s] = s * 64 + lane < W_out;
    }

    // window w[s][row][col]: rows y-1, y, y+1; columns x-1, x, x+1
    double w[NS][3][3];
    auto load_col = [&](int col, int xc) {
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const int yy = y + r - 1;
            const bool ok = (xc >= 0) && (xc < nx) && (yy >= 0) && (yy < nx);
            const Tin* base = U + ((size_t)yy * nx + xc) * ldu + lane;
#pragma unroll
            for (int s = 0; s < NS; ++s) w[s][r][col] = (ok && vin[s]) ? ld_as_double(base + s * 64) : 0.0;
        }
    };
    load_col(0, x0 - 1);
    load_col(1, x0);

    for (int x = x0; x < x1; ++x) {
        load_col(2, x + 1);
        // four cells around the node: SW (x, y), SE (x+1, y), NW (x, y+1), NE (x+1, y+1)
        const double* cSW = cell + ((size_t)y * n + x) * (M + 1);
        const double* cSE = cSW + (M + 1);
        const double* cNW = cell + ((size_t)(y + 1) * n + x) * (M + 1);
        const double* cNE = cNW + (M + 1);
        double s0[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            s0[s] = 0.0;
            if (s * 64 >= W_in) continue;
            const double uc4 = 4.0 * w[s][1][1];
            const double rSW = fma(-2.0, w[s][0][0], uc4 - (w[s][0][1] + w[s][1][0]));
            const double rSE = fma(-2.0, w[s][0][2], uc4 - (w[s][0][1] + w[s][1][2]));
            const double rNW = fma(-2.0, w[s][2][0], uc4 - (w[s][2][1] + w[s][1][0]));
            const double rNE = fma(-2.0, w[s][2][2], uc4 - (w[s][2][1] + w[s][1][2]));
            s0[s] = fma(cSW[0], rSW, fma(cSE[0], rSE, fma(cNW[0], rNW, cNE[0] * rNE)));
#pragma unroll
            for (int k = 1; k <= M; ++k) {
                const double sk = fma(cSW[k], rSW, fma(cSE[k], rSE, fma(cNW[k], rNW, cNE[k] * rNE)));
                S[(k - 1) * LANES + s * 64 + lane] = sk;
            }
        }
        // make this wave's LDS writes visible to its own later reads
        __builtin_amdgcn_s_waitcnt(0xC07F);
        __asm__ __volatile__("" ::: "memory");
        const size_t node = (size_t)y * nx + x;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (s * 64 >= W_out) continue;
            double acc = self ? s0[s] : 0.0;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const uint32_t o = off[s][k];
                acc = fma(cu[s][k], S[o & 0xFFFFu], acc);
                acc = fma(cd[s][k], S[o >> 16], acc);
            }
            if (vout[s]) {
                if (R) acc = R[node * ldr + s * 64 + lane] - acc;
                st_from_double(Y + node * ldy + s * 64 + lane, acc);
            }
        }
        __builtin_amdgcn_s_waitcnt(0xC07F);
        __asm__ __volatile__("" ::: "memory");
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                w[s][r][0] = w[s][r][1];
                w[s][r][1] = w[s][r][2];
            }
    }
}

template <typename Tin, typename Tout, int M, int NS>
hipError_t launch_t(hipStream_t st, const Plan& pl, const void* U, int ldu, const double* R, int ldr, void* Y,
                    int ldy, const double* cell, int n) {
    const int nx = n - 1;
    const int seg = 64;
    const int nseg = (nx + seg - 1) / seg;
    const int waves = nx * nseg;
    const int wpb = 4;
    const int blocks = (waves + wpb - 1) / wpb;
    const size_t shm = (size_t)wpb * ((M > 0 ? M : 1) * NS * 64 + 2) * sizeof(double);
    hipLaunchKernelGGL((k_sg_apply<M, NS, Tin, Tout>), dim3(blocks), dim3(wpb * 64), shm, st,
                       (const Tin*)U, ldu, R, ldr, (Tout*)Y, ldy, cell, pl.d_off, pl.d_coef, n, pl.W_in, pl.W_out, pl.self,
                       seg, nseg);
    return hipGetLastError();
}

template <typename Tin, typename Tout, int M>
hipError_t launch_ns(hipStream_t st, const Plan& pl, const void* U, int ldu, const double* R, int ldr, void* Y,
                     int ldy, const double* cell, int n) {
    switch (pl.nslot) {
        case 1: return launch_t<Tin, Tout, M, 1>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n);
        case 2: return launch_t<Tin, Tout, M, 2>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n);
        case 3: return launch_t<Tin, Tout, M, 3>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n);
        case 4: return launch_t<Tin, Tout, M, 4>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n);
    }
    return hipErrorInvalidValue;
}

template <typename Tin, typename Tout>
hipError_t launch_m(hipStream_t st, int m, const Plan& pl, const void* U, int ldu, const double* R, int ldr,
                    void* Y, int ldy, const double* cell, int n) {
    switch (m) {
        case 0: return launch_ns<Tin, Tout, 0>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n);
        case 1: return launch_ns<Tin, Tout, 1>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n);
        case 2: return launch_ns<Tin, Tout, 2>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n);
        case 3: return launch_ns<Tin, Tout, 3>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n);
        case 4: return launch_ns<Tin, Tout, 4>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n);
        case 5: return launch_ns<Tin, Tout, 5>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n);
        case 6: return launch_ns<Tin, Tout, 6>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n);
        case 7: return launch_ns<Tin, Tout, 7>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n);
        case 8: return launch_ns<Tin, Tout, 8>(st, pl, U, ldu, R, ldr, Y, ldy, cell, n);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int launch_apply(sg_ctx* c, const Plan& pl, const void* U, int in_float, const double* R, void* Y, int out_float,
                 int ldu, int ldy, int ldr) {
    hipError_t e;
    const int m = c->hs.m, n = c->hs.n;
    if (!in_float && !out_float)
        e = launch_m<double, double>(c->stream, m, pl, U, ldu, R, ldr, Y, ldy, c->cell64, n);
    else if (in_float && !out_float)
        e = launch_m<float, double>(c->stream, m, pl, U, ldu, R, ldr, Y, ldy, c->cell64, n);
    else if (in_float && out_float)
        e = launch_m<float, float>(c->stream, m, pl, U, ldu, R, ldr, Y, ldy, c->cell64, n);
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
