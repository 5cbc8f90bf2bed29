// Krylov vector kernels, QoI reductions and the adjoint cell gradient.
//
// Reductions are deterministic: a fixed grid of kRedBlocks blocks walks the
// vector with a grid stride, each block reduces in a fixed tree (wavefront
// shuffles, then LDS across its 4 waves) and writes one partial per output;
// a second one-block kernel sums the partials in a fixed order.  No float
// atomics, so repeated runs are bitwise identical.

#include <mutex>
#include <type_traits>

#include "sg_internal.h"

#include "sg_vec.h"

namespace sg {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// block of 256 threads: returns the block sum in every thread of wave 0 lane 0
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    return t;
}

// Arnoldi orthogonalization by classical Gram-Schmidt with delayed
// reorthogonalization: the newest basis vector u is orthogonalized a second
// time in the same two passes that orthogonalize the next candidate w, so
// each step reads the basis twice (a pass of dot products, then a pass of
// updates) instead of three times plus a normalization.  Bases longer than
// kDc vectors are processed in chunks.
//
// Basis passes work on pairs of doubles (16-byte loads): the basis stride
// must be even (the launchers check it); an odd length leaves one last
// element, handled by one thread.

// partial[b][i] = sum_e Q_i[e] u[e], partial[b][kDc + i] = sum_e Q_i[e] w[e]
// (i < nv), partial[b][2 kDc] = u.u, partial[b][2 kDc + 1] = u.w, summed over
// block b's elements
template <int NV>
__global__ void __launch_bounds__(256) k_dots2(const double* __restrict__ Q, size_t stride, int nv,
                                               const double* __restrict__ u, const double* __restrict__ w,
                                               size_t len, double* __restrict__ partial) {
    __shared__ double sh[4];
    double aa[NV], bb[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) aa[i] = bb[i] = 0.0;
    double uu = 0.0, uw = 0.0;
    const size_t half = len / 2;
    const double2* u2 = (const double2*)u;
    const double2* w2 = (const double2*)w;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < half; e += (size_t)gridDim.x * blockDim.x) {
        const double2 ue = u2[e], we = w2[e];
        uu = fma(ue.x, ue.x, fma(ue.y, ue.y, uu));
        uw = fma(ue.x, we.x, fma(ue.y, we.y, uw));
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) {
                const double2 q = ((const double2*)(Q + (size_t)i * stride))[e];
                aa[i] = fma(q.x, ue.x, fma(q.y, ue.y, aa[i]));
                bb[i] = fma(q.x, we.x, fma(q.y, we.y, bb[i]));
            }
    }
    if ((len & 1) && blockIdx.x == 0 && threadIdx.x == 0) {  // odd length: last element
        const double ue = u[len - 1], we = w[len - 1];
        uu = fma(ue, ue, uu);
        uw = fma(ue, we, uw);
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) {
                const double q = Q[(size_t)i * stride + len - 1];
                aa[i] = fma(q, ue, aa[i]);
                bb[i] = fma(q, we, bb[i]);
            }
    }
    double* out = partial + (size_t)blockIdx.x * kDcLd;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i < nv) {  // uniform: keeps the loop unrolled and the sums in registers
            const double ta = block_sum(aa[i], sh);
            if (threadIdx.x == 0) out[i] = ta;
            const double tb = block_sum(bb[i], sh);
            if (threadIdx.x == 0) out[kDc + i] = tb;
        }
    }
    const double tu = block_sum(uu, sh);
    if (threadIdx.x == 0) out[2 * kDc] = tu;
    const double tw = block_sum(uw, sh);
    if (threadIdx.x == 0) out[2 * kDc + 1] = tw;
}

// Update pass over one chunk of the basis, elementwise:
//   uout = alpha uin - sum_i cf.a[i] Q_i,   wout = win - gamma uin - sum_i cf.c[i] Q_i
// and, when partial_sq is given, block partial sums of wout^2.  uout may be
// uin and wout may be win (each thread reads its elements before writing).
template <int NV>
__global__ void __launch_bounds__(256) k_update2(const double* __restrict__ Q, size_t stride, int nv, DcCoef cf,
                                                 const double* uin, const double* win, double* uout, double* wout,
                                                 size_t len, double* __restrict__ partial_sq) {
    __shared__ double sh[4];
    double sq = 0.0;
    const size_t half = len / 2;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < half; e += (size_t)gridDim.x * blockDim.x) {
        const double2 ue = ((const double2*)uin)[e];
        const double2 we = ((const double2*)win)[e];
        double2 qn, wn;
        qn.x = cf.alpha * ue.x;
        qn.y = cf.alpha * ue.y;
        wn.x = fma(-cf.gamma, ue.x, we.x);
        wn.y = fma(-cf.gamma, ue.y, we.y);
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) {
                const double2 q = ((const double2*)(Q + (size_t)i * stride))[e];
                qn.x = fma(-cf.a[i], q.x, qn.x);
                qn.y = fma(-cf.a[i], q.y, qn.y);
                wn.x = fma(-cf.c[i], q.x, wn.x);
                wn.y = fma(-cf.c[i], q.y, wn.y);
            }
        ((double2*)uout)[e] = qn;
        ((double2*)wout)[e] = wn;
        sq = fma(wn.x, wn.x, fma(wn.y, wn.y, sq));
    }
    if ((len & 1) && blockIdx.x == 0 && threadIdx.x == 0) {  // odd length: last element
        const double ue = uin[len - 1], we = win[len - 1];
        double qn = cf.alpha * ue, wn = fma(-cf.gamma, ue, we);
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < nv) {
                const double q = Q[(size_t)i * stride + len - 1];
                qn = fma(-cf.a[i], q, qn);
                wn = fma(-cf.c[i], q, wn);
            }
        uout[len - 1] = qn;
        wout[len - 1] = wn;
        sq = fma(wn, wn, sq);
    }
    if (partial_sq) {
        const double t = block_sum(sq, sh);
        if (threadIdx.x == 0) partial_sq[blockIdx.x] = t;
    }
}

// out[i] = sum_b partial[b][i] in a fixed order; workgroup i sums column i
// (launched with one workgroup per column)
__global__ void k_reduce_partials(const double* __restrict__ partial, int nblocks, int width, int ldp,
                                  double* __restrict__ out) {
    __shared__ double sh[4];
    const int i = blockIdx.x;
    if (i >= width) return;  // uniform over the workgroup
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v += partial[(size_t)b * ldp + i];
    const double t = block_sum(v, sh);
    if (threadIdx.x == 0) out[i] = t;
}

__global__ void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b, size_t len,
                              double* __restrict__ partial) {
    __shared__ double sh[4];
    double acc = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x)
        acc = fma(a[e], b[e], acc);
    const double t = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void k_scale(const double* __restrict__ src, double a, double* __restrict__ dst, size_t len) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x)
        dst[e] = a * src[e];
}

// x = (acc ? x : 0) + sum_i y[i] Z_i  (Z float or double; x is not read
// when acc is false).  A thread owns pairs of
// consecutive entries and reads the Z_i four vectors at a time, all loads of a
// group issued before its multiply-adds; the sum runs over i in order, as a
// plain loop would.
template <typename TZ>
__global__ void __launch_bounds__(256) k_combine(const TZ* __restrict__ Z, size_t stride, int nz,
                                                 const double* __restrict__ y, double* __restrict__ x, size_t len,
                                                 bool acc) {
    using TZ2 = typename std::conditional<sizeof(TZ) == 4, float2, double2>::type;
    __shared__ double ys[kMaxRestart];
    SG_POISON_LDS(ys, kMaxRestart);
    for (int i = threadIdx.x; i < nz; i += blockDim.x) ys[i] = y[i];
    __syncthreads();
    const size_t npair = len / 2;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < npair; e += (size_t)gridDim.x * blockDim.x) {
        double a0 = 0.0, a1 = 0.0;
        if (acc) {
            const double2 x0 = ((const double2*)x)[e];
            a0 = x0.x;
            a1 = x0.y;
        }
        int i = 0;
        for (; i + 4 <= nz; i += 4) {
            TZ2 v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = ((const TZ2*)(Z + (size_t)(i + q) * stride))[e];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a0 = fma(ys[i + q], (double)v[q].x, a0);
                a1 = fma(ys[i + q], (double)v[q].y, a1);
            }
        }
        for (; i < nz; ++i) {
            const TZ2 v = ((const TZ2*)(Z + (size_t)i * stride))[e];
            a0 = fma(ys[i], (double)v.x, a0);
            a1 = fma(ys[i], (double)v.y, a1);
        }
        ((double2*)x)[e] = make_double2(a0, a1);
    }
    if (len & 1) {  // the last entry of an odd length
        const size_t e = len - 1;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            double t = acc ? x[e] : 0.0;
            for (int i = 0; i < nz; ++i) t = fma(ys[i], (double)Z[(size_t)i * stride + e], t);
            x[e] = t;
        }
    }
}

// the same sum one entry per thread, for an x that is not 16-byte aligned
template <typename TZ>
__global__ void __launch_bounds__(256) k_combine_scalar(const TZ* __restrict__ Z, size_t stride, int nz,
                                                        const double* __restrict__ y, double* __restrict__ x,
                                                        size_t len, bool acc) {
    __shared__ double ys[kMaxRestart];
    SG_POISON_LDS(ys, kMaxRestart);
    for (int i = threadIdx.x; i < nz; i += blockDim.x) ys[i] = y[i];
    __syncthreads();
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x) {
        double t = acc ? x[e] : 0.0;
        for (int i = 0; i < nz; ++i) t = fma(ys[i], (double)Z[(size_t)i * stride + e], t);
        x[e] = t;
    }
}

// y = a*x + y  and partial sums of y^2 (PCG residual update)
__global__ void k_axpy_sq(double a, const double* __restrict__ x, double* __restrict__ y, size_t len,
                          double* __restrict__ partial_sq) {
    __shared__ double sh[4];
    double sq = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x) {
        const double v = fma(a, x[e], y[e]);
        y[e] = v;
        sq = fma(v, v, sq);
    }
    const double t = block_sum(sq, sh);
    if (threadIdx.x == 0) partial_sq[blockIdx.x] = t;
}

__global__ void k_axpy(double a, const double* __restrict__ x, double* __restrict__ y, size_t len) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x)
        y[e] = fma(a, x[e], y[e]);
}

// p = z + b p
__global__ void k_xpby(const double* __restrict__ z, double b, double* __restrict__ p, size_t len) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x)
        p[e] = fma(b, p[e], z[e]);
}

// F = e_0 (x) f_h with f_h,i = h^2 (f = 1)
__global__ void k_rhs(double* __restrict__ F, int N, int P, double h2) {
    const size_t len = (size_t)N * P;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x)
        F[e] = (e % P) == 0 ? h2 : 0.0;
}

// q partials: partial[b][a] = sum over node rows of block b of w_S[i] U[i][a]
__global__ void k_qoi_partial(const double* __restrict__ U, const double* __restrict__ wS, int N, int P,
                              double* __restrict__ partial, int ldp) {
    // threads cover modes (strided by blockDim.x); each block walks its node range
    const int per = (N + gridDim.x - 1) / gridDim.x;
    const int i0 = blockIdx.x * per, i1 = min(N, i0 + per);
    for (int a = threadIdx.x; a < P; a += blockDim.x) {
        double acc = 0.0;
        for (int i = i0; i < i1; ++i) acc = fma(wS[i], U[(size_t)i * P + a], acc);
        partial[(size_t)blockIdx.x * ldp + a] = acc;
    }
}

// J = q_0 + sum_{a>0} q_a^2 and the adjoint weights coef_a = (a == 0 ? 1 : 2 q_a)
__global__ void k_qoi_finish(const double* __restrict__ q, int P, double* __restrict__ J, double* __restrict__ coef) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int a = 1; a < P; ++a) s = fma(q[a], q[a], s);
        *J = q[0] + s;
    }
    for (int a = threadIdx.x; a < P; a += blockDim.x) coef[a] = a == 0 ? 1.0 : 2.0 * q[a];
}

__global__ void k_adj_rhs(const double* __restrict__ wS, const double* __restrict__ coef, int N, int P,
                          double* __restrict__ g) {
    const size_t len = (size_t)N * P;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (size_t)gridDim.x * blockDim.x) {
        const size_t i = e / P;
        g[e] = wS[i] * coef[e - i * P];
    }
}

// dc[e][k] = -sum_{a,b} G_k(a,b) lam_{a,e}^T K_ref U_{b,e}.  One wave per cell,
// lanes over modes; the element action t = K_ref U_b (times 6) is shared with
// the coupling partners through LDS.  toff/tcoef: the full coupling plan
// (packed LDS slots k*lanes + b of alpha +- e_k, coefficients G_k).
template <int NS>
__global__ void __launch_bounds__(256) k_grad_cells(const double* __restrict__ U, const double* __restrict__ L,
                                                    int n, int P, int m, const uint32_t* __restrict__ toff,
                                                    const double* __restrict__ tcoef, double* __restrict__ dc) {
    constexpr int LANES = NS * 64;
    extern __shared__ double lds_raw[];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double* T = lds_raw + wv * (4 * LANES + 2);
    SG_POISON_LDS(lds_raw, 4 * (4 * LANES + 2));
    const int cellid = blockIdx.x * 4 + wv;
    if (cellid >= n * n) return;
    const int cy = cellid / n, cx = cellid - cy * n;
    const int nx = n - 1;
    // vertices CCW from the lower-left: grid (cx,cy), (cx+1,cy), (cx+1,cy+1), (cx,cy+1)
    const int vx[4] = {cx, cx + 1, cx + 1, cx};
    const int vy[4] = {cy, cy, cy + 1, cy + 1};
    double u[NS][4], l[NS][4], t[NS][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const bool inside = vx[v] >= 1 && vx[v] <= nx && vy[v] >= 1 && vy[v] <= nx;
        const size_t node = inside ? (size_t)(vy[v] - 1) * nx + (vx[v] - 1) : 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int a = s * 64 + lane;
            const bool ok = inside && a < P;
            u[s][v] = ok ? U[node * P + a] : 0.0;
            l[s][v] = ok ? L[node * P + a] : 0.0;
        }
    }
    double acc[kMaxM + 1];
#pragma unroll
    for (int k = 0; k <= kMaxM; ++k) acc[k] = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        // 6 K_ref u: 4 u_v - u_(v+1) - u_(v+3) - 2 u_(v+2)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            t[s][v] = 4.0 * u[s][v] - u[s][(v + 1) & 3] - u[s][(v + 3) & 3] - 2.0 * u[s][(v + 2) & 3];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            acc[0] = fma(l[s][v], t[s][v], acc[0]);
            T[v * LANES + s * 64 + lane] = t[s][v];
        }
    }
    if (lane == 0) T[4 * LANES] = 0.0;
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __asm__ __volatile__("" ::: "memory");
    // coupling tables of the full plan: entry 2k / 2k+1 of lane a is the LDS
    // element k*lanes + b of the partner b = a + e_k / a - e_k (or the zero
    // entry), with coefficient G_k(a, b)
    const uint32_t zero = (uint32_t)(m * LANES);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int a = s * 64 + lane;
        if (a >= P) continue;
        for (int i = 0; i < 2 * m; ++i) {
            const uint32_t w = toff[(size_t)a * m + i / 2];
            const uint32_t idx = (i & 1) ? (w >> 16) : (w & 0xFFFFu);
            if (idx == zero) continue;
            const int k = (int)idx / LANES, b = (int)idx - k * LANES;
            const double g = tcoef[(size_t)a * 2 * m + i];
            double dotv = 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) dotv = fma(l[s][v], T[v * LANES + b], dotv);
#pragma unroll
            for (int kk = 1; kk <= kMaxM; ++kk)
                if (kk == k + 1) acc[kk] = fma(g, dotv, acc[kk]);
        }
    }
#pragma unroll
    for (int k = 0; k <= kMaxM; ++k) {
        if (k <= m) {
            const double s = wave_sum(acc[k]);
            if (lane == 0) dc[(size_t)cellid * (m + 1) + k] = -s / 6.0;
        }
    }
}

// partial[b][k] = sum over cells of block b of dc[e][k+1] * b_k(e), k < m
__global__ void k_grad_kl_partial(const double* __restrict__ dc, const double* __restrict__ kl, int ncell, int m,
                                  double* __restrict__ partial) {
    __shared__ double sh[4];
    for (int k = 0; k < m; ++k) {
        double acc = 0.0;
        for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < ncell; e += gridDim.x * blockDim.x)
            acc = fma(dc[(size_t)e * (m + 1) + k + 1], kl[(size_t)e * m + k], acc);
        const double t = block_sum(acc, sh);
        if (threadIdx.x == 0) partial[(size_t)blockIdx.x * 16 + k] = t;
    }
}

// out[0] = dJ/dsigma = sum_k s_k T_k, out[1+k] = dJ/ds_k = sigma T_k
__global__ void k_grad_kl_finish(const double* __restrict__ Tk, const double* __restrict__ amps, double sigma, int m,
                                 double* __restrict__ out) {
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) s = fma(amps[k], Tk[k], s);
        out[0] = s;
        for (int k = 0; k < m; ++k) out[1 + k] = sigma * Tk[k];
    }
}

// dJ/da0 at interior node (x, y): a quarter of dJ/dc_0 of its four cells
__global__ void k_grad_a0(const double* __restrict__ dc, int n, int m, double* __restrict__ out) {
    const int nx = n - 1;
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= nx * nx) return;
    const int y = node / nx, x = node - y * nx;
    const int s = m + 1;
    const double v = dc[((size_t)y * n + x) * s] + dc[((size_t)y * n + x + 1) * s] +
                     dc[((size_t)(y + 1) * n + x) * s] + dc[((size_t)(y + 1) * n + x + 1) * s];
    out[node] = 0.25 * v;
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t vec_dots2(hipStream_t s, const double* Q, size_t stride, int nv, const double* u, const double* w,
                     size_t len, double* partial, double* out) {
    if (stride & 1) return hipErrorInvalidValue;  // pairs of doubles need an even basis stride
    const int nch = nv == 0 ? 1 : (nv + kDc - 1) / kDc;
    for (int ch = 0; ch < nch; ++ch) {
        const int c0 = ch * kDc, cn = std::min(kDc, nv - c0);
        const double* Qc = Q + (size_t)c0 * stride;
        if (cn <= 8)
            hipLaunchKernelGGL(k_dots2<8>, dim3(kRedBlocks), dim3(256), 0, s, Qc, stride, cn, u, w, len, partial);
        else
            hipLaunchKernelGGL(k_dots2<kDc>, dim3(kRedBlocks), dim3(256), 0, s, Qc, stride, cn, u, w, len, partial);
        hipLaunchKernelGGL(k_reduce_partials, dim3(kDcLd), dim3(256), 0, s, partial, kRedBlocks, kDcLd, kDcLd,
                           out + (size_t)ch * kDcLd);
    }
    return hipGetLastError();
}
hipError_t vec_update2(hipStream_t s, const double* Q, size_t stride, int nv, const double* a, const double* c,
                       double alpha, double gamma, const double* uin, double* u, const double* w, double* wout,
                       size_t len, double* partial_sq, double* out_sq) {
    if (stride & 1) return hipErrorInvalidValue;
    const int nch = nv == 0 ? 1 : (nv + kDc - 1) / kDc;
    for (int ch = 0; ch < nch; ++ch) {
        const int c0 = ch * kDc, cn = std::min(kDc, nv - c0);
        DcCoef cf{};
        for (int i = 0; i < cn; ++i) {
            cf.a[i] = a[c0 + i];
            cf.c[i] = c[c0 + i];
        }
        // the first chunk scales uin and takes gamma uin from w; later chunks continue from the outputs
        cf.alpha = ch == 0 ? alpha : 1.0;
        cf.gamma = ch == 0 ? gamma : 0.0;
        const double* win = ch == 0 ? w : wout;
        const double* ui = ch == 0 ? uin : u;
        double* psq = ch == nch - 1 ? partial_sq : nullptr;
        const double* Qc = Q + (size_t)c0 * stride;
        if (cn <= 8)
            hipLaunchKernelGGL(k_update2<8>, dim3(kRedBlocks), dim3(256), 0, s, Qc, stride, cn, cf, ui, win, u, wout,
                               len, psq);
        else
            hipLaunchKernelGGL(k_update2<kDc>, dim3(kRedBlocks), dim3(256), 0, s, Qc, stride, cn, cf, ui, win, u,
                               wout, len, psq);
    }
    if (partial_sq && out_sq)
        hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partial_sq, kRedBlocks, 1, 1, out_sq);
    return hipGetLastError();
}
hipError_t vec_dot(hipStream_t s, const double* a, const double* b, size_t len, double* partial, double* out) {
    hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(256), 0, s, a, b, len, partial);
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partial, kRedBlocks, 1, 1, out);
    return hipGetLastError();
}

hipError_t vec_scale(hipStream_t s, const double* src, double a, double* dst, size_t len) {
    hipLaunchKernelGGL(k_scale, dim3(kRedBlocks), dim3(256), 0, s, src, a, dst, len);
    return hipGetLastError();
}

hipError_t vec_combine(hipStream_t s, const void* Z, int z_float, size_t stride, int nz, const double* y, double* x,
                       size_t len, bool accumulate) {
    // pairs of entries need x 16-byte aligned and Z_i starting on an even entry (an even stride)
    const bool pairs = ((uintptr_t)x % 16 == 0) && ((uintptr_t)Z % 16 == 0) && stride % 2 == 0;
    if (z_float) {
        if (pairs)
            hipLaunchKernelGGL(k_combine<float>, dim3(kRedBlocks), dim3(256), 0, s, (const float*)Z, stride, nz, y, x,
                               len, accumulate);
        else
            hipLaunchKernelGGL(k_combine_scalar<float>, dim3(kRedBlocks), dim3(256), 0, s, (const float*)Z, stride, nz,
                               y, x, len, accumulate);
    } else {
        if (pairs)
            hipLaunchKernelGGL(k_combine<double>, dim3(kRedBlocks), dim3(256), 0, s, (const double*)Z, stride, nz, y,
                               x, len, accumulate);
        else
            hipLaunchKernelGGL(k_combine_scalar<double>, dim3(kRedBlocks), dim3(256), 0, s, (const double*)Z, stride,
                               nz, y, x, len, accumulate);
    }
    return hipGetLastError();
}

hipError_t vec_axpy_sq(hipStream_t s, double a, const double* x, double* y, size_t len, double* partial,
                       double* out_sq) {
    hipLaunchKernelGGL(k_axpy_sq, dim3(kRedBlocks), dim3(256), 0, s, a, x, y, len, partial);
    hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, s, partial, kRedBlocks, 1, 1, out_sq);
    return hipGetLastError();
}

hipError_t vec_axpy(hipStream_t s, double a, const double* x, double* y, size_t len) {
    hipLaunchKernelGGL(k_axpy, dim3(kRedBlocks), dim3(256), 0, s, a, x, y, len);
    return hipGetLastError();
}

hipError_t vec_xpby(hipStream_t s, const double* z, double b, double* p, size_t len) {
    hipLaunchKernelGGL(k_xpby, dim3(kRedBlocks), dim3(256), 0, s, z, b, p, len);
    return hipGetLastError();
}

hipError_t vec_rhs(hipStream_t s, double* F, int N, int P, double h2) {
    hipLaunchKernelGGL(k_rhs, dim3(kRedBlocks), dim3(256), 0, s, F, N, P, h2);
    return hipGetLastError();
}

hipError_t vec_qoi(hipStream_t s, const double* U, const double* wS, int N, int P, double* partial, double* q,
                   double* J, double* coef) {
    hipLaunchKernelGGL(k_qoi_partial, dim3(kRedBlocks), dim3(256), 0, s, U, wS, N, P, partial, P);
    hipLaunchKernelGGL(k_reduce_partials, dim3(P), dim3(256), 0, s, partial, kRedBlocks, P, P, q);
    hipLaunchKernelGGL(k_qoi_finish, dim3(1), dim3(256), 0, s, q, P, J, coef);
    return hipGetLastError();
}

hipError_t vec_adj_rhs(hipStream_t s, const double* wS, const double* coef, int N, int P, double* g) {
    hipLaunchKernelGGL(k_adj_rhs, dim3(kRedBlocks), dim3(256), 0, s, wS, coef, N, P, g);
    return hipGetLastError();
}

hipError_t vec_grad_cells(hipStream_t s, int nslot, const double* U, const double* L, int n, int P, int m,
                          const uint32_t* toff, const double* tcoef, double* dc) {
    const int blocks = (n * n + 3) / 4;
    const size_t shm = (size_t)4 * (4 * nslot * 64 + 2) * sizeof(double);
    switch (nslot) {
        case 1: hipLaunchKernelGGL(k_grad_cells<1>, dim3(blocks), dim3(256), shm, s, U, L, n, P, m, toff, tcoef, dc); break;
        case 2: hipLaunchKernelGGL(k_grad_cells<2>, dim3(blocks), dim3(256), shm, s, U, L, n, P, m, toff, tcoef, dc); break;
        case 3: hipLaunchKernelGGL(k_grad_cells<3>, dim3(blocks), dim3(256), shm, s, U, L, n, P, m, toff, tcoef, dc); break;
        case 4: hipLaunchKernelGGL(k_grad_cells<4>, dim3(blocks), dim3(256), shm, s, U, L, n, P, m, toff, tcoef, dc); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t vec_grad_params(hipStream_t s, const double* dc, const double* kl, const double* amps, double sigma, int n,
                           int m, double* partial, double* Tk, double* out_params, double* out_a0) {
    if (m > 0) {
        hipLaunchKernelGGL(k_grad_kl_partial, dim3(kRedBlocks), dim3(256), 0, s, dc, kl, n * n, m, partial);
        hipLaunchKernelGGL(k_reduce_partials, dim3(m), dim3(256), 0, s, partial, kRedBlocks, m, 16, Tk);
    }
    hipLaunchKernelGGL(k_grad_kl_finish, dim3(1), dim3(64), 0, s, Tk, amps, sigma, m, out_params);
    const int nn = (n - 1) * (n - 1);
    hipLaunchKernelGGL(k_grad_a0, dim3((nn + 255) / 256), dim3(256), 0, s, dc, n, m, out_a0);
    return hipGetLastError();
}

// ------------------------------------------------------------ allocation-free QoI
// Scratch of sg_qoi_noalloc: the reduction partials (kRedBlocks rows of P
// modes), then the adjoint weights (P).  A file-scope device array: every GPU
// the library runs on holds one copy until the process ends.  In host code the
// array's name is only a stand-in, so its device address is looked up once per
// device (with that device current) and that pointer is what the kernels get.
static __device__ __align__(256) double scratch[kQoiScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t qoi_scratch_address(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = (double*)ptr;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace sg
