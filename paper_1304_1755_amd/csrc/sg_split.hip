// Kernels of the block-triangular preconditioner with the 2 x 2 split of
// Sec. 4.2, B_T = [[A_hat, 0], [W, D]]: A_hat (the modes of degree <= p-1)
// is inverted by one multigrid cycle for the coupled system, with point
// Gauss-Seidel on the assembled A_hat_l in its natural order (mode by mode,
// inside a mode node by node, x fastest).
//
// Modes of one total degree do not couple (G_k(alpha, beta) != 0 only for
// beta = alpha +- e_k), and the mode order is graded, so a Gauss-Seidel sweep
// in that order updates all modes of degree d together: each from the new
// values of degree d-1 and the old ones of degree d+1 (backward sweep: the
// reverse), by one lexicographic sweep of its diagonal block K_0 against the
// right-hand side f_alpha - sum_k sum_beta G_k(alpha, beta) K_k u_beta.  This
// file holds that coupling (also the residual of A_hat_l when the K_0 term is
// included) and the direct solve on the coarsest level; the lexicographic
// sweep and the transfers are those of the K_0 hierarchy.

#include "sg_internal.h"

namespace sg {

namespace {

// out[node, t] = f[node, lo+t] - self (K_0 u_{lo+t})(node)
//                - sum over the partners beta of alpha = lo+t of G_k(alpha, beta) (K_k u_beta)(node).
// One thread per (node, output mode), modes fastest.  The stencils of K_k on
// this level are block k of sten ((m+1) x N x 9); the partners of a mode are
// packed first in its row of pidx (beta | k << 16), -1 after the last.
__global__ void __launch_bounds__(256) k_split_couple(const double* __restrict__ sten, int N,
                                                      const int* __restrict__ pidx,
                                                      const double* __restrict__ pcoef, int npart,
                                                      const double* __restrict__ u, int ldu,
                                                      const double* __restrict__ f, int ldf,
                                                      double* __restrict__ out, int ldo, int nx, int lo, int width,
                                                      int self) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)N * width) return;
    const int node = (int)(idx / width), t = (int)(idx - (long)node * width), a = lo + t;
    const int y = node / nx, x = node - y * nx;
    // (K_k u_b)(node)
    auto stencil = [&](int k, int b) -> double {
        const double* s9 = sten + ((size_t)k * N + node) * 9;
        double v = 0.0;
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = y + dy;
            if (yy < 0 || yy >= nx) continue;
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int xx = x + dx;
                if (xx < 0 || xx >= nx) continue;
                v = fma(s9[(dy + 1) * 3 + (dx + 1)], u[(size_t)(yy * nx + xx) * ldu + b], v);
            }
        }
        return v;
    };
    double acc = f[(size_t)node * ldf + a];
    if (self) acc -= stencil(0, a);
    for (int q = 0; q < npart; ++q) {
        const int e = pidx[a * npart + q];
        if (e < 0) break;
        acc -= pcoef[a * npart + q] * stencil(e >> 16, e & 0xFFFF);
    }
    out[(size_t)node * ldo + t] = acc;
}

// u = A_hat_c^{-1} f on the coarsest level: one wavefront per row of the
// inverse (rows and columns indexed node * Pa + alpha), lanes over columns.
__global__ void __launch_bounds__(256) k_split_coarse(const double* __restrict__ cinv, int nA, int Pa,
                                                      const double* __restrict__ f, int ldf,
                                                      double* __restrict__ u, int ldu) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= nA) return;  // uniform per wavefront
    double acc = 0.0;
    for (int j = lane; j < nA; j += 64) {
        const int nd = j / Pa, b = j - nd * Pa;
        acc = fma(cinv[(size_t)row * nA + j], f[(size_t)nd * ldf + b], acc);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) {
        const int nd = row / Pa, a = row - nd * Pa;
        u[(size_t)nd * ldu + a] = acc;
    }
}

}  // namespace

int launch_split_couple(sg_ctx* c, int l, const double* u, int ldu, const double* f, int ldf, double* out, int ldo,
                        int lo, int width, int self) {
    const SplitDev& sp = c->split;
    const Level& lv = c->levels[l];
    const long total = (long)lv.N * width;
    if (total == 0) return SG_OK;
    hipLaunchKernelGGL(k_split_couple, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, c->stream, sp.sten[l],
                       lv.N, sp.pidx, sp.pcoef, sp.npart, u, ldu, f, ldf, out, ldo, lv.nx, lo, width, self);
    return hipGetLastError() == hipSuccess ? SG_OK : SG_EHIP;
}

int launch_split_coarse(sg_ctx* c, const double* f, int ldf, double* u, int ldu) {
    const SplitDev& sp = c->split;
    const int nA = c->levels.back().N * sp.Pa;
    hipLaunchKernelGGL(k_split_coarse, dim3((nA + 3) / 4), dim3(256), 0, c->stream, sp.cinv, nA, sp.Pa, f, ldf, u,
                       ldu);
    return hipGetLastError() == hipSuccess ? SG_OK : SG_EHIP;
}

}  // namespace sg
