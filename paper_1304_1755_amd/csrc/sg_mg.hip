// Batched geometric multigrid V-cycle for the mean stiffness K_0.
//
// The paper inverts every diagonal block K_0 of B_D and B_T by one V-cycle
// (Sec. 4.1, Sec. 4.2; Sec. 6 uses V(2,2) with point Gauss-Seidel).  All
// diagonal blocks are the same K_0, so the cycle runs on many right-hand
// sides at once: an N_l x W node-major block, with the W modes of a node
// contiguous.  Threads are laid out (modes x nodes) so a node's stencil
// (9 coefficients, Galerkin coarse operators from setup) is fetched once per
// node and broadcast to the lanes of its modes, and every access to the
// block is a contiguous run of W values.
//
// Components: multi-colour Gauss-Seidel (four colours (I mod 2, J mod 2), or
// red/black with each colour updated from its start-of-colour values) or
// lexicographic point Gauss-Seidel, x fastest (a reading of the point
// Gauss-Seidel that Sec. 6 names without an ordering; front by front, one
// workgroup per right-hand side; for grids of the paper's sizes),
// residual, restriction R = P^T, prolongation P, and the coarsest grid
// solved with the explicit inverse of its operator in double precision.  P is
// the bilinear interpolation for Q1 elements, or the linear interpolation of
// the triangulation of Sec. 6 (its diagonals run south-west to north-east)
// for P1 elements: the two agree on the grid lines, and a fine cell centre
// takes the mean of the coarse SW and NE corners instead of all four.
//
// Kernel forms by block width W (modes) and grid size:
//   * four-colour smoothing runs as row phases (one launch per row parity,
//     both colours of a row): for W >= 32 a workgroup walks a row segment
//     with lanes over modes (k_gs_rows; the first sweep from the zero start
//     takes both phases in one launch, k_gs_sweep0); narrower blocks give each
//     lane one (row, S node, mode) triple (k_gs_rows_narrow);
//   * for W >= 16 residual + restriction is one walking pass
//     (k_resid_restrict) and the prolongation another (k_prolong_rows);
//     narrower blocks use one node per thread (k_residual, k_restrict,
//     k_prolong_add);
//   * walking kernels use short segments on coarse grids, where long walks
//     would leave too few wavefronts;
//   * grids of at most 63 x 63 (float) or 31 x 31 (double) interior nodes are
//     cycled by one launch that keeps them in LDS (k_vcycle_pad for grids of
//     2^k - 1 nodes per side, k_vcycle_fused4 for other four-colour
//     hierarchies, k_vcycle_fused for red/black and lexicographic);
//   * the finest level iterates in its own compact block; only the last
//     post-smoothing sweep writes the caller's (possibly strided) output.

#include "sg_internal.h"

namespace sg {

namespace {

struct Tile {
    int tx, ty;
};

Tile tile_for(int width) {
    int tx = 1;
    while (tx < width && tx < 64) tx <<= 1;
    return {tx, 256 / tx};
}

// Blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
// Mapping block b to a contiguous range of node chunks per XCD keeps a
// node's stencil neighbours (the rows above and below) in the same L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int x = b & 7, i = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + i;
}

// Weight of a coarse node in the interpolated value at a fine node offset by
// (dx, dy) from the coarse node's own fine position (|dx|, |dy| <= 1).
template <typename T>
__device__ __forceinline__ T transfer_w(int dx, int dy, bool p1) {
    if (dx != 0 && dy != 0) return p1 ? (dx == dy ? T(0.5) : T(0)) : T(0.25);
    return (dx == 0 ? T(1) : T(0.5)) * (dy == 0 ? T(1) : T(0.5));
}

// (P^T r) at coarse node (X, Y): get(x, y) reads the fine residual at fine node (x, y)
template <typename T, typename G>
__device__ __forceinline__ T restrict_value(G get, int X, int Y, bool p1) {
    const int fx = 2 * X + 1, fy = 2 * Y + 1;
    T acc = T(0);
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const T w = transfer_w<T>(dx, dy, p1);
            if (w != T(0)) acc += w * get(fx + dx, fy + dy);
        }
    return acc;
}

// (P e)(x, y) at fine node (x, y): get(X, Y) reads the coarse correction at
// coarse node (X, Y), nxc coarse nodes per side (zero outside)
template <typename T, typename G>
__device__ __forceinline__ T prolong_value(G get, int nxc, int x, int y, bool p1) {
    if (p1 && !(x & 1) && !(y & 1)) {
        // a fine cell centre: on the diagonal from the coarse SW to NE corner
        const int cx0 = (x >> 1) - 1, cy0 = (y >> 1) - 1, cx1 = x >> 1, cy1 = y >> 1;
        T a = T(0);
        if (cx0 >= 0 && cy0 >= 0) a += get(cx0, cy0);
        if (cx1 < nxc && cy1 < nxc) a += get(cx1, cy1);
        return T(0.5) * a;
    }
    // fine x odd: on coarse column (x-1)/2; x even: between x/2-1 and x/2
    int cx0, cx1, cy0, cy1;
    T wx, wy;
    if (x & 1) { cx0 = cx1 = (x - 1) >> 1; wx = T(1); } else { cx0 = (x >> 1) - 1; cx1 = x >> 1; wx = T(0.5); }
    if (y & 1) { cy0 = cy1 = (y - 1) >> 1; wy = T(1); } else { cy0 = (y >> 1) - 1; cy1 = y >> 1; wy = T(0.5); }
    T acc = T(0);
    const int ncx = (cx0 == cx1) ? 1 : 2, ncy = (cy0 == cy1) ? 1 : 2;
    for (int b = 0; b < ncy; ++b) {
        const int cy = b ? cy1 : cy0;
        if (cy < 0 || cy >= nxc) continue;
        for (int a = 0; a < ncx; ++a) {
            const int cx = a ? cx1 : cx0;
            if (cx < 0 || cx >= nxc) continue;
            acc += get(cx, cy);
        }
    }
    return wx * wy * acc;
}

template <typename T>
__global__ void k_fill(T* __restrict__ dst, int ld, int rows, int width) {
    const int mode = blockIdx.y * blockDim.x + threadIdx.x;
    const int row = blockIdx.x * blockDim.y + threadIdx.y;
    if (mode < width && row < rows) dst[(size_t)row * ld + mode] = T(0);
}

template <typename T>
__global__ void k_axpy_cols(const T* __restrict__ src, int lds, T* __restrict__ dst, int ldd, int rows, int width,
                            T a) {
    const int mode = blockIdx.y * blockDim.x + threadIdx.x;
    const int row = blockIdx.x * blockDim.y + threadIdx.y;
    if (mode < width && row < rows) dst[(size_t)row * ldd + mode] += a * src[(size_t)row * lds + mode];
}

template <typename Ts, typename Td>
__global__ void k_cast(const Ts* __restrict__ src, int lds, Td* __restrict__ dst, int ldd, int rows, int width) {
    const int mode = blockIdx.y * blockDim.x + threadIdx.x;
    const int row = blockIdx.x * blockDim.y + threadIdx.y;
    if (mode < width && row < rows) dst[(size_t)row * ldd + mode] = (Td)src[(size_t)row * lds + mode];
}

// Gauss-Seidel update of the nodes of one colour.  Colour lattice: nodes
// (x0 + sx*i, y) with row-dependent start for red/black.
//   four colours: px, py fixed parities, x = px + 2i, y = py + 2j
//   red/black   : (x + y) & 1 == q, x = ((q + y) & 1) + 2i
// snap == nullptr: in-place update (four colours never touch each other).
// snap != nullptr: red/black first pass, new values are written to `snap`
// (a staging buffer) and copied back by k_copy_colour.
// first != 0: the first sweep after a zero initial guess.  Every node of a
// colour that has not been updated yet in this sweep still holds zero, so
// those neighbours are skipped and u needs no clearing beforehand.  (For
// red/black the same-colour diagonal neighbours are also still zero.)
template <typename T, bool WAVE_NODE>
__global__ void k_gs(const T* __restrict__ sten, const T* __restrict__ rdiag, T* __restrict__ u, int ldu,
                     const T* __restrict__ f, int ldf, T* __restrict__ out, int ldo, int nx, int width, int rb, int q,
                     int nxc, int nyc, int first) {
    const int mode = blockIdx.y * blockDim.x + threadIdx.x;
    int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.y + threadIdx.y;
    if (WAVE_NODE) t = __builtin_amdgcn_readfirstlane(t);  // one node per wavefront: scalar stencil loads
    if (mode >= width || t >= nxc * nyc) return;
    const int j = t / nxc, i = t - j * nxc;
    int x, y;
    if (rb) {
        y = j;
        x = ((q + y) & 1) + 2 * i;
        if (x >= nx) return;
    } else {
        x = (((q & 1) ^ 1)) + 2 * i;
        y = (((q >> 1) ^ 1)) + 2 * j;
    }
    const size_t node = (size_t)y * nx + x;
    const T* st = sten + node * 9;
    T acc = f[node * ldf + mode];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        const int yy = y + dy;
        if (yy < 0 || yy >= nx) continue;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const int xx = x + dx;
            if (xx < 0 || xx >= nx) continue;
            if (first) {
                // colour of the neighbour from its grid indices (xx+1, yy+1)
                const int qn = rb ? ((xx + yy) & 1) : (((xx + 1) & 1) + 2 * ((yy + 1) & 1));
                if (qn >= q) continue;
            }
            acc -= st[(dy + 1) * 3 + (dx + 1)] * u[((size_t)yy * nx + xx) * ldu + mode];
        }
    }
    const T val = acc * rdiag[node];
    if (out)
        out[node * ldo + mode] = val;
    else
        u[node * ldu + mode] = val;
}

template <typename T>
__global__ void k_copy_colour(const T* __restrict__ src, int lds, T* __restrict__ u, int ldu, int nx, int width,
                              int q, int nxc, int nyc) {
    const int mode = blockIdx.y * blockDim.x + threadIdx.x;
    const int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.y + threadIdx.y;
    if (mode >= width || t >= nxc * nyc) return;
    const int y = t / nxc, i = t - y * nxc;
    const int x = ((q + y) & 1) + 2 * i;
    if (x >= nx) return;
    const size_t node = (size_t)y * nx + x;
    u[node * ldu + mode] = src[node * lds + mode];
}

template <typename T, bool WAVE_NODE>
__global__ void k_residual(const T* __restrict__ sten, const T* __restrict__ u, int ldu, const T* __restrict__ f,
                           int ldf, T* __restrict__ r, int ldr, int nx, int width) {
    const int mode = blockIdx.y * blockDim.x + threadIdx.x;
    int node = xcd_block(blockIdx.x, gridDim.x) * blockDim.y + threadIdx.y;
    if (WAVE_NODE) node = __builtin_amdgcn_readfirstlane(node);  // one node per wavefront
    if (mode >= width || node >= nx * nx) return;
    const int y = node / nx, x = node - y * nx;
    const T* st = sten + (size_t)node * 9;
    T acc = f[(size_t)node * ldf + mode];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        const int yy = y + dy;
        if (yy < 0 || yy >= nx) continue;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int xx = x + dx;
            if (xx < 0 || xx >= nx) continue;
            acc -= st[(dy + 1) * 3 + (dx + 1)] * u[((size_t)yy * nx + xx) * ldu + mode];
        }
    }
    r[(size_t)node * ldr + mode] = acc;
}

// coarse node (X, Y) sits on fine node (2X+1, 2Y+1)
template <typename T>
__global__ void k_restrict(const T* __restrict__ r, int ldr, T* __restrict__ fc, int ldc, int nxc, int width,
                           int p1) {
    const int mode = blockIdx.y * blockDim.x + threadIdx.x;
    const int node = xcd_block(blockIdx.x, gridDim.x) * blockDim.y + threadIdx.y;
    if (mode >= width || node >= nxc * nxc) return;
    const int Y = node / nxc, X = node - Y * nxc;
    const int nxf = 2 * nxc + 1;
    auto get = [&](int x, int y) { return r[((size_t)y * nxf + x) * ldr + mode]; };
    fc[(size_t)node * ldc + mode] = restrict_value<T>(get, X, Y, p1 != 0);
}

// Residual and restriction in one pass for wide blocks (W >= 16 modes):
// fc = R (f - K u) without storing the fine residual.  A workgroup walks a
// segment of kRrSeg nodes of one coarse row Y; lanes are modes.  Per coarse
// column X it forms the fine residual of the three rows fy-1, fy, fy+1
// (fy = 2Y+1) at columns x = 2X+1 and 2X+2, from a window of five fine rows
// of u.  Bilinear transfer: with c(x) = r(x, fy-1)/2 + r(x, fy) + r(x, fy+1)/2,
// fc(X) = c(2X)/2 + c(2X+1) + c(2X+2)/2.  P1 transfer (P1T): the centre
// column weighs the rows as c does, the west column takes (r(fy-1) + r(fy))/2
// and the east column (r(fy) + r(fy+1))/2.
// Loads are clamped into the grid (zero outside) and issued a ring of steps
// ahead; the stencils of the three fine rows are staged in LDS.
constexpr int kRrSeg = 16;       // coarse nodes per segment on the fine levels
constexpr int kRrSegShort = 4;   // on coarse levels, where long walks leave too few workgroups
// narrowest block the walking transfer kernels take (narrower: one node per thread)
constexpr int kWalkMinWidth = 16;

template <typename T, int SEG, bool P1T>
__global__ void __launch_bounds__(256) k_resid_restrict(const T* __restrict__ sten, const T* __restrict__ u, int ldu,
                                                        const T* __restrict__ f, int ldf, T* __restrict__ fc,
                                                        int ldc, int nxc, int width, int nseg) {
    constexpr int D = 2;
    constexpr int NC = 2 * SEG + 1;                 // staged fine columns 2 X0 .. 2 X0 + 2 SEG
    constexpr int SP = sizeof(T) == 4 ? 12 : 10;
    __shared__ T stl[3 * NC * SP];
    const int lane = threadIdx.x & 63;
    const int s_w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = s_w * 64 + lane;
    const bool ok = t < width;
    const int tc = ok ? t : width - 1;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    if (lb >= nxc * nseg) return;  // uniform over the workgroup
    SG_POISON_LDS(stl, sizeof(stl) / sizeof(T));
    const int Y = lb / nseg;
    const int X0 = (lb - Y * nseg) * SEG;
    const int X1 = min(X0 + SEG, nxc);
    const int nxf = 2 * nxc + 1;
    const int fy = 2 * Y + 1;
    const int xb = 2 * X0;  // first fine column of the walk
    for (int i = threadIdx.x; i < 3 * NC * 9; i += blockDim.x) {
        const int rk = i / (NC * 9), rem = i - rk * (NC * 9);
        const int c = rem / 9, e = rem - c * 9;
        const int x = min(xb + c, nxf - 1);
        stl[(rk * NC + c) * SP + e] = sten[((size_t)(fy - 1 + rk) * nxf + x) * 9 + e];
    }
    __syncthreads();
    // fine rows fy-2 .. fy+2 of u (k = 0..4): only the outer two can leave the grid
    const bool rv0 = fy - 2 >= 0, rv4 = fy + 2 < nxf;
    auto cx = [&](int x) { return min(max(x, 0), nxf - 1); };
    auto inx = [&](int x) { return x >= 0 && x < nxf; };
    // row bases computed once (fine rows fy-2 .. fy+2 of u clamped into the grid, rows fy-1 .. fy+1 of f)
    const T* urow[5];
    const T* frow[3];
#pragma unroll
    for (int k = 0; k < 5; ++k) urow[k] = u + (size_t)min(max(fy - 2 + k, 0), nxf - 1) * nxf * ldu;
#pragma unroll
    for (int k = 0; k < 3; ++k) frow[k] = f + (size_t)(fy - 1 + k) * nxf * ldf;
    T* const fcrow = fc + (size_t)Y * nxc * ldc;
    auto gu = [&](int k, int x) -> T { return (urow[k] + cx(x) * ldu)[tc]; };
    auto gf = [&](int k, int x) -> T { return (frow[k] + x * ldf)[tc]; };
    auto zu = [&](T v, int k, int x) -> T {
        const bool rv = k == 0 ? rv0 : (k == 4 ? rv4 : true);
        return (rv && inx(x)) ? v : T(0);
    };
    // residuals r3[k] at (x, fy-1+k) from u columns x-1, x, x+1 (U[k][0..2]) and f at rows fy-1..fy+1
    auto colres = [&](int x, const T (*U)[3], const T* fv, T* r3) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T* st = stl + (k * NC + (x - xb)) * SP;
            T acc = fv[k];
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) acc -= st[dy * 3 + dx] * U[k + dy][dx];
            r3[k] = acc;
        }
    };
    auto mid = [](const T* r3) -> T { return T(0.5) * r3[0] + r3[1] + T(0.5) * r3[2]; };
    // the column's share as the west / east neighbour column of a coarse node
    auto west = [&](const T* r3) -> T { return P1T ? T(0.5) * (r3[0] + r3[1]) : T(0.5) * mid(r3); };
    auto east = [&](const T* r3) -> T { return P1T ? T(0.5) * (r3[1] + r3[2]) : T(0.5) * mid(r3); };
    // ring slots: step i (X = X0 + i) loads u columns 2X+2, 2X+3 and f columns 2X+1, 2X+2
    T qu2[D][5], qu3[D][5], qf1[D][3], qf2[D][3];
    auto issue = [&](int i, int s) {
        const int x = 2 * (X0 + i);
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            qu2[s][k] = gu(k, x + 2);
            qu3[s][k] = gu(k, x + 3);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            qf1[s][k] = gf(k, min(x + 1, nxf - 1));
            qf2[s][k] = gf(k, min(x + 2, nxf - 1));
        }
    };
    // prologue: u columns xb-1, xb, xb+1 and f at xb give c(xb)
    T W[5][3], f0[3];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        W[k][0] = gu(k, xb - 1);
        W[k][1] = gu(k, xb);
        W[k][2] = gu(k, xb + 1);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) f0[k] = gf(k, xb);
#pragma unroll
    for (int s = 0; s < D; ++s) issue(s, s);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        W[k][0] = zu(W[k][0], k, xb - 1);
        W[k][1] = zu(W[k][1], k, xb);
        W[k][2] = zu(W[k][2], k, xb + 1);
    }
    T cprev;  // west share of column 2X
    {
        T r3[3];
        colres(xb, W, f0, r3);
        cprev = west(r3);
    }
#pragma unroll
    for (int i = 0; i < SEG; ++i) {
        const int s = i % D;
        const int X = X0 + i;
        const int x = 2 * X;
        // window for column x+1: u columns x, x+1, x+2
        T A[5][3], Bw[5][3], fa[3], fb[3];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const T u2 = zu(qu2[s][k], k, x + 2), u3 = zu(qu3[s][k], k, x + 3);
            A[k][0] = W[k][1];
            A[k][1] = W[k][2];
            A[k][2] = u2;
            Bw[k][0] = W[k][2];
            Bw[k][1] = u2;
            Bw[k][2] = u3;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            fa[k] = qf1[s][k];
            fb[k] = qf2[s][k];
        }
        if (i + D < SEG) issue(i + D, s);
        if (X < X1) {
            T r1[3], r2[3];
            colres(x + 1, A, fa, r1);
            colres(x + 2, Bw, fb, r2);
            if (ok) (fcrow + X * ldc)[t] = cprev + mid(r1) + east(r2);
            cprev = west(r2);
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            W[k][1] = Bw[k][1];
            W[k][2] = Bw[k][2];
        }
    }
}

// Prolongation added to u for wide blocks (W >= 16 modes): a workgroup
// walks kPrSeg nodes of one fine row; lanes are modes.  The fine row takes
// the coarse row it lies on (odd y) or the mean of the two it lies between
// (even y); along the row, odd x takes the coarse value it lies on and even
// x the mean of its two neighbours.  With the P1 transfer (P1T) a node with
// even x and even y (a fine cell centre) takes the mean of the coarse SW and
// NE corners instead.  Loads are clamped (zero outside the coarse grid) and
// issued a ring of steps ahead.
constexpr int kPrSeg = 32;       // fine nodes per segment on the fine levels
constexpr int kPrSegShort = 8;   // on coarse levels

template <typename T, int SEG, bool P1T>
__global__ void __launch_bounds__(256) k_prolong_rows(const T* __restrict__ ec, int ldc, T* __restrict__ u, int ldu,
                                                      int nxf, int width, int nseg) {
    constexpr int D = 4;
    constexpr int NIT = SEG / 2;
    const int lane = threadIdx.x & 63;
    const int s_w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = s_w * 64 + lane;
    const bool ok = t < width;
    const int tc = ok ? t : width - 1;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    if (lb >= nxf * nseg) return;
    const int y = lb / nseg;
    const int x0 = (lb - y * nseg) * SEG;  // even
    const int x1 = min(x0 + SEG, nxf);
    const int nxc = (nxf - 1) / 2;
    int ya, yb;
    T wy;
    if (y & 1) { ya = yb = (y - 1) >> 1; wy = T(1); }
    else { ya = (y >> 1) - 1; yb = y >> 1; wy = T(0.5); }
    const bool va_ok = ya >= 0, vb_ok = (y & 1) ? false : yb < nxc;
    const int yac = max(ya, 0), ybc = min(yb, nxc - 1);
    auto cX = [&](int X) { return min(max(X, 0), nxc - 1); };
    const T* const earow = ec + (size_t)yac * nxc * ldc;
    const T* const ebrow = ec + (size_t)ybc * nxc * ldc;
    T* const urow = u + (size_t)y * nxf * ldu;
    auto gca = [&](int X) -> T { return (earow + cX(X) * ldc)[tc]; };
    auto gcb = [&](int X) -> T { return (ebrow + cX(X) * ldc)[tc]; };
    // the coarse values below (a) and above (b) the fine row, zero outside
    auto am = [&](T a, int X) -> T { return (X < 0 || X >= nxc || !va_ok) ? T(0) : a; };
    auto bm = [&](T b, int X) -> T { return (X < 0 || X >= nxc || !vb_ok) ? T(0) : b; };
    auto erow = [&](T av, T bv) -> T { return (y & 1) ? av : wy * (av + bv); };
    auto gu = [&](int x) -> T { return (urow + min(x, nxf - 1) * ldu)[tc]; };
    const int Xs = x0 >> 1;  // step i covers fine columns 2(Xs+i), 2(Xs+i)+1
    T qa[D], qb[D], q0[D], q1[D];
    auto issue = [&](int i, int s) {
        const int X = Xs + i;
        qa[s] = gca(X);
        qb[s] = gcb(X);
        q0[s] = gu(2 * X);
        q1[s] = gu(2 * X + 1);
    };
    T pa = gca(Xs - 1), pb = gcb(Xs - 1);
#pragma unroll
    for (int s = 0; s < D; ++s) issue(s, s);
    T aprev = am(pa, Xs - 1);
    T eprev = erow(aprev, bm(pb, Xs - 1));
    const bool centre = P1T && !(y & 1);  // even x on this row: SW / NE mean
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int s = i % D;
        const int X = Xs + i;
        const T a = am(qa[s], X), b = bm(qb[s], X);
        const T e = erow(a, b);
        const T u0 = q0[s], u1 = q1[s];
        if (i + D < NIT) issue(i + D, s);
        const int xe = 2 * X, xo = 2 * X + 1;
        const T ev = centre ? T(0.5) * (aprev + b) : T(0.5) * (eprev + e);
        if (ok && xe < x1) (urow + xe * ldu)[t] = u0 + ev;
        if (ok && xo < x1) (urow + xo * ldu)[t] = u1 + e;
        eprev = e;
        aprev = a;
    }
}

template <typename T, bool WAVE_NODE>
__global__ void k_prolong_add(const T* __restrict__ ec, int ldc, T* __restrict__ u, int ldu, int nxf, int width,
                              int p1) {
    const int mode = blockIdx.y * blockDim.x + threadIdx.x;
    int node = xcd_block(blockIdx.x, gridDim.x) * blockDim.y + threadIdx.y;
    if (WAVE_NODE) node = __builtin_amdgcn_readfirstlane(node);  // one node per wavefront
    if (mode >= width || node >= nxf * nxf) return;
    const int y = node / nxf, x = node - y * nxf;
    const int nxc = (nxf - 1) / 2;
    auto get = [&](int X, int Y) { return ec[((size_t)Y * nxc + X) * ldc + mode]; };
    u[(size_t)node * ldu + mode] += prolong_value<T>(get, nxc, x, y, p1 != 0);
}

// u = Kinv f for every column; one block per column, double arithmetic
template <typename T>
__global__ void k_coarse(const double* __restrict__ kinv, const T* __restrict__ f, int ldf, T* __restrict__ u,
                         int ldu, int Nc) {
    extern __shared__ double fs[];
    SG_POISON_LDS(fs, Nc);
    const int col = blockIdx.x;
    for (int i = threadIdx.x; i < Nc; i += blockDim.x) fs[i] = (double)f[(size_t)i * ldf + col];
    __syncthreads();
    for (int i = threadIdx.x; i < Nc; i += blockDim.x) {
        const double* row = kinv + (size_t)i * Nc;
        double acc = 0.0;
        for (int j = 0; j < Nc; ++j) acc = fma(row[j], fs[j], acc);
        u[(size_t)i * ldu + col] = (T)acc;
    }
}

// ----------------------------------------------------------------- row-phase Gauss-Seidel
// Four-colour Gauss-Seidel visits, in a forward sweep, the rows with odd y
// (grid index J even) and then the rows with even y; inside a row it updates
// first the nodes with x parity fx ("F") and then the others ("S").  The F
// nodes of a row only need old values of their row and the (stable) rows
// above and below, and the S nodes need the new F values of their row.  So
// one launch per row parity updates both colours: a workgroup walks a row
// segment of kRowSeg nodes, S node by S node, computing F(s+1) and then S(s),
// with the new F values kept in registers and the F node left of the first S
// node recomputed.  Reads come from A (the sweep's input: own rows) and V
// (the neighbour rows: A in the first phase, B in the second), writes go to
// B, so no workgroup reads what another one writes.  One wavefront per 64
// modes; lanes are modes.
//
// The walk is a chain of dependent steps, so the loads of step i + D are
// issued before step i is computed (a ring of D register slots): every load
// address is clamped into the grid and the value is replaced by zero where
// the node lies outside, so the loads carry no branches and stay in flight
// while earlier steps compute.  The segment's stencils are staged in LDS
// once per workgroup.
constexpr int kRowSeg = 32;       // nodes per segment on the fine levels
constexpr int kRowSegShort = 8;   // on coarse levels, where long walks leave too few workgroups

template <typename T>
constexpr int gs_ring() { return sizeof(T) == 4 ? 4 : 3; }

template <typename T, int SEG>
__global__ void __launch_bounds__(256) k_gs_rows(const T* __restrict__ sten, const T* __restrict__ rdiag,
                                                 const T* __restrict__ A, int lda,
                                                 const T* __restrict__ V, int ldv, const T* __restrict__ f, int ldf,
                                                 T* __restrict__ B, int ldb, int nx, int width, int py, int fx,
                                                 int nseg, int nrows) {
    constexpr int NIT = SEG / 2;          // S nodes per segment
    constexpr int D = gs_ring<T>();
    constexpr int SP = sizeof(T) == 4 ? 12 : 10;  // LDS pitch of a staged stencil
    __shared__ T stl[(SEG + 2) * SP];
    const int lane = threadIdx.x & 63;
    const int s_w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = s_w * 64 + lane;
    const bool ok = t < width;
    const int tc = ok ? t : width - 1;  // lanes past the block load a valid column and store nothing
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    if (lb >= nrows * nseg) return;     // uniform over the workgroup
    SG_POISON_LDS(stl, sizeof(stl) / sizeof(T));
    const int r = lb / nseg;
    const int y = py + 2 * r;
    const int x0 = (lb - r * nseg) * SEG;  // even
    const int x1 = min(x0 + SEG, nx);
    const bool has_dn = y > 0, has_up = y + 1 < nx;
    const int ydn = y > 0 ? y - 1 : y, yup = y + 1 < nx ? y + 1 : y;
    // stencils of columns x0-1 .. x0+SEG (clamped), column c at stl[c * SP], the reciprocal
    // of its diagonal at stl[c * SP + 9]
    for (int i = threadIdx.x; i < (SEG + 2) * 10; i += blockDim.x) {
        const int c = i / 10, e = i - c * 10;
        const int x = min(max(x0 - 1 + c, 0), nx - 1);
        stl[c * SP + e] = e < 9 ? sten[((size_t)y * nx + x) * 9 + e] : rdiag[(size_t)y * nx + x];
    }
    __syncthreads();
    auto cx = [&](int x) { return min(max(x, 0), nx - 1); };
    auto inx = [&](int x) { return x >= 0 && x < nx; };
    // row bases computed once: own row of A, f and B, the rows below and above in V
    const T* const arow = A + (size_t)y * nx * lda;
    const T* const frow = f + (size_t)y * nx * ldf;
    const T* const dnrow = V + (size_t)ydn * nx * ldv;
    const T* const uprow = V + (size_t)yup * nx * ldv;
    T* const brow = B + (size_t)y * nx * ldb;
    auto gA = [&](int x) -> T { return (arow + cx(x) * lda)[tc]; };
    auto gD = [&](int x) -> T { return (dnrow + cx(x) * ldv)[tc]; };
    auto gU = [&](int x) -> T { return (uprow + cx(x) * ldv)[tc]; };
    auto gf = [&](int x) -> T { return (frow + cx(x) * ldf)[tc]; };
    auto zA = [&](T v, int x) -> T { return inx(x) ? v : T(0); };
    auto zD = [&](T v, int x) -> T { return (has_dn && inx(x)) ? v : T(0); };
    auto zU = [&](T v, int x) -> T { return (has_up && inx(x)) ? v : T(0); };
    // new value at column x from its same-row neighbours wl, wr and the rows
    // below (d0..d2) and above (u0..u2) at x-1, x, x+1
    auto relax = [&](int x, T fv, T wl, T wr, T d0, T d1, T d2, T u0, T u1, T u2) -> T {
        const T* st = stl + (x - x0 + 1) * SP;
        T acc = fv;
        acc -= st[0] * d0 + st[1] * d1 + st[2] * d2;
        acc -= st[6] * u0 + st[7] * u1 + st[8] * u2;
        acc -= st[3] * wl + st[5] * wr;
        return acc * st[9];
    };
    const int sf = x0 + (fx ? 0 : 1);  // first S node of the segment (S parity is 1 - fx)
    // ring slots: step i reads A(s+2), f(s), f(s+1) and the neighbour rows at s+1, s+2
    T qa[D], qfs[D], qff[D], qd1[D], qd2[D], qu1[D], qu2[D];
    auto issue = [&](int i, int k) {
        const int s = sf + 2 * i;
        qa[k] = gA(s + 2);
        qfs[k] = gf(s);
        qff[k] = gf(s + 1);
        qd1[k] = gD(s + 1);
        qd2[k] = gD(s + 2);
        qu1[k] = gU(s + 1);
        qu2[k] = gU(s + 2);
    };
    // prologue: window columns sf-2 .. sf, own values at sf-2 and sf, f(sf-1)
    T dm = gD(sf - 2), d0 = gD(sf - 1), d1 = gD(sf);
    T um = gU(sf - 2), u0 = gU(sf - 1), u1 = gU(sf);
    T am = gA(sf - 2), Sold = gA(sf);
    const T fp = gf(sf - 1);
#pragma unroll
    for (int k = 0; k < D; ++k) issue(k, k);
    dm = zD(dm, sf - 2); d0 = zD(d0, sf - 1); d1 = zD(d1, sf);
    um = zU(um, sf - 2); u0 = zU(u0, sf - 1); u1 = zU(u1, sf);
    am = zA(am, sf - 2); Sold = zA(Sold, sf);
    // new F(sf - 1): belongs to this segment when fx = 0, else to the one on the left
    T Fprev = T(0);
    if (sf - 1 >= 0) {
        Fprev = relax(sf - 1, fp, am, Sold, dm, d0, d1, um, u0, u1);
        if (!fx && ok) (brow + (sf - 1) * ldb)[t] = Fprev;
    }
#pragma unroll
    for (int i = 0; i < NIT; ++i) {
        const int k = i % D;
        const int s = sf + 2 * i;
        const T Snext = zA(qa[k], s + 2);
        const T fS = qfs[k], fF = qff[k];
        const T d2 = zD(qd1[k], s + 1), d3 = zD(qd2[k], s + 2);
        const T u2 = zU(qu1[k], s + 1), u3 = zU(qu2[k], s + 2);
        if (i + D < NIT) issue(i + D, k);
        // F(s+1) from old S(s), S(s+2); zero outside the grid
        T Fnew = T(0);
        if (s + 1 < nx) {
            Fnew = relax(s + 1, fF, Sold, Snext, d1, d2, d3, u1, u2, u3);
            if (s + 1 < x1 && ok) (brow + (s + 1) * ldb)[t] = Fnew;
        }
        // S(s) from new F(s-1), F(s+1)
        if (s < x1) {
            const T Snew = relax(s, fS, Fprev, Fnew, d0, d1, d2, u0, u1, u2);
            if (ok) (brow + s * ldb)[t] = Snew;
        }
        d0 = d2;
        d1 = d3;
        u0 = u2;
        u1 = u3;
        Sold = Snext;
        Fprev = Fnew;
    }
}

// The first four-colour sweep from the zero start, both row phases in one
// launch (W >= 32 modes).  A workgroup owns a segment of one phase-1 row y1
// (parity p1) and walks it together with the two phase-0 rows y1 - 1 and
// y1 + 1 around it: each step relaxes the phase-0 rows at S node s0 and F
// node s0 + 1 (from f alone: every old value is the zero start), then the
// phase-1 row one step behind, at s0 - 2 and s0 - 1, from the new values of
// the phase-0 rows kept in registers.  The phase-0 rows are relaxed twice (by
// the workgroups of y1 and y1 + 2; row 0 by the one of y1 = 1) and written
// once, by the workgroup below them; their walk starts two S nodes left of
// the segment and ends one right of it so that the phase-1 row has all its
// new neighbours.  Every node gets the update of k_gs_rows (same formula, the
// old values as exact zeros), so the launch equals the two row-phase launches
// of the sweep; only f is read.  (A form of this walk for sweeps with old
// values ran no faster than their two row-phase launches.)
template <typename T, int SEG>
__global__ void __launch_bounds__(256) k_gs_sweep0(const T* __restrict__ stp, const T* __restrict__ f, int ldf,
                                                   T* __restrict__ B, int ldb, int nx, int width, int p1, int fx,
                                                   int nseg, int nrows1) {
    constexpr int NIT = SEG / 2;                   // phase-1 S nodes per segment
    constexpr int NJ = NIT + 2;                    // phase-0 steps
    constexpr int D = 2;                           // steps of loads in flight
    constexpr int SP = sizeof(T) == 4 ? 12 : 10;  // pitch of a padded stencil (9 + reciprocal diagonal)
    constexpr int NC = SEG + 8;                    // staged columns sf - 4 .. sf + SEG + 3
    constexpr int NL = 6;                          // loads per step
    __shared__ T stl[3 * NC * SP];
    const int lane = threadIdx.x & 63;
    const int s_w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int t = s_w * 64 + lane;
    const bool ok = t < width;
    const int tc = ok ? t : width - 1;
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    if (lb >= nrows1 * nseg) return;  // uniform over the workgroup
    SG_POISON_LDS(stl, sizeof(stl) / sizeof(T));
    const int r = lb / nseg;
    const int y1 = p1 + 2 * r;
    const int x0 = (lb - r * nseg) * SEG;
    const int x1 = min(x0 + SEG, nx);
    const int sf = x0 + (fx ? 0 : 1);  // first S node of the segment (S parity is 1 - fx)
    const int cb = sf - 4;             // column of the first staged stencil
    // stencils of rows y1 - 1, y1, y1 + 1 (clamped into the grid)
    for (int i = threadIdx.x; i < 3 * NC * SP; i += blockDim.x) {
        const int rk = i / (NC * SP), rem = i - rk * (NC * SP);
        const int c = rem / SP, e = rem - c * SP;
        const int yy = min(max(y1 - 1 + rk, 0), nx - 1), xx = min(max(cb + c, 0), nx - 1);
        stl[i] = stp[((size_t)yy * nx + xx) * SP + e];
    }
    __syncthreads();
    const bool hasA = y1 >= 1, hasB = y1 + 1 < nx;  // phase-0 rows y1 - 1, y1 + 1
    const bool writeA = y1 == 1;                     // row 0 has no workgroup below it
    // f rows y1 - 1 .. y1 + 1 and output rows (clamped into the grid)
    const T* frow[3];
    T* brow[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int yy = min(max(y1 - 1 + k, 0), nx - 1);
        frow[k] = f + (size_t)yy * nx * ldf;
        brow[k] = B + (size_t)yy * nx * ldb;
    }
    auto cx = [&](int x) { return min(max(x, 0), nx - 1); };
    auto inx = [&](int x) { return x >= 0 && x < nx; };
    auto gF = [&](int k, int x) -> T { return (frow[k] + cx(x) * ldf)[tc]; };
    const T z = T(0);  // an old value (the zero start)
    auto relax = [&](int rk, int x, T fv, T wl, T wr, T d0, T d1, T d2, T u0, T u1, T u2) -> T {
        const T* st = stl + (rk * NC + (x - cb)) * SP;
        T acc = fv;
        acc -= st[0] * d0 + st[1] * d1 + st[2] * d2;
        acc -= st[6] * u0 + st[7] * u1 + st[8] * u2;
        acc -= st[3] * wl + st[5] * wr;
        return acc * st[9];
    };
    auto put = [&](int rk, int x, T v) {
        if (ok && x >= x0 && x < x1) (brow[rk] + x * ldb)[t] = v;
    };
    // loads of phase-0 step j (s0 = sf - 2 + 2j): f of rows y1 - 1, y1, y1 + 1 at s0, s0 + 1
    T q[D][NL];
    auto issue = [&](int j, int slot) {
        const int s0 = sf - 2 + 2 * j;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            q[slot][2 * k] = gF(k, s0);
            q[slot][2 * k + 1] = gF(k, s0 + 1);
        }
    };
    const T fa3 = gF(0, sf - 3), fb3 = gF(2, sf - 3);
#pragma unroll
    for (int k = 0; k < D; ++k) issue(k, k);
    // new F(sf - 3) of the phase-0 rows
    T FaPrev = z, FbPrev = z;
    if (inx(sf - 3)) {
        if (hasA) FaPrev = relax(0, sf - 3, fa3, z, z, z, z, z, z, z, z);
        if (hasB) FbPrev = relax(2, sf - 3, fb3, z, z, z, z, z, z, z, z);
    }
    // new values of the phase-0 rows at s0 - 3 .. s0 + 1 (after a step)
    T nA[5] = {z, z, z, z, FaPrev}, nB[5] = {z, z, z, z, FbPrev};
    T f1p0 = z, f1p1 = z, F1prev = z;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int k = j % D;
        const int s0 = sf - 2 + 2 * j;
        T v[NL];
#pragma unroll
        for (int e = 0; e < NL; ++e) v[e] = q[k][e];
        if (j + D < NJ) issue(j + D, k);
        // phase 0: F(s0 + 1) from the old S(s0), S(s0 + 2); then S(s0) from the new F(s0 - 1), F(s0 + 1)
        T Fa = z, Sa = z, Fb = z, Sb = z;
        if (hasA) {
            if (inx(s0 + 1)) Fa = relax(0, s0 + 1, v[1], z, z, z, z, z, z, z, z);
            if (inx(s0)) Sa = relax(0, s0, v[0], FaPrev, Fa, z, z, z, z, z, z);
            if (writeA) {
                put(0, s0 + 1, Fa);
                put(0, s0, Sa);
            }
        }
        if (hasB) {
            if (inx(s0 + 1)) Fb = relax(2, s0 + 1, v[5], z, z, z, z, z, z, z, z);
            if (inx(s0)) Sb = relax(2, s0, v[4], FbPrev, Fb, z, z, z, z, z, z);
            put(2, s0 + 1, Fb);
            put(2, s0, Sb);
        }
        nA[0] = nA[2]; nA[1] = nA[3]; nA[2] = nA[4]; nA[3] = Sa; nA[4] = Fa;
        nB[0] = nB[2]; nB[1] = nB[3]; nB[2] = nB[4]; nB[3] = Sb; nB[4] = Fb;
        // phase 1, one step behind: the new phase-0 rows at s0 - 3 .. s0 are final
        if (j == 1) {
            // new F(sf - 1) from the old S(sf - 2), S(sf)
            if (inx(sf - 1)) {
                F1prev = relax(1, sf - 1, f1p1, z, z, nA[1], nA[2], nA[3], nB[1], nB[2], nB[3]);
                put(1, sf - 1, F1prev);
            }
        } else if (j >= 2) {
            const int s = s0 - 2;
            T F1 = z;
            if (inx(s + 1)) {
                F1 = relax(1, s + 1, f1p1, z, z, nA[1], nA[2], nA[3], nB[1], nB[2], nB[3]);
                put(1, s + 1, F1);
            }
            if (inx(s)) put(1, s, relax(1, s, f1p0, F1prev, F1, nA[0], nA[1], nA[2], nB[0], nB[1], nB[2]));
            F1prev = F1;
        }
        f1p0 = v[2];
        f1p1 = v[3];
        FaPrev = Fa;
        FbPrev = Fb;
    }
}

// ------------------------------------------------------------ one right-hand side
// The narrowest blocks of B_T (one mode at degree 0, a few at degree 1) cycle
// on the large grids as chains of short launches.  These two kernels cut the
// cycle to two launches per level.  A workgroup of 1024 threads owns one mode
// of a tile of kTileCX x kTileCY coarse nodes (a launch covers every tile and
// mode) and keeps the 64 x 64 fine nodes around the tile's fine core in LDS
// (with a border of zeros), one 2 x 2 block of nodes per thread, so each
// thread owns one node of every colour and holds its four stencils in
// registers.  A four-colour sweep is four colour passes in LDS; the values
// near the region's edge go stale (their neighbours outside are not
// updated), but the stale band grows by at most two nodes in x and one in y
// per row phase (the row-phase sweeps of k_gs_rows_narrow update a row's F
// nodes from old S nodes, then its S nodes), so with nu <= 2 the fine core
// plus one ring is exact.  Down: nu1 forward sweeps from zero, the residual on
// the core plus one ring, R = P^T into the coarse right-hand side, and the
// smoothed core written out.  Up: the smoothed values plus P e over the
// region, nu2 backward sweeps, the core written out.  Every relaxation,
// residual, restriction and prolongation has the formula of the multi-launch
// path (k_gs_rows_narrow, k_residual, k_restrict, k_prolong_add).
constexpr int kTileCX = 22, kTileCY = 26;  // coarse nodes per tile
constexpr int kTileHX = 10, kTileHY = 6;   // fine halo of the region in x, y
constexpr int kTileR = 64;                 // region side: 2 * 22 + 2 * 10 = 2 * 26 + 2 * 6 = 64
constexpr int kTileP = kTileR + 2;         // with the border of zeros
constexpr int kTileMaxNu = 2;              // sweeps the halo covers

template <typename T>
struct TileOwn {
    T st[4][9];
    T rd[4];
    T f[4];
    bool in[4];  // the node lies in the grid
};

// thread t owns block (t % 32, t / 32); its node of colour q (x odd for q even,
// y odd for q < 2) at region coordinates (lx, ly)
__device__ __forceinline__ void tile_node(int q, int t, int& lx, int& ly) {
    lx = 2 * (t & 31) + ((q & 1) ^ 1);
    ly = 2 * (t >> 5) + ((q >> 1) ^ 1);
}

template <typename T>
__device__ __forceinline__ void tile_load(const T* __restrict__ stp, const T* __restrict__ f, int ldf, int nx, int rx0,
                                          int ry0, TileOwn<T>& on) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int lx, ly;
        tile_node(q, threadIdx.x, lx, ly);
        const int gx = rx0 + lx, gy = ry0 + ly;
        on.in[q] = gx >= 0 && gx < nx && gy >= 0 && gy < nx;
        const size_t node = on.in[q] ? (size_t)gy * nx + gx : 0;
        const T* e = stp + node * (sizeof(T) == 4 ? 12 : 10);
        if constexpr (sizeof(T) == 4) {
            const float4 a = ((const float4*)e)[0], b = ((const float4*)e)[1], c = ((const float4*)e)[2];
            on.st[q][0] = a.x; on.st[q][1] = a.y; on.st[q][2] = a.z; on.st[q][3] = a.w;
            on.st[q][4] = b.x; on.st[q][5] = b.y; on.st[q][6] = b.z; on.st[q][7] = b.w;
            on.st[q][8] = c.x; on.rd[q] = c.y;
        } else {
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const double2 v = ((const double2*)e)[k];
                on.st[q][2 * k] = v.x;
                if (k < 4) on.st[q][2 * k + 1] = v.y; else on.rd[q] = v.y;
            }
        }
        on.f[q] = f[node * ldf];
    }
}

// colour passes of nu sweeps on the padded region (forward: colours 0..3)
template <typename T>
__device__ __forceinline__ void tile_sweeps(const TileOwn<T>& on, T* u, int nu, bool reverse) {
    for (int sw = 0; sw < nu; ++sw)
#pragma unroll
        for (int qi = 0; qi < 4; ++qi) {
            const int q = reverse ? 3 - qi : qi;
            int lx, ly;
            tile_node(q, threadIdx.x, lx, ly);
            if (on.in[q]) {
                const T* s = on.st[q];
                T* c = u + (ly + 1) * kTileP + lx + 1;
                T acc = on.f[q];
                acc -= s[0] * c[-kTileP - 1] + s[1] * c[-kTileP] + s[2] * c[-kTileP + 1];
                acc -= s[6] * c[kTileP - 1] + s[7] * c[kTileP] + s[8] * c[kTileP + 1];
                acc -= s[3] * c[-1] + s[5] * c[1];
                *c = acc * on.rd[q];
            }
            __syncthreads();
        }
}

// workgroup b: tile b % ntiles of mode b / ntiles (pointers address mode 0)
template <typename T>
__global__ void __launch_bounds__(1024) k_cycle1_down(const T* __restrict__ stp, const T* __restrict__ f, int ldf,
                                                      T* __restrict__ uo, int ldo, T* __restrict__ fc, int ldc, int nx,
                                                      int nu, int ntx, int ntiles, int p1) {
    __shared__ T u[kTileP * kTileP];
    __shared__ T r[(2 * kTileCX + 1) * (2 * kTileCY + 1)];
    SG_POISON_LDS(u, kTileP * kTileP);
    SG_POISON_LDS(r, (2 * kTileCX + 1) * (2 * kTileCY + 1));
    constexpr int RW = 2 * kTileCX + 1;
    const int mode = blockIdx.x / ntiles, tile = blockIdx.x - mode * ntiles;
    f += mode;
    uo += mode;
    fc += mode;
    const int nxc = (nx - 1) / 2;
    const int X0 = (tile % ntx) * kTileCX, Y0 = (tile / ntx) * kTileCY;
    const int rx0 = 2 * X0 - kTileHX, ry0 = 2 * Y0 - kTileHY;
    for (int i = threadIdx.x; i < kTileP * kTileP; i += blockDim.x) u[i] = T(0);  // zero start and border
    TileOwn<T> on;
    tile_load<T>(stp, f, ldf, nx, rx0, ry0, on);
    __syncthreads();
    tile_sweeps<T>(on, u, nu, false);
    // residual at fine nodes 2 X0 .. 2 X0 + 2 kTileCX (and y alike), the formula of k_residual
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int lx, ly;
        tile_node(q, threadIdx.x, lx, ly);
        const int ax = rx0 + lx - 2 * X0, ay = ry0 + ly - 2 * Y0;
        if (on.in[q] && ax >= 0 && ax <= 2 * kTileCX && ay >= 0 && ay <= 2 * kTileCY) {
            const T* c = u + (ly + 1) * kTileP + lx + 1;
            T acc = on.f[q];
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) acc -= on.st[q][(dy + 1) * 3 + (dx + 1)] * c[dy * kTileP + dx];
            r[ay * RW + ax] = acc;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTileCX * kTileCY; i += blockDim.x) {
        const int X = X0 + i % kTileCX, Y = Y0 + i / kTileCX;
        if (X < nxc && Y < nxc)
            fc[((size_t)Y * nxc + X) * ldc] = restrict_value<T>(
                [&](int x, int y) { return r[(y - 2 * Y0) * RW + (x - 2 * X0)]; }, X, Y, p1 != 0);
    }
    // the smoothed core (the last tile of a row or column also owns the grid's last node)
    const int cx1 = X0 + kTileCX >= nxc ? nx : 2 * (X0 + kTileCX);
    const int cy1 = Y0 + kTileCY >= nxc ? nx : 2 * (Y0 + kTileCY);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int lx, ly;
        tile_node(q, threadIdx.x, lx, ly);
        const int gx = rx0 + lx, gy = ry0 + ly;
        if (gx >= 2 * X0 && gx < cx1 && gy >= 2 * Y0 && gy < cy1)
            uo[((size_t)gy * nx + gx) * ldo] = u[(ly + 1) * kTileP + lx + 1];
    }
}

template <typename T>
__global__ void __launch_bounds__(1024) k_cycle1_up(const T* __restrict__ stp, const T* __restrict__ f, int ldf,
                                                    const T* __restrict__ ui, int ldi, const T* __restrict__ ec,
                                                    int ldc, T* __restrict__ uo, int ldo, int nx, int nu, int ntx,
                                                    int ntiles, int p1) {
    __shared__ T u[kTileP * kTileP];
    SG_POISON_LDS(u, kTileP * kTileP);
    const int mode = blockIdx.x / ntiles, tile = blockIdx.x - mode * ntiles;
    f += mode;
    ui += mode;
    ec += mode;
    uo += mode;
    const int nxc = (nx - 1) / 2;
    const int X0 = (tile % ntx) * kTileCX, Y0 = (tile / ntx) * kTileCY;
    const int rx0 = 2 * X0 - kTileHX, ry0 = 2 * Y0 - kTileHY;
    for (int i = threadIdx.x; i < kTileP * kTileP; i += blockDim.x) u[i] = T(0);  // border, nodes outside the grid
    TileOwn<T> on;
    tile_load<T>(stp, f, ldf, nx, rx0, ry0, on);
    __syncthreads();
    // smoothed values plus the prolonged correction, the formula of k_prolong_add
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int lx, ly;
        tile_node(q, threadIdx.x, lx, ly);
        const int gx = rx0 + lx, gy = ry0 + ly;
        if (on.in[q]) {
            T v = ui[((size_t)gy * nx + gx) * ldi];
            v += prolong_value<T>([&](int X, int Y) { return ec[((size_t)Y * nxc + X) * ldc]; }, nxc, gx, gy, p1 != 0);
            u[(ly + 1) * kTileP + lx + 1] = v;
        }
    }
    __syncthreads();
    tile_sweeps<T>(on, u, nu, true);
    const int cx1 = X0 + kTileCX >= nxc ? nx : 2 * (X0 + kTileCX);
    const int cy1 = Y0 + kTileCY >= nxc ? nx : 2 * (Y0 + kTileCY);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int lx, ly;
        tile_node(q, threadIdx.x, lx, ly);
        const int gx = rx0 + lx, gy = ry0 + ly;
        if (gx >= 2 * X0 && gx < cx1 && gy >= 2 * Y0 && gy < cy1)
            uo[((size_t)gy * nx + gx) * ldo] = u[(ly + 1) * kTileP + lx + 1];
    }
}

// Row-phase Gauss-Seidel for narrow blocks (W <= 32 modes): the same update
// as k_gs_rows without the walk.  A lane owns, for one mode, the S node s of
// a row and the F node s + 1, and recomputes the F node s - 1 that its S
// update also needs; lanes cover (row, S node, mode), wpad >= W adjacent
// lanes per node pair, so narrow blocks still fill the chip and every lane
// issues all its loads at once.  Addresses are clamped into the
// grid and values outside it replaced by zero.
template <typename T, bool OWNZ>
__global__ void __launch_bounds__(256) k_gs_rows_narrow(const T* __restrict__ stp,
                                                        const T* __restrict__ A, int lda,
                                                        const T* __restrict__ V, int ldv, const T* __restrict__ f,
                                                        int ldf, T* __restrict__ B, int ldb, int nx, int width,
                                                        int wpad, int py, int fx, int vert_zero, int npairs,
                                                        int nrows) {
    // lanes (pair, mode): wpad >= W adjacent lanes per node pair
    const unsigned gl = (unsigned)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const unsigned pl = gl / (unsigned)wpad;
    const int mode = (int)(gl - pl * (unsigned)wpad);
    const int r = (int)(pl / (unsigned)npairs);
    const int j = (int)(pl - (unsigned)r * (unsigned)npairs);
    if (r >= nrows || mode >= width) return;  // no barriers below
    const int y = py + 2 * r;
    // S nodes have parity 1 - fx; with fx = 0 the first pair is (none, F(0))
    const int s = 2 * j - (fx ? 0 : 1);
    const bool has_dn = y > 0 && !vert_zero, has_up = y + 1 < nx && !vert_zero;
    const int ydn = y > 0 ? y - 1 : y, yup = y + 1 < nx ? y + 1 : y;
    auto cx = [&](int x) { return min(max(x, 0), nx - 1); };
    auto inx = [&](int x) { return x >= 0 && x < nx; };
    auto gA = [&](int x) -> T { return OWNZ ? T(0) : A[((size_t)y * nx + cx(x)) * lda + mode]; };
    auto gV = [&](int yy, int x) -> T { return V[((size_t)yy * nx + cx(x)) * ldv + mode]; };
    auto gf = [&](int x) -> T { return f[((size_t)y * nx + cx(x)) * ldf + mode]; };
    T a[3], fv[3], dn[5], up[5], st[3][9], rd[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        a[i] = gA(s - 2 + 2 * i);
        fv[i] = gf(s - 1 + i);
        // the node's padded stencil entry in 16-byte pieces
        const T* sp = stp + ((size_t)y * nx + cx(s - 1 + i)) * (sizeof(T) == 4 ? 12 : 10);
        if constexpr (sizeof(T) == 4) {
            const float4 p0 = ((const float4*)sp)[0], p1 = ((const float4*)sp)[1], p2 = ((const float4*)sp)[2];
            st[i][0] = p0.x; st[i][1] = p0.y; st[i][2] = p0.z; st[i][3] = p0.w;
            st[i][4] = p1.x; st[i][5] = p1.y; st[i][6] = p1.z; st[i][7] = p1.w;
            st[i][8] = p2.x; rd[i] = p2.y;
        } else {
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const double2 v = ((const double2*)sp)[k];
                st[i][2 * k] = v.x;
                if (k < 4) st[i][2 * k + 1] = v.y; else rd[i] = v.y;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        dn[i] = gV(ydn, s - 2 + i);
        up[i] = gV(yup, s - 2 + i);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) a[i] = (!OWNZ && inx(s - 2 + 2 * i)) ? a[i] : T(0);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        dn[i] = (has_dn && inx(s - 2 + i)) ? dn[i] : T(0);
        up[i] = (has_up && inx(s - 2 + i)) ? up[i] : T(0);
    }
    // node s - 1 + i (i = 0, 1, 2) with same-row neighbours wl, wr
    auto relax = [&](int i, T wl, T wr) -> T {
        const T* c = st[i];
        T acc = fv[i];
        acc -= c[0] * dn[i] + c[1] * dn[i + 1] + c[2] * dn[i + 2];
        acc -= c[6] * up[i] + c[7] * up[i + 1] + c[8] * up[i + 2];
        acc -= c[3] * wl + c[5] * wr;
        return acc * rd[i];
    };
    const T Fl = inx(s - 1) ? relax(0, a[0], a[1]) : T(0);
    const T Fr = inx(s + 1) ? relax(2, a[1], a[2]) : T(0);
    if (inx(s + 1)) B[((size_t)y * nx + s + 1) * ldb + mode] = Fr;
    if (inx(s)) B[((size_t)y * nx + s) * ldb + mode] = relax(1, Fl, Fr);
}

// ----------------------------------------------------------------- coarse grids in LDS
// The grids at and below kFusedNx interior nodes per side are cycled by a
// single launch: one workgroup per right-hand-side column keeps u and f of
// every coarse level (and one residual array) in LDS and runs smoothing,
// residual, restriction, the coarsest solve, prolongation and
// post-smoothing with workgroup barriers between passes.  This replaces
// about twenty launches per coarse level.
constexpr int kMaxFusedLevels = 8;

template <typename T>
struct FusedLevels {
    int nlev;                       // levels in the fused part, the last is the coarsest
    int nx[kMaxFusedLevels];
    int off[kMaxFusedLevels];       // LDS element offset of u_l (f_l follows at off + N_l)
    const T* sten[kMaxFusedLevels];
    const T* rdiag[kMaxFusedLevels];  // reciprocals of the stencil diagonals
    int roff;                       // LDS element offset of the residual / staging array
    int p1;                         // transfer of the P1 triangulation (else bilinear)
};

template <typename T>
constexpr int fused_nx_max() { return sizeof(T) == 4 ? 63 : 31; }

// one relaxation of node (x, y) against the current values of its neighbours
template <typename T, typename G>
__device__ __forceinline__ T relax_node(const T* __restrict__ s9, T rd, T fval, int x, int y, int nx, G get) {
    T acc = fval;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        const int yy = y + dy;
        if (yy < 0 || yy >= nx) continue;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            const int xx = x + dx;
            if (xx < 0 || xx >= nx) continue;
            acc -= s9[(dy + 1) * 3 + (dx + 1)] * get(yy * nx + xx);
        }
    }
    return acc * rd;
}

// Lexicographic order (x fastest, then y) for a 9-point stencil: the
// neighbours of (x, y) that come earlier all have a smaller x + 2y and the
// later ones a larger, so the nodes of one front x + 2y = d are independent
// and a sweep visits the 3(nx-1)+1 fronts in order (backward: in reverse).
// Front d holds y = ylo..yhi with x = d - 2y.
__device__ __forceinline__ void lex_front(int d, int nx, int& ylo, int& yhi) {
    ylo = max(0, (d - nx + 2) / 2);
    yhi = min(nx - 1, d / 2);
}

// Lexicographic sweeps by one wavefront, for grids of at most kLexWaveMaxNx
// nodes per side held in LDS (u and f, nx x nx each): lane y owns grid row y,
// and at front d every lane relaxes node (d - 2y, y) of its row.  One
// wavefront needs no workgroup barrier between fronts (the LDS operations of a
// wavefront complete in issue order; the wavefront-scope fences keep the
// compiler from moving LDS accesses across a front).  Each lane loads the
// stencils and right-hand sides of its next kLexAhead nodes ahead of time
// (f does not change during a sweep), and reads the eight
// neighbours at clamped addresses (zero outside the grid) so that the reads
// carry no branches and are issued together.  The relaxation sums the
// neighbours in two chains (same values as k_gs_lex up to rounding).
constexpr int kLexWaveMaxNx = 63;  // at most 64 rows, one per lane
constexpr int kLexAhead = 8;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ void wave_lex_sweeps(const T* __restrict__ sten, const T* __restrict__ rdiag, T* us,
                                                const T* fs, int nx, bool reverse, int nu) {
    const int y = threadIdx.x & 63;
    const int nd = 3 * (nx - 1) + 1;
    for (int sweep = 0; sweep < nu; ++sweep) {
        auto node_at = [&](int di) -> int {
            const int d = reverse ? nd - 1 - di : di, x = d - 2 * y;
            return (di < nd && y < nx && x >= 0 && x < nx) ? y * nx + x : -1;
        };
        T st[kLexAhead][9], rd[kLexAhead], rf[kLexAhead];
        auto fetch = [&](int j, int di) {
            const int node = max(node_at(di), 0);
#pragma unroll
            for (int t = 0; t < 9; ++t) st[j][t] = sten[(size_t)node * 9 + t];
            rd[j] = rdiag[node];
            rf[j] = fs[node];
        };
#pragma unroll
        for (int j = 0; j < kLexAhead; ++j) fetch(j, j);
        for (int di0 = 0; di0 < nd; di0 += kLexAhead) {
#pragma unroll
            for (int j = 0; j < kLexAhead; ++j) {
                const int node = node_at(di0 + j);
                if (node >= 0) {
                    const int x = node - y * nx;
                    T v[9];
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int xx = x + dx, yy = y + dy, t = (dy + 1) * 3 + (dx + 1);
                            const bool in = xx >= 0 && xx < nx && yy >= 0 && yy < nx;
                            const T w = us[in ? yy * nx + xx : node];
                            v[t] = in ? w : T(0);
                        }
                    // two partial sums (rows below and above the node) shorten the dependent chain
                    T lo = rf[j] - st[j][0] * v[0], hi = st[j][6] * v[6];
                    lo -= st[j][1] * v[1];
                    hi += st[j][7] * v[7];
                    lo -= st[j][2] * v[2];
                    hi += st[j][8] * v[8];
                    lo -= st[j][3] * v[3];
                    hi += st[j][5] * v[5];
                    us[node] = (lo - hi) * rd[j];
                }
                fetch(j, di0 + j + kLexAhead);
                wave_sync();
            }
        }
    }
}

// One lexicographic sweep per right-hand-side column, one wavefront each:
// the column sits in LDS inside a border of zeros ((nx+2)^2 values), so a
// node's eight neighbours are read at fixed offsets from one address with no
// bounds tests, and f, the stencils and the reciprocal diagonals (none of
// which the sweep changes) are loaded from global memory kLexAhead fronts
// ahead.  zero_start: the column starts from zero (not read).  Same fronts
// and arithmetic as wave_lex_sweeps.
template <typename T>
__global__ void __launch_bounds__(64) k_lex_wave(const T* __restrict__ sten, const T* __restrict__ rdiag, T* u,
                                                 int ldu, const T* __restrict__ f, int ldf, int nx, int reverse,
                                                 int zero_start) {
    extern __shared__ char smem_raw[];
    T* us = (T*)smem_raw;
    const int col = blockIdx.x, pw = nx + 2, N = nx * nx;
    SG_POISON_LDS(us, pw * pw);
    for (int i = threadIdx.x; i < pw * pw; i += 64) {
        const int py = i / pw, px = i - py * pw;
        const bool in = px >= 1 && px <= nx && py >= 1 && py <= nx;
        us[i] = (in && !zero_start) ? u[(size_t)((py - 1) * nx + px - 1) * ldu + col] : T(0);
    }
    wave_sync();
    const int y = threadIdx.x;
    const int nd = 3 * (nx - 1) + 1;
    auto x_at = [&](int di) -> int { return (reverse ? nd - 1 - di : di) - 2 * y; };
    auto live = [&](int di, int x) { return di < nd && y < nx && x >= 0 && x < nx; };
    T st[kLexAhead][9], rd[kLexAhead], rf[kLexAhead];
    auto fetch = [&](int j, int di) {
        const int x = x_at(di);
        const int node = live(di, x) ? y * nx + x : 0;
#pragma unroll
        for (int t = 0; t < 9; ++t) st[j][t] = sten[(size_t)node * 9 + t];
        rd[j] = rdiag[node];
        rf[j] = f[(size_t)node * ldf + col];
    };
#pragma unroll
    for (int j = 0; j < kLexAhead; ++j) fetch(j, j);
    for (int di0 = 0; di0 < nd; di0 += kLexAhead) {
#pragma unroll
        for (int j = 0; j < kLexAhead; ++j) {
            const int x = x_at(di0 + j);
            if (live(di0 + j, x)) {
                // b: the south-west neighbour of node (x, y) in the padded grid
                T* b = us + y * pw + x;
                const T vSW = b[0], vS = b[1], vSE = b[2], vW = b[pw], vE = b[pw + 2];
                const T vNW = b[2 * pw], vN = b[2 * pw + 1], vNE = b[2 * pw + 2];
                T lo = rf[j] - st[j][0] * vSW, hi = st[j][6] * vNW;
                lo -= st[j][1] * vS;
                hi += st[j][7] * vN;
                lo -= st[j][2] * vSE;
                hi += st[j][8] * vNE;
                lo -= st[j][3] * vW;
                hi += st[j][5] * vE;
                b[pw + 1] = (lo - hi) * rd[j];
            }
            fetch(j, di0 + j + kLexAhead);
            wave_sync();
        }
    }
    for (int i = threadIdx.x; i < N; i += 64) {
        const int py = i / nx, px = i - py * nx;
        u[(size_t)i * ldu + col] = us[(py + 1) * pw + px + 1];
    }
}

// mode 0: four colours; 1: red/black from start-of-colour values; 2: lexicographic
template <typename T>
__device__ void lds_smooth(const T* __restrict__ st, const T* __restrict__ rdiag, T* u, const T* f, T* stage, int nx,
                           int mode, bool reverse,
                           int nu) {
    if (mode == 2) {
        // the first wavefront sweeps (every fused grid has at most 63 rows); the others wait
        if (threadIdx.x < 64) wave_lex_sweeps<T>(st, rdiag, u, f, nx, reverse, nu);
        __syncthreads();
        return;
    }
    const bool rb = mode == 1;
    const int ncol = rb ? 2 : 4;
    for (int sweep = 0; sweep < nu; ++sweep)
        for (int qi = 0; qi < ncol; ++qi) {
            const int q = reverse ? ncol - 1 - qi : qi;
            int nxc, nyc;
            if (rb) { nxc = (nx + 1) / 2; nyc = nx; }
            else { nxc = (nx - (((q & 1) ^ 1)) + 1) / 2; nyc = (nx - (((q >> 1) ^ 1)) + 1) / 2; }
            for (int t = threadIdx.x; t < nxc * nyc; t += blockDim.x) {
                const int j = t / nxc, i = t - j * nxc;
                int x, y;
                if (rb) { y = j; x = ((q + y) & 1) + 2 * i; if (x >= nx) continue; }
                else { x = ((q & 1) ^ 1) + 2 * i; y = ((q >> 1) ^ 1) + 2 * j; }
                const int node = y * nx + x;
                const T* s9 = st + (size_t)node * 9;
                T acc = f[node];
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy) {
                    const int yy = y + dy;
                    if (yy < 0 || yy >= nx) continue;
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (dx == 0 && dy == 0) continue;
                        const int xx = x + dx;
                        if (xx < 0 || xx >= nx) continue;
                        acc -= s9[(dy + 1) * 3 + (dx + 1)] * u[yy * nx + xx];
                    }
                }
                const T val = acc * rdiag[node];
                if (rb) stage[node] = val; else u[node] = val;
            }
            __syncthreads();
            if (rb) {
                for (int t = threadIdx.x; t < nxc * nyc; t += blockDim.x) {
                    const int y = t / nxc, i = t - y * nxc;
                    const int x = ((q + y) & 1) + 2 * i;
                    if (x < nx) u[y * nx + x] = stage[y * nx + x];
                }
                __syncthreads();
            }
        }
}

// One lexicographic Gauss-Seidel sweep (forward, or backward when reverse)
// on the separate-launch levels: one workgroup per right-hand-side column
// walks the fronts of lex_front in place, with a workgroup barrier between
// fronts.  zero_start: the column starts from zero (cleared here).
template <typename T>
__global__ void __launch_bounds__(256) k_gs_lex(const T* __restrict__ sten, const T* __restrict__ rdiag, T* u,
                                                int ldu, const T* __restrict__ f,
                                                int ldf, int nx, int reverse, int zero_start) {
    const int col = blockIdx.x;
    if (zero_start) {
        for (int i = threadIdx.x; i < nx * nx; i += blockDim.x) u[(size_t)i * ldu + col] = T(0);
        __syncthreads();
    }
    const int nd = 3 * (nx - 1) + 1;
    for (int di = 0; di < nd; ++di) {
        const int d = reverse ? nd - 1 - di : di;
        int ylo, yhi;
        lex_front(d, nx, ylo, yhi);
        for (int y = ylo + (int)threadIdx.x; y <= yhi; y += blockDim.x) {
            const int x = d - 2 * y, node = y * nx + x;
            u[(size_t)node * ldu + col] = relax_node<T>(sten + (size_t)node * 9, rdiag[node], f[(size_t)node * ldf + col], x, y,
                                                       nx, [&](int i) { return u[(size_t)i * ldu + col]; });
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(512) k_vcycle_fused(FusedLevels<T> fl, const double* __restrict__ kinv,
                                                      const T* __restrict__ fin, int ldf, T* __restrict__ uout,
                                                      int ldu, int nu1, int nu2, int mode) {
    extern __shared__ char smem_raw[];
    T* lds = (T*)smem_raw;
    T* r = lds + fl.roff;
    SG_POISON_LDS(lds, fl.roff + fl.nx[0] * fl.nx[0]);
    const int col = blockIdx.x;
    const int L = fl.nlev - 1;
    {
        const int N0 = fl.nx[0] * fl.nx[0];
        T* f0 = lds + fl.off[0] + N0;
        for (int i = threadIdx.x; i < N0; i += blockDim.x) f0[i] = fin[(size_t)i * ldf + col];
    }
    __syncthreads();
    for (int l = 0; l < L; ++l) {
        const int nx = fl.nx[l], N = nx * nx;
        T* u = lds + fl.off[l];
        T* f = u + N;
        for (int i = threadIdx.x; i < N; i += blockDim.x) u[i] = T(0);
        __syncthreads();
        lds_smooth<T>(fl.sten[l], fl.rdiag[l], u, f, r, nx, mode, false, nu1);
        // residual r = f - K u
        for (int node = threadIdx.x; node < N; node += blockDim.x) {
            const int y = node / nx, x = node - y * nx;
            const T* s9 = fl.sten[l] + (size_t)node * 9;
            T acc = f[node];
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const int yy = y + dy;
                if (yy < 0 || yy >= nx) continue;
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int xx = x + dx;
                    if (xx < 0 || xx >= nx) continue;
                    acc -= s9[(dy + 1) * 3 + (dx + 1)] * u[yy * nx + xx];
                }
            }
            r[node] = acc;
        }
        __syncthreads();
        // restriction to the next level's right-hand side
        const int nxc = fl.nx[l + 1], Nc = nxc * nxc;
        T* fc = lds + fl.off[l + 1] + Nc;
        for (int node = threadIdx.x; node < Nc; node += blockDim.x) {
            const int Y = node / nxc, X = node - Y * nxc;
            fc[node] = restrict_value<T>([&](int x, int y) { return r[y * nx + x]; }, X, Y, fl.p1 != 0);
        }
        __syncthreads();
    }
    {
        // coarsest grid: u = K^{-1} f with the inverse precomputed in double
        const int nx = fl.nx[L], N = nx * nx;
        T* u = lds + fl.off[L];
        const T* f = u + N;
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            const double* row = kinv + (size_t)i * N;
            double acc = 0.0;
            for (int j = 0; j < N; ++j) acc = fma(row[j], (double)f[j], acc);
            u[i] = (T)acc;
        }
        __syncthreads();
    }
    for (int l = L - 1; l >= 0; --l) {
        const int nx = fl.nx[l], N = nx * nx, nxc = fl.nx[l + 1];
        T* u = lds + fl.off[l];
        const T* f = u + N;
        const T* ec = lds + fl.off[l + 1];
        for (int node = threadIdx.x; node < N; node += blockDim.x) {
            const int y = node / nx, x = node - y * nx;
            u[node] += prolong_value<T>([&](int X, int Y) { return ec[Y * nxc + X]; }, nxc, x, y, fl.p1 != 0);
        }
        __syncthreads();
        lds_smooth<T>(fl.sten[l], fl.rdiag[l], u, f, r, nx, mode, true, nu2);
    }
    {
        const int N0 = fl.nx[0] * fl.nx[0];
        const T* u0 = lds + fl.off[0];
        for (int i = threadIdx.x; i < N0; i += blockDim.x) uout[(size_t)i * ldu + col] = u0[i];
    }
}

// Four-colour variant of the fused coarse-grid cycle with the stencils in
// registers: every colour class of a fused grid has at most as many nodes as
// the workgroup has threads, so thread t owns the t-th node of every colour.  Its four 9-point stencils are loaded once per visit of a
// level; every smoothing pass, residual and prolongation then only touches
// LDS.
template <typename T>
struct OwnNodes {
    int node[4];
    int x[4], y[4];
    T st[4][9];
    T rd[4];  // reciprocal of the diagonal
};

template <typename T>
__device__ __forceinline__ void own_nodes(const T* __restrict__ sten, const T* __restrict__ rdiag, int nx,
                                          OwnNodes<T>& on) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int px = (q & 1) ^ 1, py = (q >> 1) ^ 1;
        const int nxc = (nx - px + 1) / 2, nyc = (nx - py + 1) / 2;
        const int t = threadIdx.x;
        on.node[q] = -1;
        if (t < nxc * nyc) {
            const int j = t / nxc, i = t - j * nxc;
            on.x[q] = px + 2 * i;
            on.y[q] = py + 2 * j;
            on.node[q] = on.y[q] * nx + on.x[q];
#pragma unroll
            for (int e = 0; e < 9; ++e) on.st[q][e] = sten[(size_t)on.node[q] * 9 + e];
            on.rd[q] = rdiag[on.node[q]];
        }
    }
}

// acc = f - sum over the stencil of u (skipping the centre when skip_c)
template <typename T>
__device__ __forceinline__ T stencil_rest(const OwnNodes<T>& on, int q, const T* u, T fval, int nx, bool skip_c) {
    const int x = on.x[q], y = on.y[q];
    T acc = fval;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
        const int yy = y + dy;
        if (yy < 0 || yy >= nx) continue;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            if (skip_c && dx == 0 && dy == 0) continue;
            const int xx = x + dx;
            if (xx < 0 || xx >= nx) continue;
            acc -= on.st[q][(dy + 1) * 3 + (dx + 1)] * u[yy * nx + xx];
        }
    }
    return acc;
}

template <typename T>
__device__ __forceinline__ void own_smooth(const OwnNodes<T>& on, T* u, const T* f, int nx, bool reverse, int nu) {
    for (int sweep = 0; sweep < nu; ++sweep)
#pragma unroll
        for (int qi = 0; qi < 4; ++qi) {
            const int q = reverse ? 3 - qi : qi;
            if (on.node[q] >= 0) {
                const int nd = on.node[q];
                u[nd] = stencil_rest<T>(on, q, u, f[nd], nx, true) * on.rd[q];
            }
            __syncthreads();
        }
}

// u = Kinv f on the coarsest grid (u, f = u + N in LDS), in double: output i
// is summed by a group of G threads (the largest power of two with G N <=
// blockDim, at most 64) over j = g, g + G, ..., then reduced across the group.
template <typename T>
__device__ __forceinline__ void coarsest_solve(const double* __restrict__ kinv, T* u, int N) {
    const T* f = u + N;
    int G = 1;
    while (G < 64 && 2 * G * N <= (int)blockDim.x) G *= 2;
    const int rows = (int)blockDim.x / G;  // outputs per pass
    const int g = threadIdx.x % G;
    for (int i0 = 0; i0 < N; i0 += rows) {  // uniform trip count
        const int i = i0 + (int)threadIdx.x / G;
        double acc = 0.0;
        if (i < N) {
            const double* row = kinv + (size_t)i * N;
            for (int j = g; j < N; j += G) acc = fma(row[j], (double)f[j], acc);
        }
        for (int o = G / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);  // groups lie inside a wavefront
        if (i < N && g == 0) u[i] = (T)acc;  // u and f are separate arrays
    }
    __syncthreads();
}

// NT threads: at least the largest colour class of the top fused grid
// (32 x 32 for 63 x 63 float grids, 16 x 16 for 31 x 31 double grids)
template <typename T>
constexpr int fused4_threads() { return sizeof(T) == 4 ? 1024 : 256; }

template <typename T>
__global__ void __launch_bounds__(fused4_threads<T>()) k_vcycle_fused4(FusedLevels<T> fl, const double* __restrict__ kinv,
                                                        const T* __restrict__ fin, int ldf, T* __restrict__ uout,
                                                        int ldu, int nu1, int nu2) {
    extern __shared__ char smem_raw[];
    T* lds = (T*)smem_raw;
    T* r = lds + fl.roff;
    SG_POISON_LDS(lds, fl.roff + fl.nx[0] * fl.nx[0]);
    const int col = blockIdx.x;
    const int L = fl.nlev - 1;
    {
        const int N0 = fl.nx[0] * fl.nx[0];
        T* f0 = lds + fl.off[0] + N0;
        for (int i = threadIdx.x; i < N0; i += blockDim.x) f0[i] = fin[(size_t)i * ldf + col];
    }
    __syncthreads();
    OwnNodes<T> on;
    for (int l = 0; l < L; ++l) {
        const int nx = fl.nx[l], N = nx * nx;
        T* u = lds + fl.off[l];
        T* f = u + N;
        own_nodes<T>(fl.sten[l], fl.rdiag[l], nx, on);
        for (int i = threadIdx.x; i < N; i += blockDim.x) u[i] = T(0);
        __syncthreads();
        own_smooth<T>(on, u, f, nx, false, nu1);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (on.node[q] >= 0) r[on.node[q]] = stencil_rest<T>(on, q, u, f[on.node[q]], nx, false);
        __syncthreads();
        const int nxc = fl.nx[l + 1], Nc = nxc * nxc;
        T* fc = lds + fl.off[l + 1] + Nc;
        for (int node = threadIdx.x; node < Nc; node += blockDim.x) {
            const int Y = node / nxc, X = node - Y * nxc;
            fc[node] = restrict_value<T>([&](int x, int y) { return r[y * nx + x]; }, X, Y, fl.p1 != 0);
        }
        __syncthreads();
    }
    coarsest_solve<T>(kinv, lds + fl.off[L], fl.nx[L] * fl.nx[L]);
    for (int l = L - 1; l >= 0; --l) {
        const int nx = fl.nx[l], N = nx * nx, nxc = fl.nx[l + 1];
        T* u = lds + fl.off[l];
        const T* f = u + N;
        const T* ec = lds + fl.off[l + 1];
        own_nodes<T>(fl.sten[l], fl.rdiag[l], nx, on);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (on.node[q] < 0) continue;
            u[on.node[q]] += prolong_value<T>([&](int X, int Y) { return ec[Y * nxc + X]; }, nxc, on.x[q], on.y[q],
                                              fl.p1 != 0);
        }
        __syncthreads();
        own_smooth<T>(on, u, f, nx, true, nu2);
    }
    {
        const int N0 = fl.nx[0] * fl.nx[0];
        const T* u0 = lds + fl.off[0];
        for (int i = threadIdx.x; i < N0; i += blockDim.x) uout[(size_t)i * ldu + col] = u0[i];
    }
}

// Padded form of the fused four-colour coarse cycle, for grids of 2^k - 1
// interior nodes per side (63, 31, 15, 7, 3 above the coarsest).  Every
// level's u sits in LDS inside a border of zeros, (nx + 2)^2 values, so a
// relaxation reads its eight neighbours without bounds tests; the level sizes
// are compile-time constants (one code path per size), so the neighbour
// offsets are immediates of the LDS loads.  A thread's stencils come from the
// level's colour-ordered copy in 16-byte pieces.  The arithmetic of every
// relaxation, residual, restriction and prolongation is that of
// k_vcycle_fused4 (the border's zeros enter as exact zero terms).
template <typename T>
struct PadLevels {
    int nlev;                       // fused levels, the last is the coarsest
    int nx[kMaxFusedLevels];
    int uoff[kMaxFusedLevels];      // LDS element offset of the padded u_l
    int foff[kMaxFusedLevels];      // LDS element offset of f_l (nx^2 values)
    const T* cst[kMaxFusedLevels];  // colour-ordered stencils of the levels above the coarsest
    const T* sten[kMaxFusedLevels];   // node-ordered stencils and reciprocal diagonals (lexicographic sweeps)
    const T* rdiag[kMaxFusedLevels];
    int roff;                       // LDS element offset of the residual of the top level
    int p1;                         // transfer of the P1 triangulation (else bilinear)
};

template <typename T>
constexpr int cst_pitch() { return sizeof(T) == 4 ? 12 : 10; }

template <typename T>
struct OwnPad {
    T st[4][9];
    T rd[4];
};

// the node of colour q owned by thread t on an NX x NX grid
template <int NX>
__device__ __forceinline__ bool pad_own(int q, int t, int& x, int& y) {
    const int px = (q & 1) ^ 1, py = (q >> 1) ^ 1;
    const int nxc = (NX - px + 1) / 2, nyc = (NX - py + 1) / 2;
    const int j = t / nxc, i = t - j * nxc;
    x = px + 2 * i;
    y = py + 2 * j;
    return t < nxc * nyc;
}

// entries of the colours before q in the colour-ordered stencil array
template <int NX>
__device__ __forceinline__ int pad_colour_base(int q) {
    int b = 0;
    for (int c = 0; c < q; ++c) b += ((NX - ((c & 1) ^ 1) + 1) / 2) * ((NX - ((c >> 1) ^ 1) + 1) / 2);
    return b;
}

template <typename T, int NX>
__device__ __forceinline__ void pad_load_own(const T* __restrict__ cst, OwnPad<T>& on, int tid) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        int x, y;
        if (!pad_own<NX>(q, tid, x, y)) continue;
        const T* e = cst + (size_t)(pad_colour_base<NX>(q) + tid) * cst_pitch<T>();
        if constexpr (sizeof(T) == 4) {
            const float4 a = ((const float4*)e)[0], b = ((const float4*)e)[1], c = ((const float4*)e)[2];
            on.st[q][0] = a.x; on.st[q][1] = a.y; on.st[q][2] = a.z; on.st[q][3] = a.w;
            on.st[q][4] = b.x; on.st[q][5] = b.y; on.st[q][6] = b.z; on.st[q][7] = b.w;
            on.st[q][8] = c.x; on.rd[q] = c.y;
        } else {
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const double2 v = ((const double2*)e)[k];
                if (2 * k < 9) on.st[q][2 * k] = v.x;
                if (2 * k + 1 < 9) on.st[q][2 * k + 1] = v.y; else on.rd[q] = v.y;
            }
        }
    }
}

// f - (K u) at (x, y) on the padded grid, the centre left out when skip_c;
// the same terms in the same order as stencil_rest, plus exact zeros
template <typename T, int NX>
__device__ __forceinline__ T pad_rest(const T (&s9)[9], const T* u, int x, int y, T fval, bool skip_c) {
    constexpr int PW = NX + 2;
    const T* c = u + (y + 1) * PW + (x + 1);
    T acc = fval;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            if (skip_c && dx == 0 && dy == 0) continue;
            acc -= s9[(dy + 1) * 3 + (dx + 1)] * c[dy * PW + dx];
        }
    return acc;
}

template <typename T, int NX>
__device__ __forceinline__ void pad_smooth(const OwnPad<T>& on, T* u, const T* f, bool reverse, int nu, int tid) {
    constexpr int PW = NX + 2;
    for (int sweep = 0; sweep < nu; ++sweep)
#pragma unroll
        for (int qi = 0; qi < 4; ++qi) {
            const int q = reverse ? 3 - qi : qi;
            int x, y;
            if (pad_own<NX>(q, tid, x, y))
                u[(y + 1) * PW + x + 1] = pad_rest<T, NX>(on.st[q], u, x, y, f[y * NX + x], true) * on.rd[q];
            __syncthreads();
        }
}

// nu lexicographic sweeps (backward when reverse) on the padded grid by the
// calling wavefront (the first of the workgroup; the caller meets the others
// at a barrier afterwards): the fronts of k_lex_wave with the neighbour
// offsets compile-time immediates, the stencils and reciprocal diagonals
// loaded from global memory and f from LDS kLexAhead fronts ahead
template <typename T, int NX>
__device__ __forceinline__ void pad_lex(const T* __restrict__ sten, const T* __restrict__ rdiag, T* u, const T* f,
                                        bool reverse, int nu) {
    constexpr int PW = NX + 2;
    constexpr int ND = 3 * (NX - 1) + 1;
    const int y = threadIdx.x & 63;
    for (int sweep = 0; sweep < nu; ++sweep) {
        auto x_at = [&](int di) -> int { return (reverse ? ND - 1 - di : di) - 2 * y; };
        auto live = [&](int di, int x) { return di < ND && y < NX && x >= 0 && x < NX; };
        T st[kLexAhead][9], rd[kLexAhead], rf[kLexAhead];
        auto fetch = [&](int j, int di) {
            const int x = x_at(di);
            const int node = live(di, x) ? y * NX + x : 0;
#pragma unroll
            for (int t = 0; t < 9; ++t) st[j][t] = sten[(size_t)node * 9 + t];
            rd[j] = rdiag[node];
            rf[j] = f[node];
        };
#pragma unroll
        for (int j = 0; j < kLexAhead; ++j) fetch(j, j);
        for (int di0 = 0; di0 < ND; di0 += kLexAhead) {
#pragma unroll
            for (int j = 0; j < kLexAhead; ++j) {
                const int x = x_at(di0 + j);
                if (live(di0 + j, x)) {
                    T* b = u + y * PW + x;  // the south-west neighbour of (x, y)
                    T lo = rf[j] - st[j][0] * b[0], hi = st[j][6] * b[2 * PW];
                    lo -= st[j][1] * b[1];
                    hi += st[j][7] * b[2 * PW + 1];
                    lo -= st[j][2] * b[2];
                    hi += st[j][8] * b[2 * PW + 2];
                    lo -= st[j][3] * b[PW];
                    hi += st[j][5] * b[PW + 2];
                    b[PW + 1] = (lo - hi) * rd[j];
                }
                fetch(j, di0 + j + kLexAhead);
                wave_sync();
            }
        }
    }
}

// calls f(integral_constant<int, nx>) for the level sizes of the padded cycle
template <typename F>
__device__ __forceinline__ void with_pad_nx(int nx, F&& f) {
    switch (nx) {
        case 63: f(std::integral_constant<int, 63>{}); break;
        case 31: f(std::integral_constant<int, 31>{}); break;
        case 15: f(std::integral_constant<int, 15>{}); break;
        case 7: f(std::integral_constant<int, 7>{}); break;
        case 3: f(std::integral_constant<int, 3>{}); break;
        default: break;  // the host launches this kernel only for these sizes
    }
}

__host__ __device__ constexpr bool pad_cycle_size(int nx) { return nx == 63 || nx == 31 || nx == 15 || nx == 7 || nx == 3; }

template <typename T, bool LEX>
__global__ void __launch_bounds__(fused4_threads<T>()) k_vcycle_pad(PadLevels<T> pl, const double* __restrict__ kinv,
                                                                    const T* __restrict__ fin, int ldf,
                                                                    T* __restrict__ uout, int ldu, int nu1, int nu2) {
    extern __shared__ char smem_raw[];
    T* lds = (T*)smem_raw;
    SG_POISON_LDS(lds, pl.roff + pl.nx[0] * pl.nx[0]);
    const int col = blockIdx.x;
    const int L = pl.nlev - 1;
    const int nx0 = pl.nx[0], N0 = nx0 * nx0;
    // zero every padded u: the border stays zero, the interiors are the zero initial guesses
    for (int l = 0; l <= L; ++l) {
        const int pw = pl.nx[l] + 2;
        T* u = lds + pl.uoff[l];
        for (int i = threadIdx.x; i < pw * pw; i += blockDim.x) u[i] = T(0);
    }
    {
        T* f0 = lds + pl.foff[0];
        for (int i = threadIdx.x; i < N0; i += blockDim.x) f0[i] = fin[(size_t)i * ldf + col];
    }
    __syncthreads();
    T* r = lds + pl.roff;
    OwnPad<T> on;
    for (int l = 0; l < L; ++l) {
        with_pad_nx(pl.nx[l], [&](auto knx) __attribute__((always_inline)) {
            constexpr int NX = decltype(knx)::value;
            constexpr int NXC = (NX - 1) / 2;
            // an opaque copy of the thread index keeps each level's per-thread
            // addresses inside its visit (hoisted for every level size they
            // would not fit in registers)
            int tid = threadIdx.x;
            __asm__ volatile("" : "+v"(tid));
            T* u = lds + pl.uoff[l];
            const T* f = lds + pl.foff[l];
            pad_load_own<T, NX>(pl.cst[l], on, tid);
            if constexpr (LEX) {
                if (threadIdx.x < 64) pad_lex<T, NX>(pl.sten[l], pl.rdiag[l], u, f, false, nu1);
                __syncthreads();
            } else {
                pad_smooth<T, NX>(on, u, f, false, nu1, tid);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                int x, y;
                if (pad_own<NX>(q, tid, x, y)) r[y * NX + x] = pad_rest<T, NX>(on.st[q], u, x, y, f[y * NX + x], false);
            }
            __syncthreads();
            T* fc = lds + pl.foff[l + 1];
            for (int node = tid; node < NXC * NXC; node += blockDim.x) {
                const int Y = node / NXC, X = node - Y * NXC;
                fc[node] = restrict_value<T>([&](int xx, int yy) { return r[yy * NX + xx]; }, X, Y, pl.p1 != 0);
            }
            __syncthreads();
        });
    }
    {
        // coarsest grid: u = K^{-1} f in double (as coarsest_solve), written into the padded layout
        const int nxL = pl.nx[L], N = nxL * nxL;
        const T* f = lds + pl.foff[L];
        T* u = lds + pl.uoff[L];
        int G = 1;
        while (G < 64 && 2 * G * N <= (int)blockDim.x) G *= 2;
        const int rows = (int)blockDim.x / G;
        const int g = threadIdx.x % G;
        for (int i0 = 0; i0 < N; i0 += rows) {  // uniform trip count
            const int i = i0 + (int)threadIdx.x / G;
            double acc = 0.0;
            if (i < N) {
                const double* row = kinv + (size_t)i * N;
                for (int j = g; j < N; j += G) acc = fma(row[j], (double)f[j], acc);
            }
            for (int o = G / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);  // groups lie inside a wavefront
            if (i < N && g == 0) {
                const int y = i / nxL, x = i - y * nxL;
                u[(y + 1) * (nxL + 2) + x + 1] = (T)acc;
            }
        }
        __syncthreads();
    }
    for (int l = L - 1; l >= 0; --l) {
        with_pad_nx(pl.nx[l], [&](auto knx) __attribute__((always_inline)) {
            constexpr int NX = decltype(knx)::value;
            constexpr int PW = NX + 2;
            constexpr int NXC = (NX - 1) / 2;
            int tid = threadIdx.x;
            __asm__ volatile("" : "+v"(tid));
            T* u = lds + pl.uoff[l];
            const T* f = lds + pl.foff[l];
            const T* ec = lds + pl.uoff[l + 1];
            pad_load_own<T, NX>(pl.cst[l], on, tid);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                int x, y;
                if (pad_own<NX>(q, tid, x, y))
                    u[(y + 1) * PW + x + 1] += prolong_value<T>(
                        [&](int X, int Y) { return ec[(Y + 1) * (NXC + 2) + X + 1]; }, NXC, x, y, pl.p1 != 0);
            }
            __syncthreads();
            if constexpr (LEX) {
                if (threadIdx.x < 64) pad_lex<T, NX>(pl.sten[l], pl.rdiag[l], u, f, true, nu2);
                __syncthreads();
            } else {
                pad_smooth<T, NX>(on, u, f, true, nu2, tid);
            }
        });
    }
    {
        const T* u0 = lds + pl.uoff[0];
        for (int i = threadIdx.x; i < N0; i += blockDim.x) {
            const int y = i / nx0, x = i - y * nx0;
            uout[(size_t)i * ldu + col] = u0[(y + 1) * (nx0 + 2) + x + 1];
        }
    }
}

inline dim3 grid2(int rows, int width, const Tile& tl) {
    return dim3((rows + tl.ty - 1) / tl.ty, (width + tl.tx - 1) / tl.tx);
}

template <typename T>
struct LevelPtr;
template <>
struct LevelPtr<double> {
    static double* u2(Level& l) { return l.w64; }
    static double* u(Level& l) { return l.u64; }
    static double* f(Level& l) { return l.f64; }
    static double* r(Level& l) { return l.r64; }
    static const double* s(const Level& l) { return l.sten64; }
    static const double* rd(const Level& l) { return l.rdiag64; }
    static const double* cst(const Level& l) { return l.cst64; }
    static const double* stp(const Level& l) { return l.stp64; }
};
template <>
struct LevelPtr<float> {
    static float* u2(Level& l) { return l.w32; }
    static float* u(Level& l) { return l.u32; }
    static float* f(Level& l) { return l.f32; }
    static float* r(Level& l) { return l.r32; }
    static const float* s(const Level& l) { return l.sten32; }
    static const float* rd(const Level& l) { return l.rdiag32; }
    static const float* cst(const Level& l) { return l.cst32; }
    static const float* stp(const Level& l) { return l.stp32; }
};

template <typename T>
void launch_gs(const Tile& tl, dim3 g, hipStream_t st, const T* sten, const T* rdiag, T* u, int ldu, const T* f,
               int ldf, T* out,
               int ldo, int nx, int width, int rb, int q, int nxc, int nyc, int first) {
    if (tl.tx == 64)
        hipLaunchKernelGGL((k_gs<T, true>), g, dim3(tl.tx, tl.ty), 0, st, sten, rdiag, u, ldu, f, ldf, out, ldo, nx,
                           width, rb, q, nxc, nyc, first);
    else
        hipLaunchKernelGGL((k_gs<T, false>), g, dim3(tl.tx, tl.ty), 0, st, sten, rdiag, u, ldu, f, ldf, out, ldo, nx,
                           width, rb, q, nxc, nyc, first);
}

template <typename T>
void smooth(sg_ctx* c, int l, T* u, int ldu, const T* f, int ldf, int width, bool reverse, const Tile& tl,
            bool first) {
    Level& lv = c->levels[l];
    const int nx = lv.nx;
    if (c->opt.colour_mode == SG_COLOUR_LEX) {
        if (nx <= kLexWaveMaxNx)
            hipLaunchKernelGGL(k_lex_wave<T>, dim3(width), dim3(64), (size_t)(nx + 2) * (nx + 2) * sizeof(T), c->stream,
                               LevelPtr<T>::s(lv), LevelPtr<T>::rd(lv), u, ldu, f, ldf, nx, reverse ? 1 : 0,
                               first ? 1 : 0);
        else
            hipLaunchKernelGGL(k_gs_lex<T>, dim3(width), dim3(256), 0, c->stream, LevelPtr<T>::s(lv),
                               LevelPtr<T>::rd(lv), u, ldu, f, ldf, nx, reverse ? 1 : 0, first ? 1 : 0);
        return;
    }
    const bool rb = c->opt.colour_mode == SG_COLOUR_RB;
    const int ncol = rb ? 2 : 4;
    for (int qi = 0; qi < ncol; ++qi) {
        const int q = reverse ? ncol - 1 - qi : qi;
        if (!rb) {
            const int px = (q & 1) ^ 1, py = (q >> 1) ^ 1;
            const int nxc = (nx - px + 1) / 2, nyc = (nx - py + 1) / 2;
            launch_gs<T>(tl, grid2(nxc * nyc, width, tl), c->stream, LevelPtr<T>::s(lv), LevelPtr<T>::rd(lv), u, ldu,
                         f, ldf, nullptr, 0,
                         nx, width, 0, q, nxc, nyc, first ? 1 : 0);
        } else {
            const int nxc = (nx + 1) / 2, nyc = nx;
            T* stage = LevelPtr<T>::r(lv);  // residual buffer is free during smoothing
            launch_gs<T>(tl, grid2(nxc * nyc, width, tl), c->stream, LevelPtr<T>::s(lv), LevelPtr<T>::rd(lv), u, ldu,
                         f, ldf, stage,
                         width, nx, width, 1, q, nxc, nyc, first ? 1 : 0);
            hipLaunchKernelGGL(k_copy_colour<T>, grid2(nxc * nyc, width, tl), dim3(tl.tx, tl.ty), 0, c->stream,
                               (const T*)stage, width, u, ldu, nx, width, q, nxc, nyc);
        }
    }
}

// A walk of a long segment per workgroup keeps the data of a segment in
// flight, but on a coarse grid it leaves too few wavefronts to fill the chip:
// below this many wavefronts the short-segment form of a walking kernel runs.
constexpr int kMinWalkWaves = 2048;

// nu four-colour sweeps by row phases with ping-pong between u and the
// level's second buffer; returns with the result in uout (u when null; the
// last sweep writes uout directly when it is a third buffer).  zero_start:
// u holds the zero initial guess (not read).
template <typename T>
void row_sweeps(sg_ctx* c, int l, T* u, int ldu, const T* f, int ldf, int width, bool reverse, int nu,
                bool zero_start, T* uout = nullptr, int lduo = 0) {
    if (!uout) {
        uout = u;
        lduo = ldu;
    }
    Level& lv = c->levels[l];
    const int nx = lv.nx;
    T* alt = LevelPtr<T>::u2(lv);
    const int lda_alt = width;
    const int nws = (width + 63) / 64;
    const bool shortw = (long)((nx + 1) / 2) * ((nx + kRowSeg - 1) / kRowSeg) * nws < kMinWalkWaves;
    const int seg = shortw ? kRowSegShort : kRowSeg;
    const int nseg = (nx + seg - 1) / seg;
    T* src = u;
    int lds = ldu;
    T* dst = alt;
    int ldd = lda_alt;
    for (int sw = 0; sw < nu; ++sw) {
        const bool own_zero = zero_start && sw == 0;
        if (sw == nu - 1 && uout != u && uout != src) {
            dst = uout;
            ldd = lduo;
        }
        // forward: rows y odd (fx = 1), then y even (fx = 1); backward: y even (fx = 0), then y odd (fx = 0)
        const int py1 = reverse ? 0 : 1, fx = reverse ? 0 : 1;
        if (width >= 32 && own_zero) {
            // the first sweep from the zero start: both row phases in one launch (only f is read)
            const int p1 = 1 - py1;
            const int nrows1 = (nx - p1 + 1) / 2;
            auto go = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(nrows1 * nseg), dim3(64 * nws), 0, c->stream, LevelPtr<T>::stp(lv), f,
                                   ldf, dst, ldd, nx, width, p1, fx, nseg, nrows1);
            };
            shortw ? go(k_gs_sweep0<T, kRowSegShort>) : go(k_gs_sweep0<T, kRowSeg>);
        } else if (width >= 32) {
            for (int ph = 0; ph < 2; ++ph) {
                const int py = ph == 0 ? py1 : 1 - py1;
                const int nrows = (nx - py + 1) / 2;
                const T* vsrc = ph == 0 ? src : dst;
                const int ldv = ph == 0 ? lds : ldd;
                hipLaunchKernelGGL((shortw ? k_gs_rows<T, kRowSegShort> : k_gs_rows<T, kRowSeg>), dim3(nrows * nseg),
                                   dim3(64 * nws), 0, c->stream, LevelPtr<T>::s(lv), LevelPtr<T>::rd(lv),
                                   (const T*)src, lds, vsrc, ldv, f, ldf, dst, ldd, nx, width, py, fx, nseg, nrows);
            }
        } else {
            for (int ph = 0; ph < 2; ++ph) {
                const int py = ph == 0 ? py1 : 1 - py1;
                const int nrows = (nx - py + 1) / 2;
                const T* vsrc = ph == 0 ? src : dst;
                const int ldv = ph == 0 ? lds : ldd;
                const int vzero = (ph == 0 && own_zero) ? 1 : 0;
                const int npairs = fx ? (nx - 1) / 2 + 1 : nx / 2 + 1;  // pairs (S(s), F(s+1)) covering the row
                // lanes per pair: W rounded up to a power of two in float, W itself in double
                // (measured faster each way at 21 modes)
                int wpad = width;
                if (sizeof(T) == 4)
                    for (wpad = 1; wpad < width;) wpad <<= 1;
                const long lanes = (long)nrows * npairs * wpad;
                const int nblk = (int)((lanes + 255) / 256);
                if (own_zero)
                    hipLaunchKernelGGL((k_gs_rows_narrow<T, true>), dim3(nblk), dim3(256), 0, c->stream,
                                       LevelPtr<T>::stp(lv), (const T*)src, lds, vsrc, ldv, f, ldf,
                                       dst, ldd, nx, width, wpad, py, fx, vzero, npairs, nrows);
                else
                    hipLaunchKernelGGL((k_gs_rows_narrow<T, false>), dim3(nblk), dim3(256), 0, c->stream,
                                       LevelPtr<T>::stp(lv), (const T*)src, lds, vsrc, ldv, f, ldf,
                                       dst, ldd, nx, width, wpad, py, fx, vzero, npairs, nrows);
            }
        }
        std::swap(src, dst);
        std::swap(lds, ldd);
    }
    if (src != uout) {
        // the result is in another buffer (an odd number of sweeps, or none)
        const Tile tl = tile_for(width);
        hipLaunchKernelGGL((k_cast<T, T>), grid2(lv.N, width, tl), dim3(tl.tx, tl.ty), 0, c->stream, (const T*)src,
                           lds, uout, lduo, lv.N, width);
    }
}

template <typename T>
bool use_row_sweeps(const sg_ctx* c, int width) {
    (void)width;
    return c->opt.colour_mode == SG_COLOUR_FOUR;
}

// block widths the tile cycle takes: a workgroup per (tile, mode), so the
// launch holds width times the tiles; wider blocks keep the row-phase kernels
constexpr int kTileMaxWidth = 8;   // every level with at most kTileMaxWorkgroups (tile, mode) pairs
constexpr int kTileMaxWorkgroups = 1024;  // two rounds of the chip: each workgroup is latency-bound
constexpr int kTileMidWidth = 32;  // on grids of at most kTileMidNx nodes per side
constexpr int kTileMidNx = 127;

template <typename T>
void launch_tile(bool down, int width, int ntiles, hipStream_t st, const T* stp, const T* f, int ldf, const T* ui,
                 int ldi, const T* ec, int ldc, T* uo, int ldo, T* fc, int ldfc, int nx, int nu, int ntx, int p1) {
    if (down)
        hipLaunchKernelGGL(k_cycle1_down<T>, dim3(ntiles * width), dim3(1024), 0, st, stp, f, ldf, uo, ldo, fc, ldfc,
                           nx, nu, ntx, ntiles, p1);
    else
        hipLaunchKernelGGL(k_cycle1_up<T>, dim3(ntiles * width), dim3(1024), 0, st, stp, f, ldf, ui, ldi, ec, ldc, uo,
                           ldo, nx, nu, ntx, ntiles, p1);
}

template <typename T>
int vcycle_t(sg_ctx* c, const T* f0, int ldf0, T* u0, int ldu0, int width) {
    const Tile tl = tile_for(width);
    const int L = (int)c->levels.size() - 1;
    const bool p1 = c->hs.disc == SG_DISC_P1;  // transfer of the P1 triangulation
    // first level handled by the fused LDS kernel (-1: none fits, coarsest solved by k_coarse)
    int Lc = -1;
    for (int l = 0; l <= L; ++l)
        if (c->levels[l].nx <= fused_nx_max<T>()) { Lc = l; break; }
    const int Ltop = Lc >= 0 ? Lc : L;  // levels above Ltop are cycled by separate launches
    // with row sweeps the finest level iterates in its own compact block (row
    // stride = width) and only the last post-smoothing sweep writes u0, whose
    // rows may be strided (a slice of a wider block): the stencil reads of the
    // cycle then touch W contiguous values per node, not one per cache line
    const bool compact0 = use_row_sweeps<T>(c, width) && Ltop > 0;
    T* const uc0 = compact0 ? LevelPtr<T>::u(c->levels[0]) : u0;
    const int ldc0 = compact0 ? width : ldu0;
    auto fptr = [&](int l) -> const T* { return l == 0 ? f0 : LevelPtr<T>::f(c->levels[l]); };
    auto fld = [&](int l) { return l == 0 ? ldf0 : width; };
    auto uptr = [&](int l) -> T* { return l == 0 ? uc0 : LevelPtr<T>::u(c->levels[l]); };
    auto uld = [&](int l) { return l == 0 ? ldc0 : width; };
    // the coarse part: the fused LDS cycle from level Lc, or the coarsest solve at level L
    auto coarse_part = [&]() -> int {
        const bool lex = c->opt.colour_mode == SG_COLOUR_LEX;
        bool pad = Lc >= 0 && (c->opt.colour_mode == SG_COLOUR_FOUR || lex) && L - Lc + 1 <= kMaxFusedLevels;
        for (int l = Lc; pad && l < L; ++l)
            pad = pad_cycle_size(c->levels[l].nx) && LevelPtr<T>::cst(c->levels[l]) != nullptr;
        if (pad) {
            PadLevels<T> pl{};
            pl.nlev = L - Lc + 1;
            pl.p1 = p1;
            int off = 0;
            for (int i = 0; i < pl.nlev; ++i) {
                const Level& lv = c->levels[Lc + i];
                pl.nx[i] = lv.nx;
                pl.uoff[i] = off;
                off += (lv.nx + 2) * (lv.nx + 2);
                pl.foff[i] = off;
                off += lv.N;
                pl.cst[i] = LevelPtr<T>::cst(lv);
                pl.sten[i] = LevelPtr<T>::s(lv);
                pl.rdiag[i] = LevelPtr<T>::rd(lv);
            }
            pl.roff = off;
            off += c->levels[Lc].N;
            if (lex)
                hipLaunchKernelGGL((k_vcycle_pad<T, true>), dim3(width), dim3(fused4_threads<T>()), (size_t)off * sizeof(T),
                                   c->stream, pl, (const double*)c->kinv, fptr(Lc), fld(Lc), uptr(Lc), uld(Lc),
                                   c->opt.nu1, c->opt.nu2);
            else
                hipLaunchKernelGGL((k_vcycle_pad<T, false>), dim3(width), dim3(fused4_threads<T>()), (size_t)off * sizeof(T),
                                   c->stream, pl, (const double*)c->kinv, fptr(Lc), fld(Lc), uptr(Lc), uld(Lc),
                                   c->opt.nu1, c->opt.nu2);
        } else if (Lc >= 0) {
            FusedLevels<T> fl{};
            fl.nlev = L - Lc + 1;
            if (fl.nlev > kMaxFusedLevels) {
                set_error("vcycle: too many coarse levels");
                return SG_EINVAL;
            }
            int off = 0;
            for (int i = 0; i < fl.nlev; ++i) {
                const Level& lv = c->levels[Lc + i];
                fl.nx[i] = lv.nx;
                fl.off[i] = off;
                fl.sten[i] = LevelPtr<T>::s(lv);
                fl.rdiag[i] = LevelPtr<T>::rd(lv);
                off += 2 * lv.N;
            }
            fl.roff = off;
            fl.p1 = p1;
            off += c->levels[Lc].N;
            if (c->opt.colour_mode == SG_COLOUR_FOUR)
                hipLaunchKernelGGL(k_vcycle_fused4<T>, dim3(width), dim3(fused4_threads<T>()), (size_t)off * sizeof(T),
                                   c->stream, fl,
                                   (const double*)c->kinv, fptr(Lc), fld(Lc), uptr(Lc), uld(Lc), c->opt.nu1, c->opt.nu2);
            else
                hipLaunchKernelGGL(k_vcycle_fused<T>, dim3(width), dim3(512), (size_t)off * sizeof(T), c->stream, fl,
                                   (const double*)c->kinv, fptr(Lc), fld(Lc), uptr(Lc), uld(Lc), c->opt.nu1, c->opt.nu2,
                                   c->opt.colour_mode == SG_COLOUR_LEX ? 2 : 1);
        } else {
            Level& lc = c->levels[L];
            hipLaunchKernelGGL(k_coarse<T>, dim3(width), dim3(256), (size_t)lc.N * sizeof(double), c->stream, c->kinv,
                               fptr(L), fld(L), uptr(L), uld(L), lc.N);
        }
        return SG_OK;
    };
    // Levels lt .. Ltop-1 are cycled by tiles (two launches per level): for
    // blocks of at most kTileMaxWidth modes every level with at most
    // kTileMaxWorkgroups (tile, mode) pairs, for blocks of at most kTileMidWidth
    // modes the grids of at most kTileMidNx nodes per side.  A
    // tile level keeps its smoothed values in uptr(l) and writes its corrected
    // ones to the level's second buffer (u0 on the finest level).
    auto tiles = [&](const Level& lv, int& ntx) {
        const int nxc = (lv.nx - 1) / 2;
        ntx = (nxc + kTileCX - 1) / kTileCX;
        return ntx * ((nxc + kTileCY - 1) / kTileCY);
    };
    int lt = Ltop;
    if (c->opt.colour_mode == SG_COLOUR_FOUR && c->opt.nu1 <= kTileMaxNu && c->opt.nu2 <= kTileMaxNu)
        for (int l = 0; l < Ltop; ++l) {
            int ntx;
            const long wgs = (long)tiles(c->levels[l], ntx) * width;
            if ((width <= kTileMaxWidth && wgs <= kTileMaxWorkgroups) ||
                (width <= kTileMidWidth && c->levels[l].nx <= kTileMidNx)) {
                lt = l;
                break;
            }
        }
    // the corrected values of level l, which the prolongation of level l - 1 reads
    auto sol = [&](int l) -> const T* { return l >= lt && l < Ltop ? LevelPtr<T>::u2(c->levels[l]) : uptr(l); };
    for (int l = 0; l < lt; ++l) {
        Level& lv = c->levels[l];
        T* u = uptr(l);
        // zero initial guess: the first sweep skips not-yet-updated neighbours, so u needs no clearing
        if (c->opt.nu1 == 0)
            hipLaunchKernelGGL(k_fill<T>, grid2(lv.N, width, tl), dim3(tl.tx, tl.ty), 0, c->stream, u, uld(l), lv.N,
                               width);
        if (use_row_sweeps<T>(c, width))
            row_sweeps<T>(c, l, u, uld(l), fptr(l), fld(l), width, false, c->opt.nu1, true);
        else
            for (int s = 0; s < c->opt.nu1; ++s) smooth<T>(c, l, u, uld(l), fptr(l), fld(l), width, false, tl, s == 0);
        Level& lc = c->levels[l + 1];
        if (width >= kWalkMinWidth) {
            const int nws = (width + 63) / 64;
            const bool shortw = (long)lc.nx * ((lc.nx + kRrSeg - 1) / kRrSeg) * nws < kMinWalkWaves;
            const int seg = shortw ? kRrSegShort : kRrSeg;
            const int nseg = (lc.nx + seg - 1) / seg;
            auto rr = shortw ? (p1 ? k_resid_restrict<T, kRrSegShort, true> : k_resid_restrict<T, kRrSegShort, false>)
                             : (p1 ? k_resid_restrict<T, kRrSeg, true> : k_resid_restrict<T, kRrSeg, false>);
            hipLaunchKernelGGL(rr, dim3(lc.nx * nseg), dim3(64 * nws), 0, c->stream, LevelPtr<T>::s(lv), (const T*)u,
                               uld(l), fptr(l), fld(l), LevelPtr<T>::f(lc), width, lc.nx, width, nseg);
        } else {
            T* r = LevelPtr<T>::r(lv);
            if (tl.tx == 64)
                hipLaunchKernelGGL((k_residual<T, true>), grid2(lv.N, width, tl), dim3(tl.tx, tl.ty), 0, c->stream,
                                   LevelPtr<T>::s(lv), (const T*)u, uld(l), fptr(l), fld(l), r, width, lv.nx, width);
            else
                hipLaunchKernelGGL((k_residual<T, false>), grid2(lv.N, width, tl), dim3(tl.tx, tl.ty), 0, c->stream,
                                   LevelPtr<T>::s(lv), (const T*)u, uld(l), fptr(l), fld(l), r, width, lv.nx, width);
            hipLaunchKernelGGL(k_restrict<T>, grid2(lc.N, width, tl), dim3(tl.tx, tl.ty), 0, c->stream,
                               (const T*)r, width, LevelPtr<T>::f(lc), width, lc.nx, width, (int)p1);
        }
    }
    for (int l = lt; l < Ltop; ++l) {
        Level& lv = c->levels[l];
        int ntx;
        const int nb = tiles(lv, ntx);
        launch_tile<T>(true, width, nb, c->stream, LevelPtr<T>::stp(lv), fptr(l), fld(l), nullptr, 0, nullptr, 0,
                       uptr(l), uld(l), LevelPtr<T>::f(c->levels[l + 1]), width, lv.nx, c->opt.nu1, ntx, (int)p1);
    }
    if (int rc = coarse_part()) return rc;
    for (int l = Ltop - 1; l >= lt; --l) {
        Level& lv = c->levels[l];
        int ntx;
        const int nb = tiles(lv, ntx);
        T* out = l == 0 ? u0 : LevelPtr<T>::u2(lv);
        launch_tile<T>(false, width, nb, c->stream, LevelPtr<T>::stp(lv), fptr(l), fld(l), uptr(l), uld(l), sol(l + 1),
                       width, out, l == 0 ? ldu0 : width, nullptr, 0, lv.nx, c->opt.nu2, ntx, (int)p1);
    }
    for (int l = lt - 1; l >= 0; --l) {
        Level& lv = c->levels[l];
        T* u = uptr(l);
        if (width >= kWalkMinWidth) {
            const int nws = (width + 63) / 64;
            const bool shortw = (long)lv.nx * ((lv.nx + kPrSeg - 1) / kPrSeg) * nws < kMinWalkWaves;
            const int seg = shortw ? kPrSegShort : kPrSeg;
            const int nseg = (lv.nx + seg - 1) / seg;
            auto pr = shortw ? (p1 ? k_prolong_rows<T, kPrSegShort, true> : k_prolong_rows<T, kPrSegShort, false>)
                             : (p1 ? k_prolong_rows<T, kPrSeg, true> : k_prolong_rows<T, kPrSeg, false>);
            hipLaunchKernelGGL(pr, dim3(lv.nx * nseg),
                               dim3(64 * nws), 0, c->stream, sol(l + 1), width, u,
                               uld(l), lv.nx, width, nseg);
        } else if (tl.tx == 64)
            hipLaunchKernelGGL((k_prolong_add<T, true>), grid2(lv.N, width, tl), dim3(tl.tx, tl.ty), 0, c->stream,
                               sol(l + 1), width, u, uld(l), lv.nx, width, (int)p1);
        else
            hipLaunchKernelGGL((k_prolong_add<T, false>), grid2(lv.N, width, tl), dim3(tl.tx, tl.ty), 0, c->stream,
                               sol(l + 1), width, u, uld(l), lv.nx, width, (int)p1);
        if (use_row_sweeps<T>(c, width))
            row_sweeps<T>(c, l, u, uld(l), fptr(l), fld(l), width, true, c->opt.nu2, false, l == 0 ? u0 : nullptr,
                          l == 0 ? ldu0 : 0);
        else
            for (int s = 0; s < c->opt.nu2; ++s) smooth<T>(c, l, u, uld(l), fptr(l), fld(l), width, true, tl, false);
    }
    return hipGetLastError() == hipSuccess ? SG_OK : SG_EHIP;
}

}  // namespace

int launch_vcycle(sg_ctx* c, const void* f, int ldf, void* u, int ldu, int width, int is_float) {
    int rc = is_float ? vcycle_t<float>(c, (const float*)f, ldf, (float*)u, ldu, width)
                      : vcycle_t<double>(c, (const double*)f, ldf, (double*)u, ldu, width);
    if (rc != SG_OK) set_error("vcycle: kernel launch failed");
    return rc;
}

int launch_cast(hipStream_t s, const void* src, int src_float, int lds, void* dst, int dst_float, int ldd, int rows,
                int width) {
    const Tile tl = tile_for(width);
    if (src_float && dst_float)
        hipLaunchKernelGGL((k_cast<float, float>), grid2(rows, width, tl), dim3(tl.tx, tl.ty), 0, s,
                           (const float*)src, lds, (float*)dst, ldd, rows, width);
    else if (src_float)
        hipLaunchKernelGGL((k_cast<float, double>), grid2(rows, width, tl), dim3(tl.tx, tl.ty), 0, s,
                           (const float*)src, lds, (double*)dst, ldd, rows, width);
    else if (dst_float)
        hipLaunchKernelGGL((k_cast<double, float>), grid2(rows, width, tl), dim3(tl.tx, tl.ty), 0, s,
                           (const double*)src, lds, (float*)dst, ldd, rows, width);
    else
        hipLaunchKernelGGL((k_cast<double, double>), grid2(rows, width, tl), dim3(tl.tx, tl.ty), 0, s,
                           (const double*)src, lds, (double*)dst, ldd, rows, width);
    return hipGetLastError() == hipSuccess ? SG_OK : SG_EHIP;
}

int launch_axpy_cols(hipStream_t s, const void* src, int is_float, int lds, void* dst, int ldd, int rows, int width,
                     double a) {
    const Tile tl = tile_for(width);
    if (is_float)
        hipLaunchKernelGGL(k_axpy_cols<float>, grid2(rows, width, tl), dim3(tl.tx, tl.ty), 0, s, (const float*)src, lds,
                           (float*)dst, ldd, rows, width, (float)a);
    else
        hipLaunchKernelGGL(k_axpy_cols<double>, grid2(rows, width, tl), dim3(tl.tx, tl.ty), 0, s, (const double*)src,
                           lds, (double*)dst, ldd, rows, width, a);
    return hipGetLastError() == hipSuccess ? SG_OK : SG_EHIP;
}

int launch_fill(hipStream_t s, void* dst, int is_float, int ld, int rows, int width) {
    const Tile tl = tile_for(width);
    if (is_float)
        hipLaunchKernelGGL(k_fill<float>, grid2(rows, width, tl), dim3(tl.tx, tl.ty), 0, s, (float*)dst, ld, rows,
                           width);
    else
        hipLaunchKernelGGL(k_fill<double>, grid2(rows, width, tl), dim3(tl.tx, tl.ty), 0, s, (double*)dst, ld,
                           rows, width);
    return hipGetLastError() == hipSuccess ? SG_OK : SG_EHIP;
}

int launch_restrict_block(sg_ctx* c, int l, const double* r, int ldr, double* fc, int ldc, int width) {
    const Tile tl = tile_for(width);
    const Level& lc = c->levels[l + 1];
    hipLaunchKernelGGL(k_restrict<double>, grid2(lc.N, width, tl), dim3(tl.tx, tl.ty), 0, c->stream, r, ldr, fc, ldc,
                       lc.nx, width, c->hs.disc == SG_DISC_P1 ? 1 : 0);
    return hipGetLastError() == hipSuccess ? SG_OK : SG_EHIP;
}

int launch_prolong_block(sg_ctx* c, int l, const double* ec, int ldc, double* u, int ldu, int width) {
    const Tile tl = tile_for(width);
    const Level& lv = c->levels[l];
    const int p1 = c->hs.disc == SG_DISC_P1 ? 1 : 0;
    if (tl.tx == 64)
        hipLaunchKernelGGL((k_prolong_add<double, true>), grid2(lv.N, width, tl), dim3(tl.tx, tl.ty), 0, c->stream,
                           ec, ldc, u, ldu, lv.nx, width, p1);
    else
        hipLaunchKernelGGL((k_prolong_add<double, false>), grid2(lv.N, width, tl), dim3(tl.tx, tl.ty), 0, c->stream,
                           ec, ldc, u, ldu, lv.nx, width, p1);
    return hipGetLastError() == hipSuccess ? SG_OK : SG_EHIP;
}

int launch_lex_sweep(sg_ctx* c, int l, double* u, int ldu, const double* f, int ldf, int width, int reverse) {
    const Level& lv = c->levels[l];
    if (lv.nx <= kLexWaveMaxNx)
        hipLaunchKernelGGL(k_lex_wave<double>, dim3(width), dim3(64), (size_t)(lv.nx + 2) * (lv.nx + 2) * sizeof(double),
                           c->stream,
                           lv.sten64, lv.rdiag64, u, ldu, f, ldf, lv.nx, reverse, 0);
    else
        hipLaunchKernelGGL(k_gs_lex<double>, dim3(width), dim3(256), 0, c->stream, lv.sten64, lv.rdiag64, u, ldu, f,
                           ldf, lv.nx, reverse, 0);
    return hipGetLastError() == hipSuccess ? SG_OK : SG_EHIP;
}

}  // namespace sg
