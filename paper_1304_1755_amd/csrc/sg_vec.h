// Launchers of the vector, reduction, QoI and adjoint kernels (sg_vec.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>

namespace sg {

constexpr int kRedBlocks = 1024;  // fixed reduction grid: deterministic partial sums
constexpr int kDc = 16;           // basis vectors per orthogonalization pass
constexpr int kDcLd = 2 * kDc + 2;  // outputs per chunk of vec_dots2

// per-chunk coefficients of the orthogonalization update pass (kernel argument)
struct DcCoef {
    double a[kDc];
    double c[kDc];
    double alpha, gamma;
};

// Arnoldi passes with delayed reorthogonalization (chunks of kDc basis vectors).
// vec_dots2: out[34 ch + i] = Q_{16 ch + i} . u, out[34 ch + 16 + i] = Q_{16 ch + i} . w,
// out[34 ch + 32] = u . u, out[34 ch + 33] = u . w  (ch = 0 .. ceil(nv / 16) - 1).
hipError_t vec_dots2(hipStream_t s, const double* Q, size_t stride, int nv, const double* u, const double* w,
                     size_t len, double* partial, double* out);
// vec_update2: u <- alpha uin - sum_i a[i] Q_i, wout <- w - gamma uin - sum_i c[i] Q_i (host a, c),
// out_sq = |wout|^2 when partial_sq and out_sq are given; uin may be u (in place), else 16-byte aligned.
hipError_t vec_update2(hipStream_t s, const double* Q, size_t stride, int nv, const double* a, const double* c,
                       double alpha, double gamma, const double* uin, double* u, const double* w, double* wout,
                       size_t len, double* partial_sq, double* out_sq);
hipError_t vec_dot(hipStream_t s, const double* a, const double* b, size_t len, double* partial, double* out);
hipError_t vec_scale(hipStream_t s, const double* src, double a, double* dst, size_t len);
// x = (accumulate ? x : 0) + sum_i y[i] Z_i  (y on the device)
hipError_t vec_combine(hipStream_t s, const void* Z, int z_float, size_t stride, int nz, const double* y, double* x,
                       size_t len, bool accumulate);
hipError_t vec_axpy_sq(hipStream_t s, double a, const double* x, double* y, size_t len, double* partial,
                       double* out_sq);
hipError_t vec_axpy(hipStream_t s, double a, const double* x, double* y, size_t len);
hipError_t vec_xpby(hipStream_t s, const double* z, double b, double* p, size_t len);
hipError_t vec_rhs(hipStream_t s, double* F, int N, int P, double h2);
hipError_t vec_qoi(hipStream_t s, const double* U, const double* wS, int N, int P, double* partial, double* q,
                   double* J, double* coef);
// the allocation-free QoI: capacity of its per-device scratch array (doubles), and the
// array's device address on `device` (looked up once per device, that device current)
constexpr size_t kQoiScratchDoubles = (size_t)kRedBlocks * 256 + 256;
hipError_t qoi_scratch_address(int device, double** out);
hipError_t vec_adj_rhs(hipStream_t s, const double* wS, const double* coef, int N, int P, double* g);
hipError_t vec_grad_cells(hipStream_t s, int nslot, const double* U, const double* L, int n, int P, int m,
                          const uint32_t* toff, const double* tcoef, double* dc);
hipError_t vec_grad_params(hipStream_t s, const double* dc, const double* kl, const double* amps, double sigma, int n,
                           int m, double* partial, double* Tk, double* out_params, double* out_a0);

}  // namespace sg
