// Internal declarations shared by the host setup, the kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sgbt.h"

namespace sg {

constexpr int kMaxM = 8;
constexpr int kMaxSlots = 4;  // modes per node handled by one wave: up to 4 x 64 = 256
constexpr int kMaxRestart = 64;
constexpr int kLdsCycleMaxNx = 63;  // largest grid (interior nodes per side) the fused coarse cycle takes

void set_error(const std::string& msg);

#define SG_HIP_CHECK(expr)                                                          \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess) {                                                     \
            ::sg::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));      \
            return SG_EHIP;                                                         \
        }                                                                           \
    } while (0)

// Debug build (-DSG_LDS_POISON, built beside the library as libsgbt_poison.so):
// every kernel that stages data in LDS tiles first fills its LDS with quiet
// NaNs and meets at a barrier, so that a value read before it was written
// turns the kernel's output into NaN.  Normal builds compile it to nothing.
#ifdef SG_LDS_POISON
template <typename T>
__device__ inline void lds_poison(T* p, long count) {
    const int nt = blockDim.x * blockDim.y * blockDim.z;
    const int t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    for (long i = t; i < count; i += nt) p[i] = (T)__builtin_nan("");
    __syncthreads();
}
#define SG_POISON_LDS(ptr, count) ::sg::lds_poison((ptr), (long)(count))
#else
#define SG_POISON_LDS(ptr, count) ((void)0)
#endif

// ---------------------------------------------------------------- host setup
struct HostSetup {
    int n = 0, m = 0, p = 0, P = 0, N = 0;
    int disc = SG_DISC_Q1;             // discretisation
    double gscale = 1.0;               // factor on the G_k (k >= 1) coupling entries: sqrt 3 for SG_DISC_P1
    std::vector<int> offsets;          // p+2
    std::vector<int> midx;             // P*m
    std::vector<double> lambda;        // m eigenvalues lambda_k of the 2-D modes
    std::vector<double> amps;          // m amplitudes s_k
    std::vector<double> cellc;         // (m+1) x n_elem, row k (n_elem = n*n cells, or 2 n*n triangles)
    std::vector<double> klcell;        // m x n*n values b_k at cell centres (SG_DISC_Q1)
    // operator coefficients in the apply kernel's layout, n*n positions (cx, cy) at cy*n + cx:
    //   SG_DISC_Q1: (m+1) values c_{k,cell} / 6 per cell;
    //   SG_DISC_P1: 2(m+1) values per grid vertex (cx, cy): the weights of its east edge
    //   (to (cx+1, cy)) for k = 0..m, then those of its north edge (to (cx, cy+1))
    std::vector<double> kcoef;
    std::vector<double> load;          // N: f_h (SG_DISC_P1; f = 1 is generated on the device)
    double a_min_h = 0.0;
    // multigrid, level 0 = finest
    std::vector<int> mg_n;             // cells per side per level
    std::vector<std::vector<double>> mg_sten;  // per level: N_l x 9, (dy,dx) row-major
    std::vector<double> coarse_inv;    // N_c x N_c inverse of the coarsest operator
};

int host_setup(const sg_options& opt, const double* a0_nodal, const double* kl_amp, HostSetup& hs);

// The 2 x 2 split of Sec. 4.2, A = [[A_hat, W^T], [W, D]]: A_hat couples the
// modes of degree <= p-1, D = I (x) K_0 the modes of degree p.  One multigrid
// cycle for the coupled system A_hat needs, on every level l of the K_0
// hierarchy, the Galerkin coarse operators of all K_k (A_hat_l = sum_k
// G_hat_k (x) P^T K_k P), the coupling partners of every mode, and the
// coarsest A_hat_l inverted.
struct SplitHost {
    int Pa = 0;                              // modes of degree <= p - 1
    int npart = 0;                           // partner positions per mode: 2m (at least 2)
    std::vector<std::vector<double>> sten;   // per level: (m+1) blocks of N_l x 9, block k = K_k on that level
    std::vector<int> pidx;                   // Pa x npart: partner beta | (k << 16), k = 1..m; -1 unused
    std::vector<double> pcoef;               // Pa x npart: G_k(alpha, beta)
    std::vector<double> cinv;                // (N_c Pa)^2 inverse of the coarsest A_hat_l, index node * Pa + alpha
};
constexpr int kSplitMaxCoarse = 2048;        // largest N_c Pa the coarsest direct solve of A_hat takes
int split_setup(const HostSetup& hs, SplitHost& sp);

// coupling tables of one apply "plan": output modes [out_lo, out_lo+W_out),
// input modes [in_lo, in_lo+W_in).  Lanes are grouped in slots of 64 (one
// wavefront each); the K_k u values (k >= 1) of a node row are exchanged
// through LDS at element exchange_index(k - 1, input lane).
//   Apply tables: every output lane lists its coupling partners at kNPos
//   positions (16-bit exchange indices, two per word; an absent partner reads
//   the row's zero entry).  Positions are grouped by the value of the
//   coefficient G_k(alpha, beta), so that inside one slot every position has a
//   single coefficient, shared by all lanes: xcoef[slot][position], and the
//   slot uses the first npos[slot] positions.
//   Gradient tables (full plan, read by the adjoint cell-gradient kernel):
//   for each lane and k, the partners alpha + e_k (low 16 bits of off) and
//   alpha - e_k (high 16 bits) as element k*lanes + beta, with coefficients
//   at positions 2k and 2k+1 of coef.
constexpr int kNPos = 16;

__host__ __device__ constexpr int exchange_index(int m, int lanes, int kk, int b) {
    // K_{kk+1} u of input lane b: pairs of consecutive k share one 16-byte slot
    // per lane (written with one 128-bit store); an odd last k stands alone
    return kk < 2 * (m / 2) ? (kk >> 1) * 2 * lanes + 2 * b + (kk & 1) : 2 * (m / 2) * lanes + b;
}

struct PlanHost {
    int in_lo = 0, W_in = 0, out_lo = 0, W_out = 0, nslot = 1;
    int self = 0;  // include the k = 0 (G_0 = I) term
    std::vector<uint32_t> xoff;   // nslot*64*kNPos/2
    std::vector<double> xcoef;    // nslot*kNPos
    std::vector<int> npos;        // nslot
    std::vector<uint32_t> off;    // nslot*64*m   (gradient tables)
    std::vector<double> coef;     // nslot*64*2m
    // when every output mode has at most one partner (one_partner): per output mode its
    // coefficient row k+1 | input lane << 8 and coefficient (0: none)
    int one_partner = 0;
    std::vector<int> okb;
    std::vector<double> ocoef;
};
PlanHost make_plan(const HostSetup& hs, int in_lo, int W_in, int out_lo, int W_out, bool self, bool up, bool down);

// ---------------------------------------------------------------- device side
struct Plan {
    int in_lo, W_in, out_lo, W_out, nslot, self;
    uint32_t* d_xoff;
    double* d_xcoef;
    int* d_npos;
    int nblk_max;  // max over slots of ceil(npos / 4)
    uint32_t* d_off;
    double* d_coef;
    int one_partner;
    int* d_okb;
    double* d_ocoef;
};

struct Level {
    int n, nx, N;          // cells, interior nodes per side, interior nodes
    double* sten64;        // N x 9
    float* sten32;
    double* rdiag64;       // N reciprocals of the stencil diagonals (the smoothers multiply by them)
    float* rdiag32;
    // grids the fused coarse cycle keeps in LDS: the stencils in colour order (colours in sweep
    // order, nodes of a colour y-major), 9 coefficients and the reciprocal diagonal per node,
    // padded to 10 doubles / 12 floats so that a thread loads its node's entry in 16-byte pieces
    double* cst64;
    float* cst32;
    // the stencils node by node with the reciprocal diagonal, padded to 10 doubles / 12 floats
    // (16-byte pieces) for the narrow row smoother
    double* stp64;
    float* stp32;
    // work buffers, capacity N x P
    double* u64; double* f64; double* r64; double* w64;  // w: second smoothing buffer
    float* u32; float* f32; float* r32; float* w32;
};

struct Workspace {
    // Krylov
    int restart = 0;
    double* V = nullptr;         // (restart+1) x NP
    void* Z = nullptr;           // restart x NP, float (mixed) or double
    size_t z_bytes = 0;          // capacity of Z in bytes
    int z_is_float = 0;
    double* w = nullptr;         // NP
    double* amps = nullptr;      // m KL amplitudes s_k
    double* pcg = nullptr;       // 4 x NP (PCG r, z, p, q)
    double* lt = nullptr;        // NP: A v before the preconditioner (left-preconditioned GMRES)
    double* partial = nullptr;   // reduction partials
    double* scal = nullptr;      // device scalars (h, norms, y)
    double* host_scal = nullptr; // pinned mirror
    // preconditioner staging
    void* fstage = nullptr;      // N x P (float or double) right-hand side staging
    void* ustage = nullptr;      // N x P staging for the backward sweep of B_S
    size_t fstage_bytes = 0;
    // adjoint
    double* lam = nullptr;       // NP
    double* g = nullptr;         // NP
    double* dc = nullptr;        // n*n x (m+1)
    double* wS = nullptr;        // N
    double* qv = nullptr;        // P
};

// device copies of SplitHost and the coupled cycle's work buffers (allocated on first use)
struct SplitDev {
    int ready = 0;
    int Pa = 0, npart = 0, gmax = 0;         // gmax: widest degree block of A_hat
    std::vector<double*> sten;               // per level, (m+1) x N_l x 9
    std::vector<double*> u, f, r;            // per level, N_l x Pa (u, f from level 1; r above the coarsest)
    int* pidx = nullptr;
    double* pcoef = nullptr;
    double* cinv = nullptr;
    double* g = nullptr;                     // N_0 x gmax: coupled right-hand sides of one degree block
    double* s1 = nullptr;                    // N_0 x Pa staging of the symmetric variant
    double* s2 = nullptr;
};

}  // namespace sg

struct sg_ctx {
    sg::HostSetup hs;
    sg_options opt;
    hipStream_t stream = nullptr;
    int device = 0;
    double* qoi_scratch = nullptr;  // this device's static scratch of sg_qoi_noalloc
    // device data
    double* cell64 = nullptr;   // HostSetup::kcoef on the device
    double* load = nullptr;     // HostSetup::load on the device (SG_DISC_P1)
    double* klcell = nullptr;   // n*n x m  b_k at cell centres, cell-major
    double* kinv = nullptr;     // N_c x N_c
    double* zeros = nullptr;    // 256 zeros: the value of grid neighbours outside the domain in the apply
    std::vector<sg::Level> levels;
    sg::Plan plan_full{};
    std::vector<sg::Plan> plan_down;  // index d = 1..p: level d-1 -> level d
    std::vector<sg::Plan> plan_up;    // index d = 0..p-1: level d+1 -> level d
    sg::Workspace ws;
    sg::SplitDev split;
    std::vector<void*> allocations;
};

namespace sg {

// kernel launchers (defined in the .hip files).  launch_apply takes U already
// offset to the plan's first input mode and R, Y already offset to its first
// output mode (Y may also be a compact buffer of width W_out).
int launch_apply(sg_ctx* c, const Plan& pl, const void* U, int in_float, const double* R, void* Y,
                 int out_float, int ldu, int ldy, int ldr);
// the same for SG_DISC_P1 (called by launch_apply)
int launch_apply_p1(sg_ctx* c, const Plan& pl, const void* U, int in_float, const double* R, void* Y,
                    int out_float, int ldu, int ldy, int ldr);
int launch_vcycle(sg_ctx* c, const void* f, int ldf, void* u, int ldu, int width, int is_float);
int launch_cast(hipStream_t s, const void* src, int src_float, int lds, void* dst, int dst_float, int ldd,
                int rows, int width);
int launch_fill(hipStream_t s, void* dst, int is_float, int ld, int rows, int width);
// double blocks of `width` modes on multigrid level l (node-major, row strides as given):
// fc (level l+1) = P^T r (level l); u (level l) += P ec (level l+1); one lexicographic
// Gauss-Seidel sweep of K_0 on level l (backward when reverse)
int launch_restrict_block(sg_ctx* c, int l, const double* r, int ldr, double* fc, int ldc, int width);
int launch_prolong_block(sg_ctx* c, int l, const double* ec, int ldc, double* u, int ldu, int width);
int launch_lex_sweep(sg_ctx* c, int l, double* u, int ldu, const double* f, int ldf, int width, int reverse);
// out[:, t] = f[:, lo+t] - self K_0 u[:, lo+t] - sum_partners G_k(lo+t, beta) K_k u[:, beta] on
// level l, t = 0..width-1 (sg_split.hip)
int launch_split_couple(sg_ctx* c, int l, const double* u, int ldu, const double* f, int ldf, double* out, int ldo,
                        int lo, int width, int self);
// u = A_hat_c^{-1} f on the coarsest level (both N_c x Pa, row strides ldf, ldu)
int launch_split_coarse(sg_ctx* c, const double* f, int ldf, double* u, int ldu);
// dst[:, 0:width] += a * src[:, 0:width] (both float or both double, row strides lds / ldd)
int launch_axpy_cols(hipStream_t s, const void* src, int is_float, int lds, void* dst, int ldd, int rows, int width,
                     double a);

}  // namespace sg
