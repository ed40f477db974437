// FP64 check and metrics of a coupling (gfx950).
//
// For the coupling P_ij = exp((f_i + g_j - C_ij)/eps) of the entropic dual
// (eq. entdual), one pass over rows gives r_i = sum_j P_ij, the row-marginal
// L1 sum_i |r_i - a_i|, the mass sum_ij P_ij, <f, a>, the transport cost
// <P, C> = sum_ij P_ij C_ij and sum_ij P_ij log P_ij (log P_ij is the exponent
// itself, so both are one FMA each per pair); the same kernel over columns
// gives the column-marginal L1 and <g, b>.  Everything is FP64:
// C_ij = |x_i|^2 + |y_j|^2 - 2 <x_i, y_j> with FP64 norms of the FP32 inputs
// and the cross term on v_mfma_f64_16x16x4_f64 (FP64 products of the exact
// FP32 values, FP64 accumulation), FP64 exp, FP64 sums.
//
// Tiling as in the FP32 potential kernel: a workgroup holds 64 rows in
// registers (lane l of a wave owns row l%16, lane group l/16 holds features
// [q D/4, (q+1) D/4)), streams 16-column tiles through LDS, and each lane
// accumulates its row's sum over the columns of its accumulator slots.  The
// FP64 accumulator layout differs from the FP32/BF16 16x16 ones: register r
// of lane l holds tile row 4 r + l/16 (checked on the device with a probe
// of the instruction's lane layout).

#include "progot_internal.h"

#include <algorithm>
#include <cmath>

namespace pot {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(256) void sqnorm_f64(const float *__restrict__ X, int64_t n, int d,
                                                  double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        const double v = X[i * d + k];
        s = fma(v, v, s);
    }
    out[i] = s;
}

template <int D>
__global__ __launch_bounds__(256) void fp64_rowsums(
    const float *__restrict__ U, int64_t nu, const float *__restrict__ V, int64_t nv, int d,
    const double *__restrict__ usq, const double *__restrict__ vsq, const float *__restrict__ pu,
    const float *__restrict__ pv, const float *__restrict__ w_in, double eps,
    double *__restrict__ part) {
    constexpr int KD = D / 4;
    constexpr int BN = 16;
    constexpr int STRIDE = D + 2;
    __shared__ double vt[BN * STRIDE];
    __shared__ double vb[BN];
    __shared__ double vs[BN];
    __shared__ double red[256];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int64_t row = (int64_t)blockIdx.x * 64 + wave * 16 + li;
    const bool live = row < nu;

    double ub[KD];
#pragma unroll
    for (int k = 0; k < KD; ++k) {
        const int f = lq * KD + k;
        ub[k] = (live && f < d) ? (double)U[row * d + f] : 0.0;
    }
    const double base = live ? (double)pu[row] - usq[row] : 0.0;   // f_i - |x_i|^2
    const double usq_i = live ? usq[row] : 0.0;
    const double inv_eps = 1.0 / eps;
    double rsum = 0.0, pc = 0.0, plp = 0.0;

    for (int64_t j0 = 0; j0 < nv; j0 += BN) {
        for (int e = tid; e < BN * D; e += 256) {
            const int r = e / D, c = e % D;
            const int64_t j = j0 + r;
            vt[r * STRIDE + c] = (j < nv && c < d) ? (double)V[j * d + c] : 0.0;
        }
        if (tid < BN) {
            const int64_t j = j0 + tid;
            vb[tid] = j < nv ? (double)pv[j] - vsq[j] : -INFINITY;   // g_j - |y_j|^2
            vs[tid] = j < nv ? vsq[j] : 0.0;
        }
        __syncthreads();
        d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KD; ++s) acc = mfma_f64(vt[li * STRIDE + lq * KD + s], ub[s], acc);
        // The FP64 16x16 accumulator interleaves its rows: register r of lane
        // l holds row 4 r + l/16 (measured), so acc[r] = <y_{j0 + 4 r + lq}, x_row>.
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int jl = 4 * r + lq;
            const double t = (base + vb[jl] + 2.0 * acc[r]) * inv_eps;   // log P_ij
            const double p = exp(t);
            rsum += p;
            if (vb[jl] > -INFINITY) {
                pc = fma(p, usq_i + vs[jl] - 2.0 * acc[r], pc);
                plp = fma(p, t, plp);
            }
        }
        __syncthreads();
    }
    rsum += __shfl_xor(rsum, 16);
    rsum += __shfl_xor(rsum, 32);
    pc += __shfl_xor(pc, 16);
    pc += __shfl_xor(pc, 32);
    plp += __shfl_xor(plp, 16);
    plp += __shfl_xor(plp, 32);
    const bool own = live && lq == 0;
    const double w = own ? (w_in ? (double)w_in[row] : 1.0 / (double)nu) : 0.0;
    const double vals[kCheckParts] = {own ? fabs(rsum - w) : 0.0, own ? rsum : 0.0,
                                      own ? (double)pu[row] * w : 0.0, own ? pc : 0.0,
                                      own ? plp : 0.0};
    for (int q = 0; q < kCheckParts; ++q) {
        __syncthreads();
        red[tid] = vals[q];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        if (tid == 0) part[(int64_t)blockIdx.x * kCheckParts + q] = red[0];
    }
}

// |e|^p in FP64 (p = 1.5 as |e| sqrt|e|).
__device__ __forceinline__ double pow_abs64(double e, double p) {
    const double a = fabs(e);
    return p == 1.5 ? a * sqrt(a) : (a == 0.0 ? 0.0 : pow(a, p));
}

// The same row pass for the cost h(z) = (1/p) sum_k |z_k|^p, whose C_ij has
// no inner-product form: each lane group adds its quarter of the features'
// |x_ik - y_jk|^p for 4 columns of a 16-column LDS tile (FP64 differences of
// the FP32 inputs, FP64 powers), the 4 groups' partials are summed across
// lanes, and row i's sums are accumulated as above.
template <int D>
__global__ __launch_bounds__(256) void pcost_rowsums(
    const float *__restrict__ U, int64_t nu, const float *__restrict__ V, int64_t nv, int d,
    double p, const float *__restrict__ pu, const float *__restrict__ pv,
    const float *__restrict__ w_in, double eps, double *__restrict__ part) {
    constexpr int KD = D / 4;
    constexpr int BN = 16;
    constexpr int STRIDE = D + 2;
    __shared__ double vt[BN * STRIDE];
    __shared__ double vb[BN];
    __shared__ double red[256];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int64_t row = (int64_t)blockIdx.x * 64 + wave * 16 + li;
    const bool live = row < nu;
    double ub[KD];
#pragma unroll
    for (int k = 0; k < KD; ++k) {
        const int f = lq * KD + k;
        ub[k] = (live && f < d) ? (double)U[row * d + f] : 0.0;
    }
    const double fu = live ? (double)pu[row] : 0.0;
    const double inv_eps = 1.0 / eps, inv_p = 1.0 / p;
    double rsum = 0.0, pc = 0.0, plp = 0.0;
    for (int64_t j0 = 0; j0 < nv; j0 += BN) {
        for (int e = tid; e < BN * D; e += 256) {
            const int r = e / D, c = e % D;
            const int64_t j = j0 + r;
            vt[r * STRIDE + c] = (j < nv && c < d) ? (double)V[j * d + c] : 0.0;
        }
        if (tid < BN) vb[tid] = j0 + tid < nv ? (double)pv[j0 + tid] : -INFINITY;
        __syncthreads();
#pragma unroll 1
        for (int jl = 0; jl < BN; ++jl) {
            double c = 0.0;
#pragma unroll
            for (int k = 0; k < KD; ++k) c += pow_abs64(ub[k] - vt[jl * STRIDE + lq * KD + k], p);
            c += __shfl_xor(c, 16);
            c += __shfl_xor(c, 32);
            c *= inv_p;
            if (vb[jl] > -INFINITY) {
                const double t = (fu + vb[jl] - c) * inv_eps;   // log P_ij
                const double pr = exp(t);
                rsum += pr;
                pc = fma(pr, c, pc);
                plp = fma(pr, t, plp);
            }
        }
        __syncthreads();
    }
    // every lane of a row holds the row's sums; the lq == 0 lane reports them
    const bool own = live && lq == 0;
    const double w = own ? (w_in ? (double)w_in[row] : 1.0 / (double)nu) : 0.0;
    const double vals[kCheckParts] = {own ? fabs(rsum - w) : 0.0, own ? rsum : 0.0,
                                      own ? (double)pu[row] * w : 0.0, own ? pc : 0.0,
                                      own ? plp : 0.0};
    for (int q = 0; q < kCheckParts; ++q) {
        __syncthreads();
        red[tid] = vals[q];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        if (tid == 0) part[(int64_t)blockIdx.x * kCheckParts + q] = red[0];
    }
}

template <int D>
void prowsums_t(const float *U, int64_t nu, const float *V, int64_t nv, int d, double p,
                const float *pu, const float *pv, const float *w, double eps, double *part,
                hipStream_t s) {
    hipLaunchKernelGGL((pcost_rowsums<D>), dim3((unsigned)fp64_check_blocks(nu)), dim3(256), 0, s, U,
                       nu, V, nv, d, p, pu, pv, w, eps, part);
}

void prowsums(const float *U, int64_t nu, const float *V, int64_t nv, int d, double p,
              const float *pu, const float *pv, const float *w, double eps, double *part,
              hipStream_t s) {
    if (d <= 16) prowsums_t<16>(U, nu, V, nv, d, p, pu, pv, w, eps, part, s);
    else if (d <= 32) prowsums_t<32>(U, nu, V, nv, d, p, pu, pv, w, eps, part, s);
    else if (d <= 64) prowsums_t<64>(U, nu, V, nv, d, p, pu, pv, w, eps, part, s);
    else if (d <= 128) prowsums_t<128>(U, nu, V, nv, d, p, pu, pv, w, eps, part, s);
    else prowsums_t<256>(U, nu, V, nv, d, p, pu, pv, w, eps, part, s);
}

// Diagonal of the coupling (n == m): per block, sum_i P_ii and
// sum_i log P_ii with P_ii = exp((f_i + g_i - |x_i - y_i|^2)/eps), the cost by
// FP64 direct differences.
__global__ __launch_bounds__(256) void diag_sums(const float *__restrict__ X, const float *__restrict__ Y,
                                                 int64_t n, int d, const float *__restrict__ f,
                                                 const float *__restrict__ g, double eps, double cp,
                                                 double *__restrict__ part) {
    __shared__ double red[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double lp = 0.0, p = 0.0;
    if (i < n) {
        double c = 0.0;
        for (int k = 0; k < d; ++k) {
            const double e = (double)X[i * d + k] - (double)Y[i * d + k];
            c = cp > 0.0 ? c + pow_abs64(e, cp) : fma(e, e, c);
        }
        if (cp > 0.0) c /= cp;
        lp = ((double)f[i] + (double)g[i] - c) / eps;
        p = exp(lp);
    }
    const double vals[2] = {p, lp};
    for (int q = 0; q < 2; ++q) {
        __syncthreads();
        red[threadIdx.x] = vals[q];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 2 + q] = red[0];
    }
}

template <int D>
void rowsums_t(const float *U, int64_t nu, const float *V, int64_t nv, int d, const double *usq,
               const double *vsq, const float *pu, const float *pv, const float *w, double eps,
               double *part, hipStream_t s) {
    hipLaunchKernelGGL((fp64_rowsums<D>), dim3((unsigned)fp64_check_blocks(nu)), dim3(256), 0, s, U,
                       nu, V, nv, d, usq, vsq, pu, pv, w, eps, part);
}

void rowsums(const float *U, int64_t nu, const float *V, int64_t nv, int d, const double *usq,
             const double *vsq, const float *pu, const float *pv, const float *w, double eps,
             double *part, hipStream_t s) {
    if (d <= 16) rowsums_t<16>(U, nu, V, nv, d, usq, vsq, pu, pv, w, eps, part, s);
    else if (d <= 32) rowsums_t<32>(U, nu, V, nv, d, usq, vsq, pu, pv, w, eps, part, s);
    else if (d <= 64) rowsums_t<64>(U, nu, V, nv, d, usq, vsq, pu, pv, w, eps, part, s);
    else if (d <= 128) rowsums_t<128>(U, nu, V, nv, d, usq, vsq, pu, pv, w, eps, part, s);
    else rowsums_t<256>(U, nu, V, nv, d, usq, vsq, pu, pv, w, eps, part, s);
}

// Per-block FP64 partials of sum_i v_i w_i (w == NULL: uniform 1/n).
__global__ __launch_bounds__(256) void weighted_sum_f64(const float *__restrict__ v,
                                                        const float *__restrict__ w, int64_t n,
                                                        double *__restrict__ part) {
    __shared__ double red[256];
    double s = 0.0;
    const double u = 1.0 / (double)n;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        s = fma((double)v[i], w ? (double)w[i] : u, s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace

int weighted_sum_blocks(int64_t n) { return (int)std::min<int64_t>(256, (n + 255) / 256); }

hipError_t launch_weighted_sum(const float *v, const float *w, int64_t n, double *part,
                               hipStream_t s) {
    hipLaunchKernelGGL(weighted_sum_f64, dim3((unsigned)weighted_sum_blocks(n)), dim3(256), 0, s, v, w,
                       n, part);
    return hipGetLastError();
}

int fp64_check_blocks(int64_t n) { return (int)((n + 63) / 64); }
int diag_blocks(int64_t n) { return (int)((n + 255) / 256); }

hipError_t launch_diag_sums(const float *X, const float *Y, int64_t n, int d, const float *f,
                            const float *g, float eps, float cost_p, double *part, hipStream_t s) {
    hipLaunchKernelGGL(diag_sums, dim3((unsigned)diag_blocks(n)), dim3(256), 0, s, X, Y, n, d, f, g,
                       (double)eps, (double)cost_p, part);
    return hipGetLastError();
}

hipError_t launch_fp64_check_pcost(const float *X, int64_t n, const float *Y, int64_t m, int d,
                                   float p, const float *f, const float *g, const float *a,
                                   const float *b, float eps, double *part_rows,
                                   double *part_cols, hipStream_t s) {
    // h is even, so the columns' pass is the rows' pass with the roles swapped
    prowsums(X, n, Y, m, d, (double)p, f, g, a, (double)eps, part_rows, s);
    prowsums(Y, m, X, n, d, (double)p, g, f, b, (double)eps, part_cols, s);
    return hipGetLastError();
}

hipError_t launch_fp64_check(const float *X, int64_t n, const float *Y, int64_t m, int d,
                             const float *f, const float *g, const float *a, const float *b,
                             float eps, double *xsq64, double *ysq64, double *part_rows,
                             double *part_cols, hipStream_t s) {
    hipLaunchKernelGGL(sqnorm_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, n, d, xsq64);
    hipLaunchKernelGGL(sqnorm_f64, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, Y, m, d, ysq64);
    rowsums(X, n, Y, m, d, xsq64, ysq64, f, g, a, (double)eps, part_rows, s);
    rowsums(Y, m, X, n, d, ysq64, xsq64, g, f, b, (double)eps, part_cols, s);
    return hipGetLastError();
}

}  // namespace pot
