// General translation-invariant costs h(z) = (1/p) sum_k |z_k|^p on gfx950.
//
// ProgOT is stated for any strictly convex translation-invariant cost (Sec. 3);
// the experiments of Sec. 5.2 and the map appendix use this h with p = 1.5.
// For it grad h(z)_k = sign(z_k) |z_k|^(p-1) and grad h*(w)_k =
// sign(w_k) |w_k|^(1/(p-1)), elementwise.  There is no inner-product form of
// C_ij = h(x_i - y_j), so nothing here maps onto MFMA: every pair and
// feature costs a subtraction, a power (p = 1.5: one v_sqrt_f32, since
// |z|^1.5 = |z| sqrt|z| and |z|^0.5 = sqrt|z| serve both the cost and its
// gradient; other p: v_log_f32 and v_exp_f32) and an FMA on the VALU.
//
// Layout of the work:
//   * cost matrix: during one Sinkhorn solve the cost C(X^(k), Y) does not
//     change, so it is computed once per solve (pcost_matrix: 64 x 64 tiles,
//     4 x 4 pairs per lane, features staged through LDS in 32-feature
//     slices) into the workspace, row-major with a row stride ldc = m
//     rounded up to 4 floats, with FP64 per-block sums for the mean cost that
//     sets eps.  Rebuilding it per half-iteration would cost d x (sub, sqrt,
//     fma) per pair; reading it back costs 4 bytes per pair, which HBM (or
//     the 256 MB last-level cache, when C fits) serves faster for any d
//     beyond a handful.
//   * f-update: pcost_lse_rows, one wave per row of C and column split,
//     float4 loads (12 in flight per lane), per-lane running (max, sum) in
//     log2 units with one rescale per 48 values, then a wave reduction;
//     with one split (n large enough to fill the chip) the wave writes the
//     potential and its marginal-error term itself.
//   * g-update: pcost_lse_cols, 256 columns per workgroup (4 per lane, so a
//     wave reads 1 KB of each row), 8 waves walk interleaved 8-row chunks
//     of the split's rows and combine through LDS.
//   * split updates write the same per-split (max, sum) partials as the
//     squared-Euclidean potential kernels, and the same merge kernel turns
//     them into the potential and the row-marginal error.
//   * map (eq. Tent / Alg. 2 and 3 step x - alpha grad h*(sum_j p_j grad
//     h(x - y_j))): pcost_map, fused and on the fly (the gradient needs the
//     per-feature root anyway).  A lane group of LQ lanes owns one query
//     (F = min(D, 48) or 32 features each, query and accumulators in
//     registers); target
//     tiles of 32 points are staged in LDS; the weight is an online softmax
//     in log2 units with a rescale only when some lane's maximum rises.  With
//     few queries the targets are split S ways; each split writes (max, sum,
//     accumulator) partials and pcost_map_merge combines them and applies
//     grad h* and the step.

#include "progot_internal.h"
#include "progot_device.h"

#include <algorithm>

namespace pot {
namespace {

// |z|^(p-1) for a = |z|; PK = 1 is p = 1.5.
template <int PK> __device__ __forceinline__ float pow_pm1(float a, float pm1);
template <> __device__ __forceinline__ float pow_pm1<1>(float a, float) {
    return __builtin_amdgcn_sqrtf(a);
}
template <> __device__ __forceinline__ float pow_pm1<0>(float a, float pm1) {
    return ex2(pm1 * __builtin_amdgcn_logf(a));   // a = 0: 2^(-inf) = 0
}

// grad h*(w) = sign(w) |w|^(1/(p-1)); p = 1.5: w |w|.
template <int PK> __device__ __forceinline__ float grad_h_star(float w, float inv_pm1);
template <> __device__ __forceinline__ float grad_h_star<1>(float w, float) { return w * fabsf(w); }
template <> __device__ __forceinline__ float grad_h_star<0>(float w, float inv_pm1) {
    return __builtin_copysignf(ex2(inv_pm1 * __builtin_amdgcn_logf(fabsf(w))), w);
}

// ---------------------------------------------------------------- cost matrix
constexpr int kCT = 64;        // tile rows and columns
constexpr int kCK = 32;        // features per LDS slice
constexpr int kCS = kCT + 4;   // LDS stride of a transposed slice (16-byte aligned)

template <int PK, bool STORE>
__global__ __launch_bounds__(256) void pcost_matrix(const float *__restrict__ X, int64_t n,
                                                    const float *__restrict__ Y, int64_t m, int d,
                                                    float pm1, float inv_p, int64_t col_tiles,
                                                    float *__restrict__ Cm, int64_t ldc,
                                                    double *__restrict__ part) {
    __shared__ __align__(16) float xs[kCK * kCS];
    __shared__ __align__(16) float ys[kCK * kCS];
    __shared__ double red[256];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int64_t bt = blockIdx.x;
    const int64_t r0 = (bt / col_tiles) * kCT, c0 = (bt % col_tiles) * kCT;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < d; k0 += kCK) {
        // slices stored transposed ([feature][point]); features beyond d are
        // zero on both sides and add h(0) = 0
        for (int e = tid; e < kCT * kCK; e += 256) {
            const int r = e / kCK, k = e % kCK;
            const bool kin = k0 + k < d;
            xs[k * kCS + r] = (kin && r0 + r < n) ? X[(r0 + r) * d + k0 + k] : 0.f;
            ys[k * kCS + r] = (kin && c0 + r < m) ? Y[(c0 + r) * d + k0 + k] : 0.f;
        }
        __syncthreads();
        const int kn = std::min(kCK, d - k0);
        for (int k = 0; k < kn; k += 4) {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const f4 xv = *reinterpret_cast<const f4 *>(&xs[(k + kk) * kCS + ty * 4]);
                const f4 yv = *reinterpret_cast<const f4 *>(&ys[(k + kk) * kCS + tx * 4]);
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const float z = fabsf(xv[a] - yv[b]);
                        acc[a][b] = fmaf(z, pow_pm1<PK>(z, pm1), acc[a][b]);
                    }
            }
        }
        __syncthreads();
    }
    double s = 0.0;
    const int64_t cc = c0 + tx * 4;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t r = r0 + ty * 4 + a;
        f4 v;
        v.x = acc[a][0] * inv_p; v.y = acc[a][1] * inv_p;
        v.z = acc[a][2] * inv_p; v.w = acc[a][3] * inv_p;
        if (r < n) {
#pragma unroll
            for (int b = 0; b < 4; ++b)
                if (cc + b < m) s += (double)v[b];
            // ldc is a multiple of 4, so the 4 columns are inside the row
            if (STORE && cc < ldc) *reinterpret_cast<f4 *>(Cm + r * ldc + cc) = v;
        }
    }
    red[tid] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) part[bt] = red[0];
}

// Fixed-order FP64 sum of n partials (one workgroup).
__global__ __launch_bounds__(256) void sum_f64(const double *__restrict__ part, int64_t n,
                                               double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------- potentials
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// f-update partials: row i of C against the split's columns,
//   t_ij = (gamma vpot_j - C_ij) log2(e)/eps,  (max_j t, sum_j 2^(t - max)).
// FUSE (one split): the wave holds the whole row, so it writes the potential
// and its row-marginal error term itself (the merge kernel's arithmetic),
// and the workgroup writes one error partial per 4 rows.
template <bool FUSE>
__global__ __launch_bounds__(256) void pcost_lse_rows(LseJob J) {
    __shared__ float errw[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int S = J.S;
    const int split = (int)(blockIdx.x % S);
    const int64_t row = (int64_t)(blockIdx.x / S) * 4 + wave;
    const bool live = row < J.nu;
    if (!FUSE && !live) return;   // whole wave; no workgroup barrier in this form
    const int64_t c_lo = (int64_t)split * J.cps;
    const int64_t c_hi = std::min(J.nv, c_lo + J.cps);
    const float k = J.bscale, gk = J.gamma * J.bscale;
    const float *__restrict__ crow = J.cmat + (live ? row : 0) * J.ldc;
    const float *__restrict__ vp = J.vpot;
    // vector loads of the potential only where it is 16-byte aligned (a row
    // of a caller's K x m array need not be)
    const bool vp4 = vp && (reinterpret_cast<uintptr_t>(vp) & 15) == 0;
    float M = kNegBig, s = 0.f;
    // 12 float4 per lane in flight: a row of up to 3072 columns in one round
    // of loads (a second, short round cost 20-30 % at m = 2800; 16 per lane
    // costs occupancy)
    for (int64_t c = c_lo + 4 * lane; live && c < c_hi; c += 256 * 12) {
        float t[48];
#pragma unroll
        for (int u = 0; u < 12; ++u) {
            const int64_t cc = c + 256 * u;
            // cc and ldc are multiples of 4: the float4 stays inside the row
            const f4 cv = cc < c_hi ? *reinterpret_cast<const f4 *>(crow + cc) : f4{0.f, 0.f, 0.f, 0.f};
            f4 gv = {0.f, 0.f, 0.f, 0.f};
            if (vp) {
                if (vp4 && cc + 4 <= c_hi) {
                    gv = *reinterpret_cast<const f4 *>(vp + cc);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) gv[e] = cc + e < c_hi ? vp[cc + e] : 0.f;
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
                t[4 * u + e] = cc + e < c_hi ? fmaf(gv[e], gk, -cv[e] * k) : -INFINITY;
        }
        float cm = kNegBig;
#pragma unroll
        for (int e = 0; e < 48; ++e) cm = fmaxf(cm, t[e]);
        if (cm > M) {
            s *= ex2(M - cm);
            M = cm;
        }
        float a0 = 0.f, a1 = 0.f;
#pragma unroll
        for (int e = 0; e < 48; e += 2) {
            a0 += ex2(t[e] - M);
            a1 += ex2(t[e + 1] - M);
        }
        s += a0 + a1;
    }
    const float Mw = wave_max(M);
    s = wave_sum(s * ex2(M - Mw));
    if (!FUSE) {
        if (lane == 0) {
            J.part_m[(int64_t)split * J.nu + row] = Mw;
            J.part_s[(int64_t)split * J.nu + row] = s;
        }
        return;
    }
    float e = 0.f;
    if (live && lane == 0) {
        const float L = Mw + log2f(s);
        const float lw = J.logw[row];
        const float pot = fmaf(J.eps, lw, 0.f) - J.eps * kLn2 * L;
        if (J.pot_old) e = expf(lw) * fabsf(expm1f((J.pot_old[row] - pot) / J.eps));
        J.pot_out[row] = pot;
    }
    if (J.pot_old) {
        if (lane == 0) errw[wave] = e;
        __syncthreads();
        if (threadIdx.x == 0) J.err_part[blockIdx.x] = (errw[0] + errw[1]) + (errw[2] + errw[3]);
    }
}

// Merge of split partials for the general-cost updates: one wave per
// output (its lanes fold the splits), the potential as in the squared
// path's merge, one error partial per 4 outputs.
__global__ __launch_bounds__(256) void pcost_merge(LseJob J) {
    __shared__ float errw[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 4 + wave;
    const bool live = i < J.nu;
    float M = kNegBig, sum = 0.f;
    for (int s = lane; live && s < J.S; s += 64) {
        const float m = J.part_m[(int64_t)s * J.nu + i], v = J.part_s[(int64_t)s * J.nu + i];
        const float Mn = fmaxf(M, m);
        sum = sum * ex2(M - Mn) + v * ex2(m - Mn);
        M = Mn;
    }
    const float Mw = wave_max(M);
    sum = wave_sum(sum * ex2(M - Mw));
    float e = 0.f;
    if (live && lane == 0) {
        const float L = Mw + log2f(sum);
        const float lw = J.logw[i];
        const float pot = fmaf(J.eps, lw, 0.f) - J.eps * kLn2 * L;
        if (J.pot_old) e = expf(lw) * fabsf(expm1f((J.pot_old[i] - pot) / J.eps));
        J.pot_out[i] = pot;
    }
    if (J.pot_old) {
        if (lane == 0) errw[wave] = e;
        __syncthreads();
        if (threadIdx.x == 0) J.err_part[blockIdx.x] = (errw[0] + errw[1]) + (errw[2] + errw[3]);
    }
}

// g-update partials: column j of C (the output index, J.nu = m columns)
// against the split's rows (J.cps rows per split, J.nv = n rows),
//   t_ij = (gamma vpot_i - C_ij) log2(e)/eps.
// kColWaves waves share the workgroup's 256 columns and walk interleaved
// 8-row chunks, so one split covers kColWaves x more rows per launch and the
// merge has fewer splits to fold.
constexpr int kColWaves = 8;

// Sum of n floats in the order of the standalone error sum (thread t < 256
// adds t, t + 256, ..., then a halving tree in LDS), by a workgroup of any
// size >= 256; every thread of the workgroup calls it (it holds barriers).
__device__ __forceinline__ float sum_in_order(const float *__restrict__ part, int n, float *red) {
    const int tid = threadIdx.x;
    if (tid < 256) {
        float v = 0.f;
        for (int i = tid; i < n; i += 256) v += part[i];
        red[tid] = v;
    }
    __syncthreads();
#pragma unroll
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    return red[0];
}

__global__ __launch_bounds__(64 * kColWaves) void pcost_lse_cols(LseJob J) {
    __shared__ float sm[kColWaves][256], ss[kColWaves][256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (J.esum_out && blockIdx.x == 0) {   // uniform over the workgroup
        const float tot = sum_in_order(J.esum_in, J.esum_n, sm[0]);
        if (tid == 0) J.esum_out[0] = tot;
        __syncthreads();   // sm[0] is reused below
    }
    const int S = J.S;
    const int split = (int)(blockIdx.x % S);
    const int64_t jb = (int64_t)(blockIdx.x / S) * 256;
    const int64_t j0 = jb + 4 * lane;
    const bool live = j0 < J.nu;            // then j0 + 3 < ldc
    const int64_t r_lo = (int64_t)split * J.cps;
    const int64_t r_hi = std::min(J.nv, r_lo + J.cps);
    const float k = J.bscale, gk = J.gamma * J.bscale;
    const float *__restrict__ vp = J.vpot;
    float M[4] = {kNegBig, kNegBig, kNegBig, kNegBig};
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    for (int64_t r = r_lo + 8 * wave; r < r_hi; r += 8 * kColWaves) {
        f4 cv[8];
        float fv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const bool ok = r + u < r_hi;
            cv[u] = (ok && live) ? *reinterpret_cast<const f4 *>(J.cmat + (r + u) * J.ldc + j0)
                                 : f4{0.f, 0.f, 0.f, 0.f};
            fv[u] = ok ? (vp ? vp[r + u] * gk : 0.f) : -INFINITY;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            float t[8];
            float cm = kNegBig;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                t[u] = fv[u] - cv[u][e] * k;
                cm = fmaxf(cm, t[u]);
            }
            if (cm > M[e]) {
                s[e] *= ex2(M[e] - cm);
                M[e] = cm;
            }
            float a = 0.f;
#pragma unroll
            for (int u = 0; u < 8; ++u) a += ex2(t[u] - M[e]);
            s[e] += a;
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        sm[wave][4 * lane + e] = M[e];
        ss[wave][4 * lane + e] = s[e];
    }
    __syncthreads();
    const int64_t j = jb + tid;
    if (tid < 256 && j < J.nu) {
        float Mx = sm[0][tid];
#pragma unroll
        for (int w = 1; w < kColWaves; ++w) Mx = fmaxf(Mx, sm[w][tid]);
        float tot = 0.f;
#pragma unroll
        for (int w = 0; w < kColWaves; ++w) tot += ss[w][tid] * ex2(sm[w][tid] - Mx);
        J.part_m[(int64_t)split * J.nu + j] = Mx;
        J.part_s[(int64_t)split * J.nu + j] = tot;
    }
}

// ---------------------------------------------------------------- map
constexpr int kMapTJ = 32;      // targets per LDS tile

int pmap_dim(int d) {
    return d <= 16 ? 16 : d <= 32 ? 32 : d <= 48 ? 48 : d <= 64 ? 64 : d <= 128 ? 128 : 256;
}
constexpr int kMapMaxSplit = 16;

template <int D> struct PShape {
    // features per lane: up to 48 keeps the query, its gradient terms and the
    // accumulators (3F registers) within 2 waves per SIMD; 64 would spill
    static constexpr int F = D <= 48 ? D : 32;
    static constexpr int LQ = D / F;                    // lanes per query (1, 2, 4, 8)
    static constexpr int QB = 256 / LQ;                 // queries per workgroup
    static constexpr int SEG = F + (LQ > 1 ? 4 : 0);    // LDS segment: lane groups on distinct banks
    static constexpr int RS = LQ * SEG;                 // LDS floats per target
};

// Cost partial of the lane group reduced over its LQ lanes (adjacent lanes).
template <int LQ> __device__ __forceinline__ float group_sum(float c) {
    if (LQ >= 2)
        c += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(c), 0xB1, 0xF, 0xF, true));  // lane ^ 1
    if (LQ >= 4)
        c += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(c), 0x4E, 0xF, 0xF, true));  // lane ^ 2
    if (LQ >= 8)   // lane ^ 4: swizzle in bit-mask mode (and 0x1f, xor 4)
        c += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(c), 0x101F));
    return c;
}

template <int D, int PK>
__global__ __launch_bounds__(256) void pcost_map(PcostMapArgs A, int S, int64_t tps) {
    using P = PShape<D>;
    constexpr int F = P::F, LQ = P::LQ, QB = P::QB, SEG = P::SEG, RS = P::RS;
    __shared__ __align__(16) float yt[kMapTJ * RS];
    __shared__ float gt[kMapTJ];
    const int tid = threadIdx.x, lq = tid % LQ;
    const int d = A.d;
    const int split = (int)(blockIdx.x % S);
    const int64_t q = (int64_t)(blockIdx.x / S) * QB + tid / LQ;
    const bool live = q < A.nq;
    const int f0 = lq * F;
    float x[F], acc[F];
#pragma unroll
    for (int k = 0; k < F; ++k) {
        x[k] = (live && f0 + k < d) ? A.Xq[q * d + f0 + k] : 0.f;
        acc[k] = 0.f;
    }
    float M = kNegBig, sum = 0.f;
    const float k2 = kLog2e / A.eps;
    const float kc = k2 / A.p;                 // cost h = c/p, scaled by log2(e)/eps
    const float pm1 = A.p - 1.f;
    const int64_t j_lo = (int64_t)split * tps;
    const int64_t j_hi = std::min(A.m, j_lo + tps);
    for (int64_t j0 = j_lo; j0 < j_hi; j0 += kMapTJ) {
        const int64_t nt = std::min<int64_t>(kMapTJ, j_hi - j0);
        __syncthreads();   // the previous tile is consumed
        for (int e = tid; e < kMapTJ * D; e += 256) {
            const int jj = e / D, kk = e % D;
            yt[jj * RS + (kk / F) * SEG + kk % F] =
                (jj < nt && kk < d) ? A.Y[(j0 + jj) * d + kk] : 0.f;
        }
        if (tid < kMapTJ) gt[tid] = tid < nt ? A.g[j0 + tid] * k2 : -INFINITY;
        __syncthreads();
        for (int jj = 0; jj < kMapTJ; ++jj) {
            const float *yj = yt + jj * RS + lq * SEG;
            float gs[F];
            float c0 = 0.f, c1 = 0.f, c2 = 0.f, c3 = 0.f;
#pragma unroll
            for (int k = 0; k < F; k += 4) {
                const f4 yv = *reinterpret_cast<const f4 *>(yj + k);
                float cp[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float z = x[k + e] - yv[e];
                    const float a = fabsf(z);
                    const float r = pow_pm1<PK>(a, pm1);
                    gs[k + e] = __builtin_copysignf(r, z);
                    cp[e] = a * r;
                }
                c0 += cp[0]; c1 += cp[1]; c2 += cp[2]; c3 += cp[3];
            }
            const float c = group_sum<LQ>((c0 + c1) + (c2 + c3));
            const float t = fmaf(-c, kc, gt[jj]);
            if (__builtin_amdgcn_ballot_w64(t > M)) {
                const float Mn = fmaxf(M, t);
                const float r = ex2(M - Mn);
                sum *= r;
#pragma unroll
                for (int k = 0; k < F; ++k) acc[k] *= r;
                M = Mn;
            }
            const float w = ex2(t - M);
            sum += w;
#pragma unroll
            for (int k = 0; k < F; ++k) acc[k] = fmaf(w, gs[k], acc[k]);
        }
    }
    if (!live) return;
    if (S == 1) {
        const float inv = 1.f / sum;
        const float inv_pm1 = 1.f / pm1;
#pragma unroll
        for (int k = 0; k < F; ++k)
            if (f0 + k < d)
                A.Xout[q * d + f0 + k] = x[k] - A.alpha * grad_h_star<PK>(acc[k] * inv, inv_pm1);
    } else {
        const int64_t slot = (int64_t)split * A.nq + q;
        if (lq == 0) {
            A.pm[slot] = M;
            A.ps[slot] = sum;
        }
#pragma unroll
        for (int k = 0; k < F; ++k) A.pacc[slot * D + f0 + k] = acc[k];
    }
}

template <int PK>
__global__ __launch_bounds__(256) void pcost_map_merge(PcostMapArgs A, int S, int D) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int d = A.d;
    if (idx >= A.nq * d) return;
    const int64_t q = idx / d;
    const int k = (int)(idx % d);
    float Mx = kNegBig;
    for (int s = 0; s < S; ++s) Mx = fmaxf(Mx, A.pm[(int64_t)s * A.nq + q]);
    float tot = 0.f, a = 0.f;
    for (int s = 0; s < S; ++s) {
        const int64_t slot = (int64_t)s * A.nq + q;
        const float r = ex2(A.pm[slot] - Mx);
        tot = fmaf(A.ps[slot], r, tot);
        a = fmaf(A.pacc[slot * D + k], r, a);
    }
    const float x = A.Xq[q * d + k];
    A.Xout[q * d + k] = x - A.alpha * grad_h_star<PK>(a / tot, 1.f / (A.p - 1.f));
}

// Potential update without the cost matrix (pairs too many to keep it):
// row i of U against the split's columns of V, the cost h(u_i - v_j) formed
// on the fly as in the map kernel (LQ lanes per row, column tiles of 32 in
// LDS), t_ij = (gamma vpot_j - h)/eps in log2 units, running (max, sum);
// writes the split partials that pcost_merge folds.
template <int D, int PK>
__global__ __launch_bounds__(256) void pcost_lse_fly(LseJob J, int64_t tps) {
    using P = PShape<D>;
    constexpr int F = P::F, LQ = P::LQ, QB = P::QB, SEG = P::SEG, RS = P::RS;
    __shared__ __align__(16) float vt[kMapTJ * RS];
    __shared__ float gt[kMapTJ];
    const int tid = threadIdx.x, lq = tid % LQ;
    const int d = J.d;
    const int S = J.S;
    const int split = (int)(blockIdx.x % S);
    const int64_t row = (int64_t)(blockIdx.x / S) * QB + tid / LQ;
    const bool live = row < J.nu;
    const int f0 = lq * F;
    float x[F];
#pragma unroll
    for (int k = 0; k < F; ++k) x[k] = (live && f0 + k < d) ? J.U[row * d + f0 + k] : 0.f;
    const float k2 = J.bscale;                 // log2(e)/eps
    const float kc = k2 / J.cost_p;            // h = c/p
    const float gk = J.gamma * k2;
    const float pm1 = J.cost_p - 1.f;
    float M = kNegBig, sum = 0.f;
    const int64_t j_lo = (int64_t)split * tps;
    const int64_t j_hi = std::min(J.nv, j_lo + tps);
    for (int64_t j0 = j_lo; j0 < j_hi; j0 += kMapTJ) {
        const int64_t nt = std::min<int64_t>(kMapTJ, j_hi - j0);
        __syncthreads();   // the previous tile is consumed
        for (int e = tid; e < kMapTJ * D; e += 256) {
            const int jj = e / D, kk = e % D;
            vt[jj * RS + (kk / F) * SEG + kk % F] = (jj < nt && kk < d) ? J.V[(j0 + jj) * d + kk] : 0.f;
        }
        if (tid < kMapTJ)
            gt[tid] = tid < nt ? (J.vpot ? J.vpot[j0 + tid] * gk : 0.f) : -INFINITY;
        __syncthreads();
        for (int jj = 0; jj < kMapTJ; ++jj) {
            const float *vj = vt + jj * RS + lq * SEG;
            float c0 = 0.f, c1 = 0.f, c2 = 0.f, c3 = 0.f;
#pragma unroll
            for (int k = 0; k < F; k += 4) {
                const f4 vv = *reinterpret_cast<const f4 *>(vj + k);
                float cp[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float a = fabsf(x[k + e] - vv[e]);
                    cp[e] = a * pow_pm1<PK>(a, pm1);
                }
                c0 += cp[0]; c1 += cp[1]; c2 += cp[2]; c3 += cp[3];
            }
            const float c = group_sum<LQ>((c0 + c1) + (c2 + c3));
            const float t = fmaf(-c, kc, gt[jj]);
            if (__builtin_amdgcn_ballot_w64(t > M)) {
                const float Mn = fmaxf(M, t);
                sum *= ex2(M - Mn);
                M = Mn;
            }
            sum += ex2(t - M);
        }
    }
    if (live && lq == 0) {
        J.part_m[(int64_t)split * J.nu + row] = M;
        J.part_s[(int64_t)split * J.nu + row] = sum;
    }
}

template <int D, int PK>
hipError_t fly_launch_t(const LseJob &j, hipStream_t s) {
    constexpr int QB = PShape<D>::QB;
    const int64_t qb = (j.nu + QB - 1) / QB;
    if (qb * j.S > 0x7fffffff) return hipErrorInvalidValue;
    timed_launch(0, pcost_lse_fly<D, PK>, dim3((unsigned)(qb * j.S)), dim3(256), 0, s, j, j.cps);
    return hipGetLastError();
}

template <int PK>
hipError_t fly_launch_pk(const LseJob &j, hipStream_t s) {
    switch (pmap_dim(j.d)) {
        case 16: return fly_launch_t<16, PK>(j, s);
        case 32: return fly_launch_t<32, PK>(j, s);
        case 48: return fly_launch_t<48, PK>(j, s);
        case 64: return fly_launch_t<64, PK>(j, s);
        case 128: return fly_launch_t<128, PK>(j, s);
        default: return fly_launch_t<256, PK>(j, s);
    }
}


template <int D, int PK>
hipError_t pmap_launch_t(const PcostMapArgs &a, hipStream_t s) {
    constexpr int QB = PShape<D>::QB;
    // queries in chunks that fit the split partials; targets split so that
    // the grid holds >= 1024 workgroups when the queries alone do not
    const int64_t qblocks_all = (a.nq + QB - 1) / QB;
    const int64_t chunk = qblocks_all >= 1024 ? a.nq : std::max<int64_t>(1, a.cap_q);
    for (int64_t q0 = 0; q0 < a.nq; q0 += chunk) {
        PcostMapArgs c = a;
        c.Xq = a.Xq + q0 * a.d;
        c.Xout = a.Xout + q0 * a.d;
        c.nq = std::min(chunk, a.nq - q0);
        const int64_t qb = (c.nq + QB - 1) / QB;
        int64_t S = 1;
        if (qb < 1024) {
            while (S * qb < 1024 && S < kMapMaxSplit) S <<= 1;
        }
        int64_t tps = (a.m + S - 1) / S;
        tps = std::max<int64_t>(2 * kMapTJ, (tps + kMapTJ - 1) / kMapTJ * kMapTJ);
        S = (a.m + tps - 1) / tps;
        if (S > 1 && (c.nq > a.cap_q || !a.pm || !a.ps || !a.pacc)) return hipErrorInvalidValue;
        timed_launch(1, pcost_map<D, PK>, dim3((unsigned)(qb * S)), dim3(256), 0, s, c, (int)S, tps);
        if (S > 1)
            hipLaunchKernelGGL((pcost_map_merge<PK>), dim3((unsigned)((c.nq * a.d + 255) / 256)), dim3(256),
                               0, s, c, (int)S, D);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int PK>
hipError_t pmap_launch_pk(const PcostMapArgs &a, hipStream_t s) {
    switch (pmap_dim(a.d)) {
        case 16: return pmap_launch_t<16, PK>(a, s);
        case 32: return pmap_launch_t<32, PK>(a, s);
        case 48: return pmap_launch_t<48, PK>(a, s);
        case 64: return pmap_launch_t<64, PK>(a, s);
        case 128: return pmap_launch_t<128, PK>(a, s);
        default: return pmap_launch_t<256, PK>(a, s);
    }
}

bool is_p15(float p) { return p == 1.5f; }

}  // namespace

int pcost_pad_dim(int d) { return pmap_dim(d); }
int64_t pcost_ldc(int64_t m) { return (m + 3) / 4 * 4; }
int64_t pcost_matrix_blocks(int64_t n, int64_t m) {
    return ((n + kCT - 1) / kCT) * ((m + kCT - 1) / kCT);
}
int pcost_map_max_split() { return kMapMaxSplit; }

hipError_t launch_pcost_matrix(const float *X, int64_t n, const float *Y, int64_t m, int d, float p,
                               float *Cm, int64_t ldc, double *part, double *sum_out,
                               hipStream_t s) {
    const int64_t col_tiles = (m + kCT - 1) / kCT;
    const int64_t blocks = pcost_matrix_blocks(n, m);
    if (blocks > 0x7fffffff || (Cm && (ldc < m || ldc % 4))) return hipErrorInvalidValue;
    // Cm == NULL: only the FP64 sum (the matrix is formed on the fly later)
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(256), 0, s, X, n, Y, m, d, p - 1.f,
                           1.f / p, col_tiles, Cm, ldc, part);
    };
    if (is_p15(p)) {
        if (Cm) go(pcost_matrix<1, true>); else go(pcost_matrix<1, false>);
    } else {
        if (Cm) go(pcost_matrix<0, true>); else go(pcost_matrix<0, false>);
    }
    hipLaunchKernelGGL(sum_f64, dim3(1), dim3(256), 0, s, part, blocks, sum_out);
    return hipGetLastError();
}

void plan_pcost_job(LseJob &j) {
    j.scale2 = 0.f;
    j.bscale = kLog2e / j.eps;
    int64_t tiles, S, per;
    if (!j.cmat) {
        // on the fly: QB rows per workgroup, columns split so that the grid
        // holds >= 2048 workgroups as far as the split partials allow
        // (kMaxSplit x max(n, m) floats: kMaxSplit max(n, m) / nu splits of
        // nu outputs), in whole tiles of kMapTJ columns.  The g-update of a
        // pair with m << n has few row tiles and needs the extra splits: at
        // 11000 x 2800 a cap of 32 left it 352 workgroups, ~1.4 waves per SIMD
        const int QBr = 256 / (pmap_dim(j.d) <= 48 ? 1 : pmap_dim(j.d) / 32);
        tiles = (j.nu + QBr - 1) / QBr;
        const int64_t cap = kMaxSplit * std::max(j.nu, j.nv) / j.nu;
        S = std::min<int64_t>(cap, std::max<int64_t>(1, (2048 + tiles - 1) / tiles));
        per = (j.nv + S - 1) / S;
        per = std::max<int64_t>(2 * kMapTJ, (per + kMapTJ - 1) / kMapTJ * kMapTJ);
        S = (j.nv + per - 1) / per;
        j.S = (int)S;
        j.cps = per;
        j.blocks = tiles * S;
        j.mblocks = (j.nu + 3) / 4;
        return;
    }
    if (!j.cmat_cols) {
        // rows of C: 4 rows (one per wave) per workgroup, >= 256 columns per
        // split, as many splits as the split partials hold (kMaxSplit max(n,
        // m) / nu), so a pair with few rows still fills the chip
        tiles = (j.nu + 3) / 4;
        S = tiles >= 2048 ? 1 : (2048 + tiles - 1) / tiles;
        S = std::min<int64_t>(S, std::max<int64_t>(1, j.nv / 256));
        S = std::min<int64_t>(S, kMaxSplit * std::max(j.nu, j.nv) / j.nu);
        per = (j.nv + S - 1) / S;
        per = (per + 3) / 4 * 4;
    } else {
        // columns of C: 256 per workgroup, >= 128 rows per split, >= 4096
        // waves in the grid; the split partials (kMaxSplit x max(n, m)
        // floats) hold up to kMaxSplit max(n, m) / m splits of m columns
        tiles = (j.nu + 255) / 256;
        const int64_t target = 4096 / kColWaves;
        S = tiles >= target ? 1 : (target + tiles - 1) / tiles;
        S = std::min<int64_t>(S, std::max<int64_t>(1, j.nv / 128));
        S = std::min<int64_t>(S, kMaxSplit * std::max(j.nu, j.nv) / j.nu);
        per = (j.nv + S - 1) / S;
    }
    S = (j.nv + per - 1) / per;
    j.S = (int)S;
    j.cps = per;
    j.blocks = tiles * S;
    // one split of rows: the partial kernel writes the potential itself;
    // otherwise the merge runs 4 outputs per workgroup
    j.mblocks = (!j.cmat_cols && S == 1) ? tiles : (j.nu + 3) / 4;
}

bool pcost_fused(const LseJob &j) { return j.cmat && !j.cmat_cols && j.S == 1; }

hipError_t launch_pcost_merge(const LseJob &j, hipStream_t s) {
    hipLaunchKernelGGL(pcost_merge, dim3((unsigned)j.mblocks), dim3(256), 0, s, j);
    return hipGetLastError();
}

bool lse_update_folds_sum(const LseJob &j) { return j.cost_p != 0.f && j.cmat && j.cmat_cols; }

hipError_t launch_pcost_partial(const LseJob &j, hipStream_t s) {
    if (j.esum_out && (!lse_update_folds_sum(j) || !j.esum_in || j.esum_n < 1)) return hipErrorInvalidValue;
    if (!j.cmat) return is_p15(j.cost_p) ? fly_launch_pk<1>(j, s) : fly_launch_pk<0>(j, s);
    if (j.blocks > 0x7fffffff || j.ldc % 4) return hipErrorInvalidValue;
    if (pcost_fused(j))
        timed_launch(0, pcost_lse_rows<true>, dim3((unsigned)j.blocks), dim3(256), 0, s, j);
    else if (!j.cmat_cols)
        timed_launch(0, pcost_lse_rows<false>, dim3((unsigned)j.blocks), dim3(256), 0, s, j);
    else
        timed_launch(0, pcost_lse_cols, dim3((unsigned)j.blocks), dim3(64 * kColWaves), 0, s, j);
    return hipGetLastError();
}

hipError_t launch_pcost_map(const PcostMapArgs &a, hipStream_t s) {
    if (a.nq <= 0) return hipSuccess;
    return is_p15(a.p) ? pmap_launch_pk<1>(a, s) : pmap_launch_pk<0>(a, s);
}

}  // namespace pot
