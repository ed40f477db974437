// gfx950 kernels of the progressive entropic OT hot path.
//
// Potential update (f- and g-update of Alg. 1, the soft-min of Sec. 2):
//   pot_i = eps*log w_i + |u_i|^2 - eps*ln2 * log2 sum_j 2^{t_ij},
//   t_ij  = (2 log2 e / eps) <u_i, v_j> + (gamma*vpot_j - |v_j|^2) log2 e / eps,
// which is eps log w_i - eps LSE_j((vpot_j - |u_i - v_j|^2)/eps) with the cost
// expanded as |u|^2 + |v|^2 - 2<u, v>.  The cross term runs on MFMA; the
// n x m cost is never stored: a workgroup keeps its rows in registers,
// streams column tiles through LDS and keeps a running (max, sum) per lane.
//
// Layout of a 16x16 MFMA tile.  The column tile is the A operand and the
// rows are the B operand, so the accumulator holds S^T: lane l, register r
// holds S[i = l%16][j = 4*(l/16) + r].  Each lane thus owns one row i and the
// per-row reduction over j stays inside the lane until a final 4-way merge
// across the lane groups l/16.  The feature index k of MFMA step s in lane
// group q is q*(D/4) + s, so each lane reads D/4 contiguous features.
//
// Entropic map (eq. Tent, barycentric projection): the same S^T tile gives
// p_ij = 2^{t_ij - max_i}; with that layout p is already the B operand of the
// second product O^T = Y^T P^T (the k index of step (sub, r) in group q is
// j = 16 sub + 4q + r), so the projection needs no register shuffle.

#include "progot_internal.h"

#include <cmath>

namespace pot {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kNegBig = -1.0e30f;  // finite "minus infinity" of running maxima

__device__ __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int D> struct Tile {
    static constexpr int BN = D >= 256 ? 32 : 64;   // columns per LDS tile
    static constexpr int NSUB = BN / 16;           // 16-column subtiles
    static constexpr int KD = D / 4;               // features per lane group
    static constexpr int STRIDE = D + 4;           // padded LDS row (floats)
    static constexpr int NV4 = BN * D / 4;         // float4 per tile
    static constexpr int PER_T = (NV4 + 255) / 256;
};

// Load one BN x D column tile (rows j0.., zero-padded beyond nv and beyond
// feature d) into registers; thread t takes float4 slots t, t+256, ...
template <int D>
__device__ __forceinline__ void tile_fetch(const float *__restrict__ V, int64_t nv, int d,
                                           int64_t j0, f4 (&pre)[Tile<D>::PER_T]) {
    using T = Tile<D>;
#pragma unroll
    for (int r = 0; r < T::PER_T; ++r) {
        const int e = threadIdx.x + 256 * r;
        f4 v = {0.f, 0.f, 0.f, 0.f};
        if (e < T::NV4) {
            const int row = e / (D / 4);
            const int c = (e % (D / 4)) * 4;
            const int64_t j = j0 + row;
            if (j < nv) {
                if (d == D) {
                    v = *reinterpret_cast<const f4 *>(V + j * D + c);
                } else {
                    const float *p = V + j * d;
                    v.x = c + 0 < d ? p[c + 0] : 0.f;
                    v.y = c + 1 < d ? p[c + 1] : 0.f;
                    v.z = c + 2 < d ? p[c + 2] : 0.f;
                    v.w = c + 3 < d ? p[c + 3] : 0.f;
                }
            }
        }
        pre[r] = v;
    }
}

template <int D>
__device__ __forceinline__ void tile_store(float *__restrict__ lds, const f4 (&pre)[Tile<D>::PER_T]) {
    using T = Tile<D>;
#pragma unroll
    for (int r = 0; r < T::PER_T; ++r) {
        const int e = threadIdx.x + 256 * r;
        if (e < T::NV4) {
            const int row = e / (D / 4);
            const int c = (e % (D / 4)) * 4;
            *reinterpret_cast<f4 *>(lds + row * T::STRIDE + c) = pre[r];
        }
    }
}

// The lane's D/4 features of row `row` of U (zero beyond nu and d).
template <int D>
__device__ __forceinline__ void row_fetch(const float *__restrict__ U, int64_t nu, int d,
                                          int64_t row, int lq, float (&u)[D / 4]) {
    constexpr int KD = D / 4;
    const int c0 = lq * KD;
    if (row < nu && d == D) {
        const f4 *p = reinterpret_cast<const f4 *>(U + row * D + c0);
#pragma unroll
        for (int k = 0; k < KD / 4; ++k) {
            f4 v = p[k];
            u[4 * k + 0] = v.x; u[4 * k + 1] = v.y; u[4 * k + 2] = v.z; u[4 * k + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < KD; ++k)
            u[k] = (row < nu && c0 + k < d) ? U[row * d + c0 + k] : 0.f;
    }
}

// Partial log-sum-exp of t_ij over one column split, for ROWS = 64*QB rows.
// Output: part_m/part_s[split*nu + i] = (max, sum 2^{t - max}) in log2 units.
template <int D, int QB>
__global__ __launch_bounds__(256) void lse_partial_f32(
    const float *__restrict__ U, int64_t nu, const float *__restrict__ V,
    const float *__restrict__ vsq, const float *__restrict__ vpot, int64_t nv, int d,
    float gamma, float scale2, float bscale, int S, int64_t cols_per_split,
    float *__restrict__ part_m, float *__restrict__ part_s) {
    using T = Tile<D>;
    constexpr int ROWS = 64 * QB;
    __shared__ float vt[2][T::BN * T::STRIDE];
    __shared__ float bt[2][T::BN];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int split = blockIdx.x % S;   // consecutive blocks -> different XCDs -> one split each
    const int64_t tile = blockIdx.x / S;
    const int64_t row0 = tile * ROWS + wave * (QB * 16);

    float ub[QB][T::KD];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) row_fetch<D>(U, nu, d, row0 + qb * 16 + li, lq, ub[qb]);

    float run_m[QB], run_s[QB];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) { run_m[qb] = kNegBig; run_s[qb] = 0.f; }

    const int64_t c0 = (int64_t)split * cols_per_split;
    const int64_t c1 = c0 + cols_per_split < nv ? c0 + cols_per_split : nv;
    const int ntiles = c0 < c1 ? (int)((c1 - c0 + T::BN - 1) / T::BN) : 0;

    f4 pre[T::PER_T];
    float bpre = 0.f;
    auto fetch_beta = [&](int64_t j0) {
        if (tid < T::BN) {
            const int64_t j = j0 + tid;
            bpre = j < c1 ? ((vpot ? gamma * vpot[j] : 0.f) - vsq[j]) * bscale : -INFINITY;
        }
    };
    if (ntiles > 0) {
        tile_fetch<D>(V, c1, d, c0, pre);
        fetch_beta(c0);
        tile_store<D>(vt[0], pre);
        if (tid < T::BN) bt[0][tid] = bpre;
    }
    __syncthreads();

    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        const bool more = t + 1 < ntiles;
        if (more) {
            const int64_t jn = c0 + (int64_t)(t + 1) * T::BN;
            tile_fetch<D>(V, c1, d, jn, pre);
            fetch_beta(jn);
        }
        const float *vb = vt[buf];
        f4 acc[QB][T::NSUB];
#pragma unroll
        for (int sub = 0; sub < T::NSUB; ++sub) {
            float a[T::KD];
            const f4 *ap = reinterpret_cast<const f4 *>(vb + (sub * 16 + li) * T::STRIDE + lq * T::KD);
#pragma unroll
            for (int k = 0; k < T::KD / 4; ++k) {
                f4 v = ap[k];
                a[4 * k + 0] = v.x; a[4 * k + 1] = v.y; a[4 * k + 2] = v.z; a[4 * k + 3] = v.w;
            }
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) {
                f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int k = 0; k < T::KD; ++k) c = mfma4(a[k], ub[qb][k], c);
                acc[qb][sub] = c;
            }
        }
        f4 beta[T::NSUB];
#pragma unroll
        for (int sub = 0; sub < T::NSUB; ++sub)
            beta[sub] = *reinterpret_cast<const f4 *>(&bt[buf][sub * 16 + lq * 4]);
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            float tv[T::NSUB * 4];
            float mx = kNegBig;
#pragma unroll
            for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float x = fmaf(acc[qb][sub][r], scale2, beta[sub][r]);
                    tv[sub * 4 + r] = x;
                    mx = fmaxf(mx, x);
                }
            const float mn = fmaxf(run_m[qb], mx);
            float s = 0.f;
#pragma unroll
            for (int e = 0; e < T::NSUB * 4; ++e) s += ex2(tv[e] - mn);
            run_s[qb] = fmaf(run_s[qb], ex2(run_m[qb] - mn), s);
            run_m[qb] = mn;
        }
        if (more) {
            tile_store<D>(vt[buf ^ 1], pre);
            if (tid < T::BN) bt[buf ^ 1][tid] = bpre;
        }
        __syncthreads();
    }

#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        float m = run_m[qb], s = run_s[qb];
#pragma unroll
        for (int off = 16; off <= 32; off <<= 1) {
            const float mo = __shfl_xor(m, off);
            const float so = __shfl_xor(s, off);
            const float mn = fmaxf(m, mo);
            s = s * ex2(m - mn) + so * ex2(mo - mn);
            m = mn;
        }
        const int64_t row = row0 + qb * 16 + li;
        if (lq == 0 && row < nu) {
            part_m[split * nu + row] = m;
            part_s[split * nu + row] = s;
        }
    }
}

__device__ __forceinline__ float block_sum_256(float v, float *red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
#pragma unroll
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    return red[0];
}

// Merge the split partials into the potential and the error partial
// w_i |exp((pot_old_i - pot_i)/eps) - 1|, which is |(P 1)_i - w_i| for the
// coupling of (pot_old, vpot): row sums of the previous iterate.
__global__ __launch_bounds__(256) void lse_merge(
    const float *__restrict__ part_m, const float *__restrict__ part_s, int S, int64_t nu,
    const float *__restrict__ usq, const float *__restrict__ logw, float eps,
    const float *__restrict__ pot_old, float *__restrict__ pot_out, float *__restrict__ err_part) {
    __shared__ float red[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float e = 0.f;
    if (i < nu) {
        float M = kNegBig;
        for (int s = 0; s < S; ++s) M = fmaxf(M, part_m[s * nu + i]);
        float sum = 0.f;
        for (int s = 0; s < S; ++s) sum += part_s[s * nu + i] * exp2f(part_m[s * nu + i] - M);
        const float L = M + log2f(sum);
        const float lw = logw[i];
        const float pot = fmaf(eps, lw, usq[i]) - eps * kLn2 * L;
        if (pot_old) e = expf(lw) * fabsf(expm1f((pot_old[i] - pot) / eps));
        pot_out[i] = pot;
    }
    if (pot_old) {
        const float tot = block_sum_256(e, red);
        if (threadIdx.x == 0) err_part[blockIdx.x] = tot;
    }
}

__global__ __launch_bounds__(256) void sum_f32(const float *__restrict__ part, int n, float *__restrict__ out) {
    __shared__ float red[256];
    float v = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) v += part[i];
    const float tot = block_sum_256(v, red);
    if (threadIdx.x == 0) out[0] = tot;
}

// Squared norms (FP64 accumulation), optional BF16 copy.
__global__ __launch_bounds__(256) void cloud_norms(const float *__restrict__ X, int64_t n, int d,
                                                   float *__restrict__ sqn, __bf16 *__restrict__ lp) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float *x = X + i * d;
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        const double v = x[k];
        s += v * v;
        if (lp) lp[i * d + k] = (__bf16)x[k];
    }
    sqn[i] = (float)s;
}

// Per-block FP64 sums of every feature and of |x|^2 over a contiguous row range.
__global__ __launch_bounds__(256) void cloud_stats(const float *__restrict__ X, int64_t n, int d,
                                                   const float *__restrict__ sqn, int64_t rows_per_blk,
                                                   double *__restrict__ part) {
    __shared__ double red[256];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = r0 + rows_per_blk < n ? r0 + rows_per_blk : n;
    for (int f = threadIdx.x; f < d; f += 256) {
        double s = 0.0;
        for (int64_t r = r0; r < r1; ++r) s += X[r * d + f];
        part[(int64_t)blockIdx.x * (d + 1) + f] = s;
    }
    double q = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) q += sqn[r];
    red[threadIdx.x] = q;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * (d + 1) + d] = red[0];
}

// Fold nblk x (d+1) partials into the first row, fixed order.
__global__ __launch_bounds__(256) void stats_fold(double *__restrict__ part, int nblk, int d) {
    for (int f = threadIdx.x; f <= d; f += 256) {
        double s = 0.0;
        for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * (d + 1) + f];
        part[f] = s;
    }
}

__global__ __launch_bounds__(256) void log_weights(const float *__restrict__ w, int64_t n, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = w ? logf(w[i]) : -logf((float)n);
}

__global__ __launch_bounds__(256) void scale_vec(const float *__restrict__ in, float gamma, int64_t n,
                                                 float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = in ? gamma * in[i] : 0.f;
}

// Entropic map + McCann-type step for ROWS = 64*QB queries per workgroup.
template <int D, int QB>
__global__ __launch_bounds__(256) void entropic_map_f32(
    const float *Xq, int64_t nq, int d, const float *__restrict__ Y,
    const float *__restrict__ ysq, const float *__restrict__ g, int64_t m, float scale2,
    float bscale, float alpha, float *Xout, float *__restrict__ out_sqn, __bf16 *__restrict__ out_lp) {
    using T = Tile<D>;
    constexpr int ROWS = 64 * QB;
    constexpr int NDB = D / 16;   // 16-feature blocks of the output
    __shared__ float vt[2][T::BN * T::STRIDE];
    __shared__ float bt[2][T::BN];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * ROWS + wave * (QB * 16);

    float ub[QB][T::KD];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) row_fetch<D>(Xq, nq, d, row0 + qb * 16 + li, lq, ub[qb]);

    float run_m[QB], run_l[QB];
    f4 o[QB][NDB];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        run_m[qb] = kNegBig;
        run_l[qb] = 0.f;
#pragma unroll
        for (int db = 0; db < NDB; ++db) o[qb][db] = f4{0.f, 0.f, 0.f, 0.f};
    }

    const int ntiles = (int)((m + T::BN - 1) / T::BN);
    f4 pre[T::PER_T];
    float bpre = 0.f;
    auto fetch_beta = [&](int64_t j0) {
        if (tid < T::BN) {
            const int64_t j = j0 + tid;
            bpre = j < m ? (g[j] - ysq[j]) * bscale : -INFINITY;
        }
    };
    if (ntiles > 0) {
        tile_fetch<D>(Y, m, d, 0, pre);
        fetch_beta(0);
        tile_store<D>(vt[0], pre);
        if (tid < T::BN) bt[0][tid] = bpre;
    }
    __syncthreads();

    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        const bool more = t + 1 < ntiles;
        if (more) {
            const int64_t jn = (int64_t)(t + 1) * T::BN;
            tile_fetch<D>(Y, m, d, jn, pre);
            fetch_beta(jn);
        }
        const float *vb = vt[buf];
        f4 acc[QB][T::NSUB];
#pragma unroll
        for (int sub = 0; sub < T::NSUB; ++sub) {
            float a[T::KD];
            const f4 *ap = reinterpret_cast<const f4 *>(vb + (sub * 16 + li) * T::STRIDE + lq * T::KD);
#pragma unroll
            for (int k = 0; k < T::KD / 4; ++k) {
                f4 v = ap[k];
                a[4 * k + 0] = v.x; a[4 * k + 1] = v.y; a[4 * k + 2] = v.z; a[4 * k + 3] = v.w;
            }
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) {
                f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int k = 0; k < T::KD; ++k) c = mfma4(a[k], ub[qb][k], c);
                acc[qb][sub] = c;
            }
        }
        f4 beta[T::NSUB];
#pragma unroll
        for (int sub = 0; sub < T::NSUB; ++sub)
            beta[sub] = *reinterpret_cast<const f4 *>(&bt[buf][sub * 16 + lq * 4]);
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            float p[T::NSUB * 4];
            float mx = kNegBig;
#pragma unroll
            for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float x = fmaf(acc[qb][sub][r], scale2, beta[sub][r]);
                    p[sub * 4 + r] = x;
                    mx = fmaxf(mx, x);
                }
            mx = fmaxf(mx, __shfl_xor(mx, 16));
            mx = fmaxf(mx, __shfl_xor(mx, 32));
            const float mn = fmaxf(run_m[qb], mx);
            const float c = ex2(run_m[qb] - mn);
            run_m[qb] = mn;
            float s = 0.f;
#pragma unroll
            for (int e = 0; e < T::NSUB * 4; ++e) {
                p[e] = ex2(p[e] - mn);
                s += p[e];
            }
            run_l[qb] = fmaf(run_l[qb], c, s);
#pragma unroll
            for (int db = 0; db < NDB; ++db) o[qb][db] *= c;
#pragma unroll
            for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float *yrow = vb + (sub * 16 + 4 * lq + r) * T::STRIDE + li;
#pragma unroll
                    for (int db = 0; db < NDB; ++db)
                        o[qb][db] = mfma4(yrow[db * 16], p[sub * 4 + r], o[qb][db]);
                }
        }
        if (more) {
            tile_store<D>(vt[buf ^ 1], pre);
            if (tid < T::BN) bt[buf ^ 1][tid] = bpre;
        }
        __syncthreads();
    }

#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        float l = run_l[qb];
        l += __shfl_xor(l, 16);
        l += __shfl_xor(l, 32);
        const float inv = 1.f / l;
        const int64_t row = row0 + qb * 16 + li;
        double sq = 0.0;
        if (row < nq) {
#pragma unroll
            for (int db = 0; db < NDB; ++db) {
                const int f0 = db * 16 + 4 * lq;
                if (f0 >= d) continue;
                float xo[4], xn[4];
                if (f0 + 3 < d && (d & 3) == 0) {
                    f4 v = *reinterpret_cast<const f4 *>(Xq + row * d + f0);
                    xo[0] = v.x; xo[1] = v.y; xo[2] = v.z; xo[3] = v.w;
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) xo[r] = f0 + r < d ? Xq[row * d + f0 + r] : 0.f;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    xn[r] = (1.f - alpha) * xo[r] + alpha * (o[qb][db][r] * inv);
                    if (f0 + r < d) sq += (double)xn[r] * xn[r];
                }
                if (f0 + 3 < d && (d & 3) == 0) {
                    *reinterpret_cast<f4 *>(Xout + row * d + f0) = f4{xn[0], xn[1], xn[2], xn[3]};
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (f0 + r < d) Xout[row * d + f0 + r] = xn[r];
                }
                if (out_lp) {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (f0 + r < d) out_lp[row * d + f0 + r] = (__bf16)xn[r];
                }
            }
        }
        sq += __shfl_xor(sq, 16);
        sq += __shfl_xor(sq, 32);
        if (out_sqn && lq == 0 && row < nq) out_sqn[row] = (float)sq;
    }
}

// FP64 check, one thread per "row" u: r_u = sum_v exp((pu_u + pv_v - |u - v|^2)/eps)
// with the distance by direct differences in FP64.  Per-block partials of
// (sum |r_u - w_u|, sum r_u, sum pu_u w_u).
constexpr int kChkTile = 32;
__global__ __launch_bounds__(256) void fp64_rowsums(
    const float *__restrict__ U, int64_t nu, const float *__restrict__ V, int64_t nv, int d,
    const float *__restrict__ pu, const float *__restrict__ pv, const float *__restrict__ w_in,
    double eps, double *__restrict__ part) {
    __shared__ float vt[kChkTile * 256];
    __shared__ double vp[kChkTile];
    __shared__ double red[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool live = i < nu;
    const double fi = live ? (double)pu[i] : 0.0;
    double rsum = 0.0;
    for (int64_t j0 = 0; j0 < nv; j0 += kChkTile) {
        const int nt = (int)(nv - j0 < kChkTile ? nv - j0 : kChkTile);
        __syncthreads();
        for (int e = threadIdx.x; e < nt * d; e += 256) vt[e] = V[j0 * d + e];
        if ((int)threadIdx.x < nt) vp[threadIdx.x] = pv[j0 + threadIdx.x];
        __syncthreads();
        double dist[kChkTile];
#pragma unroll
        for (int jj = 0; jj < kChkTile; ++jj) dist[jj] = 0.0;
        if (live) {
            for (int k = 0; k < d; ++k) {
                const double x = U[i * d + k];
#pragma unroll
                for (int jj = 0; jj < kChkTile; ++jj) {
                    if (jj < nt) {
                        const double df = x - (double)vt[jj * d + k];
                        dist[jj] = fma(df, df, dist[jj]);
                    }
                }
            }
#pragma unroll
            for (int jj = 0; jj < kChkTile; ++jj)
                if (jj < nt) rsum += exp((fi + vp[jj] - dist[jj]) / eps);
        }
    }
    const double w = live ? (w_in ? (double)w_in[i] : 1.0 / (double)nu) : 0.0;
    const double vals[3] = {live ? fabs(rsum - w) : 0.0, rsum, fi * w};
    for (int q = 0; q < 3; ++q) {
        __syncthreads();
        red[threadIdx.x] = vals[q];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 3 + q] = red[0];
    }
}

template <int D, int QB>
hipError_t lse_launch_t(const LseArgs &a, int S, int64_t cps, float scale2, float bscale, hipStream_t s) {
    const int64_t tiles = (a.nu + 64 * QB - 1) / (64 * QB);
    const dim3 grid((unsigned)(tiles * S));
    hipLaunchKernelGGL((lse_partial_f32<D, QB>), grid, dim3(256), 0, s, a.U, a.nu, a.V, a.vsq,
                       a.vpot, a.nv, a.d, a.gamma, scale2, bscale, S, cps, a.part_m, a.part_s);
    return hipGetLastError();
}

template <int D, int QB>
hipError_t map_launch_t(const MapArgs &a, float scale2, float bscale, hipStream_t s) {
    const int64_t tiles = (a.nq + 64 * QB - 1) / (64 * QB);
    hipLaunchKernelGGL((entropic_map_f32<D, QB>), dim3((unsigned)tiles), dim3(256), 0, s, a.Xq,
                       a.nq, a.d, a.Y, a.ysq, a.g, a.m, scale2, bscale, a.alpha, a.Xout,
                       a.out_sqn, (__bf16 *)a.out_lp);
    return hipGetLastError();
}

int padded_dim(int d) {
    if (d <= 16) return 16;
    if (d <= 32) return 32;
    if (d <= 64) return 64;
    if (d <= 128) return 128;
    return 256;
}

int qb_for(int D) { return D >= 256 ? 1 : 2; }

}  // namespace

int lse_rows_per_block(int d) { return 64 * qb_for(padded_dim(d)); }
int map_rows_per_block(int d) { return 64 * qb_for(padded_dim(d)); }

hipError_t launch_lse_update(const LseArgs &a, hipStream_t s, int *n_err_part) {
    const int D = padded_dim(a.d);
    const int rows = lse_rows_per_block(a.d);
    const int64_t tiles = (a.nu + rows - 1) / rows;
    // Split the columns so that the grid holds >= ~1024 workgroups (4 per CU),
    // keeping >= 256 columns per split.
    int64_t S = tiles >= 1024 ? 1 : (1024 + tiles - 1) / tiles;
    const int64_t max_by_cols = (a.nv + 255) / 256;
    if (S > max_by_cols) S = max_by_cols;
    if (S > kMaxSplit) S = kMaxSplit;
    if (S < 1) S = 1;
    const int64_t cps = (a.nv + S - 1) / S;
    const float scale2 = 2.f * kLog2e / a.eps;
    const float bscale = kLog2e / a.eps;
    hipError_t e;
    const int64_t slot = timing_begin(0, s);
    switch (D) {
        case 16: e = lse_launch_t<16, 2>(a, (int)S, cps, scale2, bscale, s); break;
        case 32: e = lse_launch_t<32, 2>(a, (int)S, cps, scale2, bscale, s); break;
        case 64: e = lse_launch_t<64, 2>(a, (int)S, cps, scale2, bscale, s); break;
        case 128: e = lse_launch_t<128, 2>(a, (int)S, cps, scale2, bscale, s); break;
        default: e = lse_launch_t<256, 1>(a, (int)S, cps, scale2, bscale, s); break;
    }
    timing_end(slot, s);
    if (e != hipSuccess) return e;
    const int nb = (int)((a.nu + 255) / 256);
    hipLaunchKernelGGL(lse_merge, dim3(nb), dim3(256), 0, s, a.part_m, a.part_s, (int)S, a.nu,
                       a.usq, a.logw, a.eps, a.pot_old, a.pot_out, a.err_part);
    if (n_err_part) *n_err_part = a.pot_old ? nb : 0;
    return hipGetLastError();
}

hipError_t launch_sum_f32(const float *part, int n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(sum_f32, dim3(1), dim3(256), 0, s, part, n, out);
    return hipGetLastError();
}

int cloud_stat_blocks(int64_t n) {
    const int64_t b = (n + 1023) / 1024;
    return (int)(b < 256 ? (b < 1 ? 1 : b) : 256);
}

hipError_t launch_cloud_prep(const float *X, int64_t n, int d, float *sqn, void *lp,
                             double *stats_part, int nblk, hipStream_t s) {
    hipLaunchKernelGGL(cloud_norms, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, n, d,
                       sqn, (__bf16 *)lp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !stats_part) return e;
    const int64_t rpb = (n + nblk - 1) / nblk;
    hipLaunchKernelGGL(cloud_stats, dim3(nblk), dim3(256), 0, s, X, n, d, sqn, rpb, stats_part);
    hipLaunchKernelGGL(stats_fold, dim3(1), dim3(256), 0, s, stats_part, nblk, d);
    return hipGetLastError();
}

hipError_t launch_log_weights(const float *w, int64_t n, float *logw, hipStream_t s) {
    hipLaunchKernelGGL(log_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, n, logw);
    return hipGetLastError();
}

hipError_t launch_scale(const float *in, float gamma, int64_t n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(scale_vec, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, gamma, n, out);
    return hipGetLastError();
}

hipError_t launch_entropic_map(const MapArgs &a, hipStream_t s) {
    if (a.nq == 0) return hipSuccess;
    const float scale2 = 2.f * kLog2e / a.eps;
    const float bscale = kLog2e / a.eps;
    const int64_t slot = timing_begin(1, s);
    hipError_t e;
    switch (padded_dim(a.d)) {
        case 16: e = map_launch_t<16, 2>(a, scale2, bscale, s); break;
        case 32: e = map_launch_t<32, 2>(a, scale2, bscale, s); break;
        case 64: e = map_launch_t<64, 2>(a, scale2, bscale, s); break;
        case 128: e = map_launch_t<128, 2>(a, scale2, bscale, s); break;
        default: e = map_launch_t<256, 1>(a, scale2, bscale, s); break;
    }
    timing_end(slot, s);
    return e;
}

int fp64_check_blocks(int64_t n) { return (int)((n + 255) / 256); }

hipError_t launch_fp64_check(const float *X, int64_t n, const float *Y, int64_t m, int d,
                             const float *f, const float *g, const float *a,
                             const float *b, float eps, double *part_rows,
                             double *part_cols, hipStream_t s) {
    hipLaunchKernelGGL(fp64_rowsums, dim3(fp64_check_blocks(n)), dim3(256), 0, s, X, n, Y, m, d, f,
                       g, a, (double)eps, part_rows);
    hipLaunchKernelGGL(fp64_rowsums, dim3(fp64_check_blocks(m)), dim3(256), 0, s, Y, m, X, n, d, g,
                       f, b, (double)eps, part_cols);
    return hipGetLastError();
}

}  // namespace pot
