// BF16 forms of the fused cost + log-sum-exp kernel and of the entropic-map
// kernel (gfx950, v_mfma_f32_16x16x32_bf16).
//
// Only the cross term <u_i, v_j> changes arithmetic: its operands are BF16
// copies (round to nearest even) of the FP32 clouds, accumulated in FP32.
// With NPART = 2 each value is split as hi + lo (hi = bf16(x), lo =
// bf16(x - hi)) and the cross term is hi*hi + hi*lo + lo*hi: three products
// whose error is ~2^-16 relative instead of 2^-8.  Norms, the log-sum-exp,
// potentials and marginal errors stay FP32, as in the FP32 form.
//
// Shadow layouts (device, written by cloud_norms / bf16_transpose):
//   rows:        [hi | lo], each n x D bf16, D = padded dimension, zero padded
//   transposed:  [hi | lo], each D x mp bf16 (mp = m rounded up to 64), used
//                as the A operand of the projection product.
//
// MFMA 16x16x32 bf16: lane l holds A[l%16][8(l/16)..+7] and
// B[8(l/16)..+7][l%16]; the accumulator holds D[4(l/16)+r][l%16].  As in the
// FP32 kernels the column tile is the A operand, so lane l owns row i = l%16.
// Lane group q holds the features [q D/4, (q+1) D/4); MFMA step s uses its
// features q D/4 + 8s .. + 7 (the k index 8q + e maps to feature
// q D/4 + 8s + e on both operands).

#include "progot_internal.h"
#include "progot_device.h"

namespace pot {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f4 mfma_bf(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf8 bf8_zero() { return __builtin_bit_cast(bf8, u4{0u, 0u, 0u, 0u}); }

template <int D, int NPART> struct TileH {
    static constexpr int BN = (D * NPART >= 512) ? 32 : 64;  // columns per LDS tile
    static constexpr int NSUB = BN / 16;
    static constexpr int KS = D / 32;        // MFMA k-steps over the features
    static constexpr int KL = D / 4;         // features per lane group
    static constexpr int STRIDE = D + 8;     // bf16 per LDS row (16-byte pad)
    static constexpr int NCH = BN * D / 8;   // 16-byte chunks per part
    static constexpr int PER_T = (NCH + 255) / 256;
};

// Partial log-sum-exp over one column split (BF16 cross term).
template <int D, int QB, int NPART>
__global__ __launch_bounds__(256) void lse_partial_bf16(
    const __bf16 *__restrict__ Ulp, int64_t nu, const __bf16 *__restrict__ Vlp, int64_t nv,
    const float *__restrict__ vsq, const float *__restrict__ vpot, float gamma, float scale2,
    float bscale, int S, int64_t cols_per_split, float *__restrict__ part_m,
    float *__restrict__ part_s) {
    using T = TileH<D, NPART>;
    constexpr int ROWS = 64 * QB;
    __shared__ __bf16 vt[2][NPART][T::BN * T::STRIDE];
    __shared__ float bt[2][T::BN];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int split = blockIdx.x % S;
    const int64_t tile = blockIdx.x / S;
    const int64_t row0 = tile * ROWS + wave * (QB * 16);

    bf8 ub[QB][NPART][T::KS];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        const int64_t row = row0 + qb * 16 + li;
#pragma unroll
        for (int p = 0; p < NPART; ++p)
#pragma unroll
            for (int s = 0; s < T::KS; ++s)
                ub[qb][p][s] = row < nu ? *reinterpret_cast<const bf8 *>(
                                              Ulp + (int64_t)p * nu * D + row * D + lq * T::KL + 8 * s)
                                        : bf8_zero();
    }

    float run_m[QB], run_s[QB];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) { run_m[qb] = kNegBig; run_s[qb] = 0.f; }

    const int64_t c0 = (int64_t)split * cols_per_split;
    const int64_t c1 = c0 + cols_per_split < nv ? c0 + cols_per_split : nv;
    const int ntiles = c0 < c1 ? (int)((c1 - c0 + T::BN - 1) / T::BN) : 0;

    u4 pre[NPART][T::PER_T];
    float bpre = 0.f;
    auto fetch = [&](int64_t j0) {
#pragma unroll
        for (int p = 0; p < NPART; ++p)
#pragma unroll
            for (int r = 0; r < T::PER_T; ++r) {
                const int c = tid + 256 * r;
                u4 v = {0u, 0u, 0u, 0u};
                if (c < T::NCH) {
                    const int row = c / (D / 8);
                    const int col = (c % (D / 8)) * 8;
                    const int64_t j = j0 + row;
                    if (j < c1) v = *reinterpret_cast<const u4 *>(Vlp + (int64_t)p * nv * D + j * D + col);
                }
                pre[p][r] = v;
            }
        if (tid < T::BN) {
            const int64_t j = j0 + tid;
            bpre = j < c1 ? ((vpot ? gamma * vpot[j] : 0.f) - vsq[j]) * bscale : -INFINITY;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < NPART; ++p)
#pragma unroll
            for (int r = 0; r < T::PER_T; ++r) {
                const int c = tid + 256 * r;
                if (c < T::NCH) {
                    const int row = c / (D / 8);
                    const int col = (c % (D / 8)) * 8;
                    *reinterpret_cast<u4 *>(&vt[buf][p][row * T::STRIDE + col]) = pre[p][r];
                }
            }
        if (tid < T::BN) bt[buf][tid] = bpre;
    };

    if (ntiles > 0) {
        fetch(c0);
        store(0);
    }
    __syncthreads();

    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        const bool more = t + 1 < ntiles;
        if (more) fetch(c0 + (int64_t)(t + 1) * T::BN);
        // k outer, (column subtile, row block) inner: NSUB x QB independent
        // accumulation chains keep the MFMA pipe busy.
        f4 acc[QB][T::NSUB];
#pragma unroll
        for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) acc[qb][sub] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < T::KS; ++s) {
            bf8 a[NPART][T::NSUB];
#pragma unroll
            for (int p = 0; p < NPART; ++p)
#pragma unroll
                for (int sub = 0; sub < T::NSUB; ++sub)
                    a[p][sub] = *reinterpret_cast<const bf8 *>(
                        &vt[buf][p][(sub * 16 + li) * T::STRIDE + lq * T::KL + 8 * s]);
#pragma unroll
            for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
                for (int qb = 0; qb < QB; ++qb) {
                    acc[qb][sub] = mfma_bf(a[0][sub], ub[qb][0][s], acc[qb][sub]);
                    if constexpr (NPART == 2) {
                        acc[qb][sub] = mfma_bf(a[0][sub], ub[qb][1][s], acc[qb][sub]);
                        acc[qb][sub] = mfma_bf(a[1][sub], ub[qb][0][s], acc[qb][sub]);
                    }
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
        if (more) store(buf ^ 1);
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

// Entropic map + McCann-type step, BF16 cross term and a BF16 projection
// product P (rounded) x (Y_hi + Y_lo); the normaliser sums the rounded P, so
// T is an exact convex combination of the targets with perturbed weights.
constexpr int kMapBN = 32;

template <int D, int QB, int NPART>
__global__ __launch_bounds__(256) void entropic_map_bf16(
    const float *Xq, int64_t nq, int d, const __bf16 *__restrict__ Ylp,
    const __bf16 *__restrict__ YTlp, int64_t m, int64_t mp, const float *__restrict__ ysq,
    const float *__restrict__ g, float scale2, float bscale, float alpha, float *Xout,
    float *__restrict__ out_sqn) {
    constexpr int BN = kMapBN;
    constexpr int KS = D / 32, KL = D / 4, STRIDE = D + 8;
    constexpr int TSTRIDE = BN + 8;
    constexpr int NDB = D / 16;
    constexpr int ROWS = 64 * QB;
    constexpr int NCH = BN * D / 8;            // row-major chunks per part
    constexpr int PER_T = (NCH + 255) / 256;
    constexpr int NCHT = D * BN / 8;           // transposed chunks per part
    constexpr int PER_TT = (NCHT + 255) / 256;
    __shared__ __bf16 yr[2][NPART][BN * STRIDE];
    __shared__ __bf16 ytr[2][2][D * TSTRIDE];
    __shared__ float bt[2][BN];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * ROWS + wave * (QB * 16);

    // queries: FP32 rows -> hi (+ lo) BF16 B operands
    bf8 ub[QB][NPART][KS];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        float u[KL];
        row_fetch<D>(Xq, nq, d, row0 + qb * 16 + li, lq, u);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            bf8 h, l;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const __bf16 hv = (__bf16)u[8 * s + e];
                h[e] = hv;
                l[e] = (__bf16)(u[8 * s + e] - (float)hv);
            }
            ub[qb][0][s] = h;
            if constexpr (NPART == 2) ub[qb][1][s] = l;
        }
    }

    float run_m[QB], run_l[QB];
    f4 o[QB][NDB];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        run_m[qb] = kNegBig;
        run_l[qb] = 0.f;
#pragma unroll
        for (int db = 0; db < NDB; ++db) o[qb][db] = f4{0.f, 0.f, 0.f, 0.f};
    }

    const int ntiles = (int)((m + BN - 1) / BN);
    u4 pre[NPART][PER_T];
    u4 pret[2][PER_TT];
    float bpre = 0.f;
    auto fetch = [&](int64_t j0) {
#pragma unroll
        for (int p = 0; p < NPART; ++p)
#pragma unroll
            for (int r = 0; r < PER_T; ++r) {
                const int c = tid + 256 * r;
                u4 v = {0u, 0u, 0u, 0u};
                if (c < NCH) {
                    const int row = c / (D / 8);
                    const int col = (c % (D / 8)) * 8;
                    const int64_t j = j0 + row;
                    if (j < m) v = *reinterpret_cast<const u4 *>(Ylp + (int64_t)p * m * D + j * D + col);
                }
                pre[p][r] = v;
            }
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int r = 0; r < PER_TT; ++r) {
                const int c = tid + 256 * r;
                u4 v = {0u, 0u, 0u, 0u};
                if (c < NCHT) {
                    const int dd = c / (BN / 8);
                    const int jc = (c % (BN / 8)) * 8;
                    // mp is a multiple of 64 >= every tile end, padding is zero
                    v = *reinterpret_cast<const u4 *>(YTlp + (int64_t)p * D * mp + (int64_t)dd * mp + j0 + jc);
                }
                pret[p][r] = v;
            }
        if (tid < BN) {
            const int64_t j = j0 + tid;
            bpre = j < m ? (g[j] - ysq[j]) * bscale : -INFINITY;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < NPART; ++p)
#pragma unroll
            for (int r = 0; r < PER_T; ++r) {
                const int c = tid + 256 * r;
                if (c < NCH) {
                    const int row = c / (D / 8);
                    const int col = (c % (D / 8)) * 8;
                    *reinterpret_cast<u4 *>(&yr[buf][p][row * STRIDE + col]) = pre[p][r];
                }
            }
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int r = 0; r < PER_TT; ++r) {
                const int c = tid + 256 * r;
                if (c < NCHT) {
                    const int dd = c / (BN / 8);
                    const int jc = (c % (BN / 8)) * 8;
                    *reinterpret_cast<u4 *>(&ytr[buf][p][dd * TSTRIDE + jc]) = pret[p][r];
                }
            }
        if (tid < BN) bt[buf][tid] = bpre;
    };

    if (ntiles > 0) {
        fetch(0);
        store(0);
    }
    __syncthreads();

    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        const bool more = t + 1 < ntiles;
        if (more) fetch((int64_t)(t + 1) * BN);
        f4 acc[QB][2];
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
            bf8 a[NPART][KS];
#pragma unroll
            for (int p = 0; p < NPART; ++p)
#pragma unroll
                for (int s = 0; s < KS; ++s)
                    a[p][s] = *reinterpret_cast<const bf8 *>(
                        &yr[buf][p][(sub * 16 + li) * STRIDE + lq * KL + 8 * s]);
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) {
                f4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    c = mfma_bf(a[0][s], ub[qb][0][s], c);
                    if constexpr (NPART == 2) {
                        c = mfma_bf(a[0][s], ub[qb][1][s], c);
                        c = mfma_bf(a[1][s], ub[qb][0][s], c);
                    }
                }
                acc[qb][sub] = c;
            }
        }
        const f4 beta0 = *reinterpret_cast<const f4 *>(&bt[buf][lq * 4]);
        const f4 beta1 = *reinterpret_cast<const f4 *>(&bt[buf][16 + lq * 4]);
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            float p[8];
            float mx = kNegBig;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                p[r] = fmaf(acc[qb][0][r], scale2, beta0[r]);
                p[4 + r] = fmaf(acc[qb][1][r], scale2, beta1[r]);
                mx = fmaxf(mx, fmaxf(p[r], p[4 + r]));
            }
            mx = fmaxf(mx, __shfl_xor(mx, 16));
            mx = fmaxf(mx, __shfl_xor(mx, 32));
            const float mn = fmaxf(run_m[qb], mx);
            const float cs = ex2(run_m[qb] - mn);
            run_m[qb] = mn;
            bf8 pb;
            float s = 0.f;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const __bf16 v = (__bf16)ex2(p[e] - mn);
                pb[e] = v;
                s += (float)v;
            }
            run_l[qb] = fmaf(run_l[qb], cs, s);
#pragma unroll
            for (int db = 0; db < NDB; ++db) {
                f4 acc_o = o[qb][db] * cs;
#pragma unroll
                for (int p2 = 0; p2 < 2; ++p2) {
                    const __bf16 *row = &ytr[buf][p2][(db * 16 + li) * TSTRIDE + 4 * lq];
                    const u2 lo4 = *reinterpret_cast<const u2 *>(row);
                    const u2 hi4 = *reinterpret_cast<const u2 *>(row + 16);
                    const bf8 av = __builtin_bit_cast(bf8, u4{lo4.x, lo4.y, hi4.x, hi4.y});
                    acc_o = mfma_bf(av, pb, acc_o);
                }
                o[qb][db] = acc_o;
            }
        }
        if (more) store(buf ^ 1);
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
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (f0 + r < d) {
                        const float xo = Xq[row * d + f0 + r];
                        const float xn = (1.f - alpha) * xo + alpha * (o[qb][db][r] * inv);
                        Xout[row * d + f0 + r] = xn;
                        sq += (double)xn * xn;
                    }
                }
            }
        }
        sq += __shfl_xor(sq, 16);
        sq += __shfl_xor(sq, 32);
        if (out_sqn && lq == 0 && row < nq) out_sqn[row] = (float)sq;
    }
}

// BF16 hi/lo row copies with zero padding to D: lp = [hi | lo], each n x D.
__global__ __launch_bounds__(256) void bf16_split_rows(const float *__restrict__ X, int64_t n, int d,
                                                       int D, __bf16 *__restrict__ lp) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * D) return;
    const int64_t i = e / D;
    const int k = (int)(e % D);
    const float x = k < d ? X[i * d + k] : 0.f;
    const __bf16 h = (__bf16)x;
    lp[e] = h;
    lp[n * D + e] = (__bf16)(x - (float)h);
}

// Transposed copy of both parts: yt[p][k][j] = lp[p][j][k], zero for j >= m.
__global__ __launch_bounds__(256) void bf16_transpose(const __bf16 *__restrict__ lp, int64_t m, int D,
                                                      int64_t mp, __bf16 *__restrict__ yt) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= mp) return;
    for (int p = 0; p < 2; ++p)
        for (int k = 0; k < D; ++k)
            yt[(int64_t)p * D * mp + (int64_t)k * mp + j] =
                j < m ? lp[(int64_t)p * m * D + j * D + k] : (__bf16)0.f;
}

template <int D, int QB, int NPART>
hipError_t lse_bf16_t(const LseJob &a, hipStream_t s) {
    // the plan must cover every row tile of this kernel variant
    if (a.blocks != (a.nu + 64 * QB - 1) / (64 * QB) * a.S) return hipErrorInvalidValue;
    hipLaunchKernelGGL((lse_partial_bf16<D, QB, NPART>), dim3((unsigned)a.blocks), dim3(256), 0, s,
                       (const __bf16 *)a.U_lp, a.nu, (const __bf16 *)a.V_lp, a.nv, a.vsq, a.vpot,
                       a.gamma, a.scale2, a.bscale, a.S, a.cps, a.part_m, a.part_s);
    return hipGetLastError();
}

template <int D, int QB, int NPART>
hipError_t map_bf16_t(const MapArgs &a, float scale2, float bscale, hipStream_t s) {
    const int64_t tiles = (a.nq + 64 * QB - 1) / (64 * QB);
    hipLaunchKernelGGL((entropic_map_bf16<D, QB, NPART>), dim3((unsigned)tiles), dim3(256), 0, s,
                       a.Xq, a.nq, a.d, (const __bf16 *)a.Y_lp, (const __bf16 *)a.YT_lp, a.m,
                       a.mp, a.ysq, a.g, scale2, bscale, a.alpha, a.Xout, a.out_sqn);
    return hipGetLastError();
}

}  // namespace

int bf16_dim(int d) {
    if (d <= 32) return 32;
    if (d <= 64) return 64;
    if (d <= 128) return 128;
    return 256;
}

int64_t bf16_mpad(int64_t m) { return (m + 63) / 64 * 64; }

// Rows per workgroup: 4 waves x QB x 16.  Each column fragment read from LDS
// feeds QB (x3 for the split form) MFMAs; QB = 2 keeps two waves per SIMD
// (measured faster than QB = 4 at one wave per SIMD on d = 256).
constexpr int lse_qb(int npart) { (void)npart; return 2; }
int lse_bf16_rows_per_block(int d, int precision) {
    (void)d;
    return 64 * lse_qb(precision == 2 ? 2 : 1);
}

hipError_t launch_lse_partial_bf16(const LseJob &a, hipStream_t s) {
    const bool x3 = a.precision == 2;
    switch (bf16_dim(a.d)) {
        case 32: return x3 ? lse_bf16_t<32, lse_qb(2), 2>(a, s)
                           : lse_bf16_t<32, lse_qb(1), 1>(a, s);
        case 64: return x3 ? lse_bf16_t<64, lse_qb(2), 2>(a, s)
                           : lse_bf16_t<64, lse_qb(1), 1>(a, s);
        case 128: return x3 ? lse_bf16_t<128, lse_qb(2), 2>(a, s)
                            : lse_bf16_t<128, lse_qb(1), 1>(a, s);
        default: return x3 ? lse_bf16_t<256, lse_qb(2), 2>(a, s)
                           : lse_bf16_t<256, lse_qb(1), 1>(a, s);
    }
}

hipError_t launch_map_bf16(const MapArgs &a, float scale2, float bscale, hipStream_t s) {
    const bool x3 = a.precision == 2;
    switch (bf16_dim(a.d)) {
        case 32: return x3 ? map_bf16_t<32, 4, 2>(a, scale2, bscale, s) : map_bf16_t<32, 4, 1>(a, scale2, bscale, s);
        case 64: return x3 ? map_bf16_t<64, 4, 2>(a, scale2, bscale, s) : map_bf16_t<64, 4, 1>(a, scale2, bscale, s);
        case 128: return x3 ? map_bf16_t<128, 2, 2>(a, scale2, bscale, s) : map_bf16_t<128, 4, 1>(a, scale2, bscale, s);
        default: return x3 ? map_bf16_t<256, 1, 2>(a, scale2, bscale, s) : map_bf16_t<256, 1, 1>(a, scale2, bscale, s);
    }
}

hipError_t launch_bf16_rows(const float *X, int64_t n, int d, void *lp, hipStream_t s) {
    const int D = bf16_dim(d);
    const int64_t tot = n * D;
    hipLaunchKernelGGL(bf16_split_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, n, d, D,
                       (__bf16 *)lp);
    return hipGetLastError();
}

hipError_t launch_bf16_transpose(const void *lp, int64_t m, int d, void *yt, hipStream_t s) {
    const int D = bf16_dim(d);
    const int64_t mp = bf16_mpad(m);
    hipLaunchKernelGGL(bf16_transpose, dim3((unsigned)((mp + 255) / 256)), dim3(256), 0, s,
                       (const __bf16 *)lp, m, D, mp, (__bf16 *)yt);
    return hipGetLastError();
}

}  // namespace pot
