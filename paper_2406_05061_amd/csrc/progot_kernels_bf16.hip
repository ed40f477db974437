// BF16 forms of the fused cost + log-sum-exp kernel and of the entropic-map
// kernel (gfx950, v_mfma_f32_16x16x32_bf16).
//
// Only the cross term <u_i, v_j> changes arithmetic: its operands are BF16
// (round to nearest even), accumulated in FP32.  With NPART = 2 each value is
// split as hi + lo (hi = bf16(x), lo = bf16(x - hi)) and the cross term is
// hi*hi + hi*lo + lo*hi: three products whose error is ~2^-16 relative
// instead of 2^-8.  Norms, the log-sum-exp, potentials and marginal errors
// stay FP32, as in the FP32 form.
//
// On gfx950 the MFMA, the VALU and the transcendental unit of a SIMD do not
// overlap in practice (measured: their issue times add), so these kernels
// are written to issue as few VALU instructions per (row, column) pair as
// possible:
//   * the row operand is held in registers already multiplied by
//     scale2 = 2 log2(e)/eps (converted from the FP32 rows in the kernel),
//   * the column bias beta_j enters as the accumulator's initial value, so
//     the MFMA output is the log2-domain exponent itself,
//   * the column copies are padded to whole tiles, so tile loads carry no
//     bounds checks,
//   * MFMA results live in VGPRs (the library is built with the VGPR form).
// What remains per pair is a max (half a v_max3), a subtraction, an exp2
// and an add for the log-sum-exp.
//
// Shadow layouts (device, written by bf16_split_rows / bf16_transpose, both
// in the tile layout described below):
//   rows:        [hi | lo], each np x D bf16, np = rows rounded up to 128,
//                D = padded dimension, zero padded
//   transposed:  [hi | lo], each D x np bf16 in blocks of 32 columns: within
//                a block, position k holds column perm32(k), the order in
//                which the projection product consumes them (below).
//
// MFMA 16x16x32 bf16: lane l holds A[l%16][8(l/16)..+7] and
// B[8(l/16)..+7][l%16]; the accumulator holds D[4(l/16)+r][l%16].  The
// column tile is the A operand, so lane l owns row i = l%16.  Lane group q
// holds the features [q D/4, (q+1) D/4); MFMA step s uses its features
// q D/4 + 8s .. + 7 (the k index 8q + e maps to feature q D/4 + 8s + e on
// both operands).

#include "progot_internal.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include "progot_device.h"

namespace pot {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void *lds_ptr;
// s_waitcnt operand (gfx9 encoding): vector memory count 0, the export and
// LDS/scalar counts at their maxima, i.e. wait for every vector memory
// operation of the wave, including loads into LDS
constexpr int kWaitVmem = 0x0F70;

__device__ __forceinline__ f4 mfma_bf(bf8 a, bf8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf8 bf8_zero() { return __builtin_bit_cast(bf8, u4{0u, 0u, 0u, 0u}); }

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f4 mfma_h(h8 a, h8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Projection product of the plain BF16 form: FP16 weights times an FP16
// transposed copy of Y (one product instead of BF16 weights times Y_hi +
// Y_lo).  The weights are formed as 2^(t - (m - kF16Shift)), i.e. scaled by
// 2^14, so the largest (exactly 2^14) and those down to ~4e-9 of it stay in
// FP16's normal range with 11 significant bits (FP16 subnormals start at
// 6.1e-5); the normaliser sums the same scaled weights, so the scale cancels.
constexpr float kF16Shift = 14.f;

// The weights 2^(t - shift) of one lane's 8 scores, rounded to FP16 (nearest
// even), in the B-operand order of the projection product.
__device__ __forceinline__ h8 weights_f16(const f4 (&acc)[2], float shift) {
    h8 w;
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
        const f2 v = {ex2(acc[e >> 2][e & 3] - shift), ex2(acc[(e + 1) >> 2][(e + 1) & 3] - shift)};
        const h2 h = __builtin_convertvector(v, h2);
        w[e] = h[0];
        w[e + 1] = h[1];
    }
    return w;
}

__device__ __forceinline__ h8 as_h8(bf8 x) { return __builtin_bit_cast(h8, x); }

// The BF16X3 weights of 8 values: hi = v rounded to BF16, lo = v - hi
// rounded to BF16, as B operands.  One packed conversion rounds two values;
// the hi halves come back to FP32 by a shift and a mask, so each value is
// rounded once per part.
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split_weights(const float (&v)[8], bf8 &hi, bf8 &lo) {
    u4 h, l;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const f2v x = {v[2 * q], v[2 * q + 1]};
        const unsigned hb = __builtin_bit_cast(unsigned, __builtin_convertvector(x, b2v));
        const f2v xh = {__builtin_bit_cast(float, hb << 16), __builtin_bit_cast(float, hb & 0xFFFF0000u)};
        h[q] = hb;
        l[q] = __builtin_bit_cast(unsigned, __builtin_convertvector(x - xh, b2v));
    }
    hi = __builtin_bit_cast(bf8, h);
    lo = __builtin_bit_cast(bf8, l);
}

// Keeps an operand computed before the tile loop in its registers: without
// this the compiler re-derives the BF16 row operands from the FP32 rows in
// every iteration (a v_mul and a v_cvt_pk per element).
__device__ __forceinline__ void pin(bf8 &x) {
    u4 t = __builtin_bit_cast(u4, x);
    asm volatile("" : "+v"(t));
    x = __builtin_bit_cast(bf8, t);
}

// The lane's D/4 features of row `row` of U times `scale`, as hi (and lo)
// BF16 B operands of the KS = D/32 MFMA steps (zero beyond nu and d).
template <int D, int NPART>
__device__ __forceinline__ void scaled_row_operand(const float *__restrict__ U, int64_t nu, int d,
                                                   int64_t row, int lq, float scale,
                                                   bf8 (&ub)[NPART][D / 32]) {
    float u[D / 4];
    row_fetch<D>(U, nu, d, row, lq, u);
#pragma unroll
    for (int s = 0; s < D / 32; ++s) {
        bf8 h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float v = u[8 * s + e] * scale;
            const __bf16 hv = (__bf16)v;
            h[e] = hv;
            l[e] = (__bf16)(v - (float)hv);
        }
        ub[0][s] = h;
        pin(ub[0][s]);
        if constexpr (NPART == 2) {
            ub[1][s] = l;
            pin(ub[1][s]);
        }
    }
}

// Tile layout, in global memory and in LDS alike.  On gfx950 a ds_read_b128
// is conflict-free when each group of 16 consecutive lanes reads 16
// consecutive 16-byte chunks (one 256-byte block); padded row strides, which
// suffice on other parts, measured 2-way conflicted.  Rows are therefore
// stored "16 rows per chunk column": chunk c (8 bf16) of row j, with C
// chunks per row, sits at chunk index ((j / 16) * C + c) * 16 + j % 16.  The
// MFMA operand read of lane (li, lq) -- row 16 b + li, chunk c(lq) -- is one
// 256-byte block per lane group.  The BF16 copies are written in this
// layout, so a tile of whole 16-row blocks is one contiguous range: thread i
// loads chunk i (1 KiB contiguous per wave instruction) and stores it to
// LDS chunk i.
__device__ __forceinline__ int tile_chunk(int blk16, int C, int c, int li) {
    return ((blk16 * C) + c) * 16 + li;
}

// Shape of the potential kernel per (D, NPART): QB 16-row blocks per wave
// and BN columns per LDS tile.  A wave holds 16 QB rows in registers and
// reads every column fragment of a tile from LDS once, so LDS traffic per
// MFMA flop is 1 / (16 QB) bytes for BF16 operands: at QB = 2 the MFMA peak
// would take ~127 bytes of LDS reads per clock per CU, of the order of the
// LDS read rate, and the kernel was co-bound by it.  QB = 4 with 32-column
// tiles (the same accumulator registers, half the LDS per workgroup)
// measured 7-11 % faster at D = 128 and 256 (BF16) and D = 64 and 128
// (BF16X3), 2 % at D = 64 (BF16).  BF16X3 at D = 256 keeps QB = 2 (its row
// operand alone would take 256 registers at QB = 4); D = 32 keeps 64-column
// tiles (a tile must be whole loader rounds); QB = 8 at D = 64 would halve
// the waves per SIMD.  BF16 at D = 256 runs two waves per SIMD (241
// registers); QB = 3 there (187 registers, or 168 with 3 waves per SIMD and
// a small spill) measured 21 % and 14 % slower at 65536^2: the fragment
// reuse counts for more than the occupancy.
struct LseShape { int qb, bn; };
constexpr LseShape lse_shape(int D, int npart) {
    return (D >= 64 && D * npart <= 256) ? LseShape{4, 32} : LseShape{2, D * npart >= 512 ? 32 : 64};
}

template <int D, int NPART, int BN_ = lse_shape(D, NPART).bn> struct TileH {
    static constexpr int BN = BN_;           // columns per LDS tile
    static constexpr int NSUB = BN / 16;
    static constexpr int KS = D / 32;        // MFMA k-steps over the features
    static constexpr int C = D / 8;          // 16-byte chunks per column
    static constexpr int NCH = BN * C;       // 16-byte chunks per part
    static constexpr int PER_T = NCH / 256;
    static_assert(NCH % 256 == 0, "tile chunks must cover the workgroup");
};

// Sums of a fixed-shift sweep must land in [kSumLo, kSumHi]: then no term
// that matters against the row's largest overflowed or fell below FP32's
// normal range (every term is at most the sum, and terms under 2^-126 are
// below 2^-62 of a sum of at least 2^-64).  The upper bound is a kernel
// argument so that the host can fail every check (sum_hi < 0) and run the
// fallback on purpose.
constexpr float kSumLo = 0x1p-64f, kSumHi = 0x1p64f;

// Partial log-sum-exp over one column split (BF16 cross term).  Splits start
// on multiples of 64 columns and the column copy is padded to a multiple of
// 128 rows, so every tile load is in bounds; columns past the split get
// beta = kNegBig.
//
// Exponent shift: with shift_pot (an estimate of the rows' new potential,
// scaled by shift_gamma: the previous iterate's, or a ProgOT step's warm
// start) each row i is shifted by the log-sum-exp that potential implies,
// L_i = (eps log w_i + |u_i|^2 - shift_gamma shift_pot_i) / (eps ln 2), the
// value the merge inverts.  Between Sinkhorn iterations, and from a warm
// start to the first iterate, L_i moves little, so the sum of 2^(t_ij - L_i)
// stays near 1 and no running maximum (a max per pair and a rescale per
// tile) is needed; the partial is written as (L_i, sum).  If
// any row's sum over the split leaves [kSumLo, kSumHi] (a stale potential, a
// non-finite value), the workgroup sweeps its split again with the running
// maximum, which is what runs without shift_pot.
template <int D, int QB, int NPART, int BN>
__global__ __launch_bounds__(256) void lse_partial_bf16(
    const float *__restrict__ U, int64_t nu, int d, const __bf16 *__restrict__ Vlp, int64_t nv,
    int64_t vstride, const float *__restrict__ vsq, const float *__restrict__ vpot, float gamma,
    float scale2, float bscale, int S, int64_t cols_per_split, float *__restrict__ part_m,
    float *__restrict__ part_s, const float *__restrict__ shift_pot, const float *__restrict__ usq,
    const float *__restrict__ logw, float eps, float sum_hi, float shift_gamma) {
    using T = TileH<D, NPART, BN>;
    constexpr int ROWS = 64 * QB;
    __shared__ __bf16 vt[2][NPART][T::BN * D];
    __shared__ float bt[2][T::BN];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int split = blockIdx.x % S;
    const int64_t tile = blockIdx.x / S;
    const int64_t row0 = tile * ROWS + wave * (QB * 16);

    bf8 ub[QB][NPART][T::KS];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb)
        scaled_row_operand<D, NPART>(U, nu, d, row0 + qb * 16 + li, lq, scale2, ub[qb]);

    float sh[QB];
    if (shift_pot) {
        const float inv = 1.f / (eps * kLn2);
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            const int64_t row = row0 + qb * 16 + li;
            sh[qb] = row < nu ? (fmaf(eps, logw[row], usq[row]) - shift_gamma * shift_pot[row]) * inv : 0.f;
        }
    }

    const int64_t c0 = (int64_t)split * cols_per_split;
    const int64_t c1 = c0 + cols_per_split < nv ? c0 + cols_per_split : nv;
    const int ntiles = c0 < c1 ? (int)((c1 - c0 + T::BN - 1) / T::BN) : 0;
    u4 pre[NPART][T::PER_T];
    // column biases: raw values loaded with the tile, combined where they are
    // stored, so that no wave waits on the loads ahead of its MFMAs (index
    // clamped into the split, -inf past it; the product rounded on its own)
    int64_t jpre = 0;
    float gpre = 0.f, ypre = 0.f;
    auto fetch = [&](int t) {
        // uniform tile base, 32-bit per-lane offsets
#pragma unroll
        for (int p = 0; p < NPART; ++p) {
            const __bf16 *src = Vlp + p * vstride + (c0 + (int64_t)t * T::BN) * D;
#pragma unroll
            for (int r = 0; r < T::PER_T; ++r)
                pre[p][r] = *reinterpret_cast<const u4 *>(src + (tid + 256 * r) * 8);
        }
        jpre = c0 + (int64_t)t * T::BN + tid;
        if (tid < T::BN) {
            const int64_t jc = jpre < c1 ? jpre : c1 - 1;
            gpre = vpot ? vpot[jc] : 0.f;
            ypre = vsq[jc];
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < NPART; ++p)
#pragma unroll
            for (int r = 0; r < T::PER_T; ++r)
                *reinterpret_cast<u4 *>(&vt[buf][p][(tid + 256 * r) * 8]) = pre[p][r];
        if (tid < T::BN)
            bt[buf][tid] = jpre < c1 ? ((vpot ? __fmul_rn(gamma, gpre) : 0.f) - ypre) * bscale : kNegBig;
    };

    // One sweep over the split's column tiles; (run_m, run_s) per row,
    // combined over the four lane groups that share it.
    float run_m[QB], run_s[QB];
    auto sweep = [&](auto fixed_tag) {
        constexpr bool FIXED = decltype(fixed_tag)::value;
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) { run_m[qb] = FIXED ? sh[qb] : kNegBig; run_s[qb] = 0.f; }
        if (ntiles > 0) {
            fetch(0);
            store(0);
        }
        __syncthreads();

        for (int t = 0; t < ntiles; ++t) {
            const int buf = t & 1;
            const bool more = t + 1 < ntiles;
            if (more) fetch(t + 1);
            // raised priority while the products issue (as in the FP32
            // kernel; same bits, 0.5-1.5 % at d = 128 and 256)
            __builtin_amdgcn_s_setprio(1);
            // accumulators start at beta_j: the MFMA output is the exponent
            f4 acc[QB][T::NSUB];
#pragma unroll
            for (int sub = 0; sub < T::NSUB; ++sub) {
                const f4 beta = *reinterpret_cast<const f4 *>(&bt[buf][sub * 16 + lq * 4]);
#pragma unroll
                for (int qb = 0; qb < QB; ++qb) acc[qb][sub] = beta;
            }
            // k outer; the column fragments of step s + 1 are read while step
            // s runs, and each product term sweeps all NSUB x QB
            // accumulators, so consecutive MFMAs are independent.
            bf8 a[2][NPART][T::NSUB];
            auto read_a = [&](int s, bf8 (&dst)[NPART][T::NSUB]) {
#pragma unroll
                for (int p = 0; p < NPART; ++p)
#pragma unroll
                    for (int sub = 0; sub < T::NSUB; ++sub)
                        dst[p][sub] = *reinterpret_cast<const bf8 *>(
                            &vt[buf][p][tile_chunk(sub, T::C, lq * T::KS + s, li) * 8]);
            };
            read_a(0, a[0]);
#pragma unroll
            for (int s = 0; s < T::KS; ++s) {
                if (s + 1 < T::KS) read_a(s + 1, a[(s + 1) & 1]);
                const int cs = s & 1;
#pragma unroll
                for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
                    for (int qb = 0; qb < QB; ++qb)
                        acc[qb][sub] = mfma_bf(a[cs][0][sub], ub[qb][0][s], acc[qb][sub]);
                if constexpr (NPART == 2) {
#pragma unroll
                    for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
                        for (int qb = 0; qb < QB; ++qb)
                            acc[qb][sub] = mfma_bf(a[cs][0][sub], ub[qb][1][s], acc[qb][sub]);
#pragma unroll
                    for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
                        for (int qb = 0; qb < QB; ++qb)
                            acc[qb][sub] = mfma_bf(a[cs][1][sub], ub[qb][0][s], acc[qb][sub]);
                }
            }
            __builtin_amdgcn_s_setprio(0);
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) {
                // partial sums start at the first subtile's terms (an add to
                // 0 cannot be dropped by the compiler; the terms are never -0)
                float s4[4];
                if constexpr (FIXED) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) s4[r] = ex2(acc[qb][0][r] - sh[qb]);
#pragma unroll
                    for (int sub = 1; sub < T::NSUB; ++sub)
#pragma unroll
                        for (int r = 0; r < 4; ++r) s4[r] += ex2(acc[qb][sub][r] - sh[qb]);
                    run_s[qb] += (s4[0] + s4[1]) + (s4[2] + s4[3]);
                } else {
                    float mx = kNegBig;
#pragma unroll
                    for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
                        for (int r = 0; r < 4; ++r) mx = fmaxf(mx, acc[qb][sub][r]);
                    const float mn = fmaxf(run_m[qb], mx);
#pragma unroll
                    for (int r = 0; r < 4; ++r) s4[r] = ex2(acc[qb][0][r] - mn);
#pragma unroll
                    for (int sub = 1; sub < T::NSUB; ++sub)
#pragma unroll
                        for (int r = 0; r < 4; ++r) s4[r] += ex2(acc[qb][sub][r] - mn);
                    run_s[qb] = fmaf(run_s[qb], ex2(run_m[qb] - mn), (s4[0] + s4[1]) + (s4[2] + s4[3]));
                    run_m[qb] = mn;
                }
            }
            if (more) store(buf ^ 1);
            __syncthreads();
        }

#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            float m = run_m[qb], s = run_s[qb];
#pragma unroll
            for (int off = 16; off <= 32; off <<= 1) {
                const float so = __shfl_xor(s, off);
                if constexpr (FIXED) {
                    s += so;
                } else {
                    const float mo = __shfl_xor(m, off);
                    const float mn = fmaxf(m, mo);
                    s = s * ex2(m - mn) + so * ex2(mo - mn);
                    m = mn;
                }
            }
            run_m[qb] = m;
            run_s[qb] = s;
        }
    };

    bool redo = true;
    if (shift_pot) {
        sweep(std::true_type{});
        int bad = 0;
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            const bool in_range = run_s[qb] <= sum_hi && (ntiles == 0 || run_s[qb] >= kSumLo);
            if (row0 + qb * 16 + li < nu && !in_range) bad = 1;
        }
        redo = __syncthreads_or(bad) != 0;
    }
    if (redo) sweep(std::false_type{});

#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        const int64_t row = row0 + qb * 16 + li;
        if (lq == 0 && row < nu) {
            part_m[split * nu + row] = run_m[qb];
            part_s[split * nu + row] = run_s[qb];
        }
    }
}

// Position k of a 32-column group of the transposed copy holds column
// perm32(k): the B operand of the projection product takes, in lane group q,
// the columns 4q..4q+3 of the first score subtile and then the same four of
// the second (the accumulator layout of the score tile), so k = 8q + e is
// column 4q + e (e < 4) or 16 + 4q + e - 4 (e >= 4).
__host__ __device__ constexpr int perm32(int k) {
    return (k & 7) < 4 ? 4 * (k >> 3) + (k & 7) : 16 + 4 * (k >> 3) + (k & 7) - 4;
}

// Entropic map + McCann-type step.  The projection product is FP16 weights
// times one FP16 copy of Y scaled by a power of two (NPART = 1), or P split
// as P_hi + P_lo with the three products P_hi Y_hi + P_hi Y_lo + P_lo Y_hi
// (NPART = 2, so both products of the split form carry ~16 bits).  The
// normaliser is the same product against a row of ones, so it sums exactly
// the weights applied to the targets: T is a convex combination of the
// targets.  A tile is NG groups of 32 columns (kMapBN); the transposed copy
// holds each group in the perm32 order, and the softmax (maximum, rescale,
// weights) runs once per tile.
// P = 2^(t - m_used) with m_used the running maximum.  The output
// accumulator is rescaled only in tiles where some row of the wave sets a new
// maximum (a row does so about log(tiles) times for columns in random
// order), not in every tile.  The threshold stays 0: with m_used exactly the
// maximum, the largest weight of each row is 1.0, exact in BF16 (a stale
// maximum rounds it too and measurably doubles the map's rounding error).
constexpr int kMapBN = 32;
constexpr float kLazy = 0.f;

template <int D, int QB, int NPART, int NG>
__global__ __launch_bounds__(256) void entropic_map_bf16(
    const float *Xq, int64_t nq, int d, const __bf16 *__restrict__ Ylp,
    const __bf16 *__restrict__ YTlp, int64_t m, int64_t mp, const float *__restrict__ ysq,
    const float *__restrict__ g, float scale2, float bscale, float alpha, float *Xout,
    float *__restrict__ out_sqn, const float *__restrict__ yt_unscale) {
    constexpr int BN = kMapBN * NG;            // NG groups of 32 columns per tile
    constexpr int NS = 2 * NG;                 // 16-column score subtiles
    constexpr int KS = D / 32, C = D / 8;
    constexpr int NDB = D / 16;
    constexpr int ROWS = 64 * QB;
    constexpr int NCH = BN * D / 8;            // 16-byte chunks per part (both copies)
    constexpr int PER_T = (NCH + 255) / 256;
    constexpr int NYT = NPART == 2 ? 2 : 1;    // parts of the transposed copy (FP16: one)
    // row tile: BN columns x C chunks; transposed tile: D dims x 4 chunks
    __shared__ __bf16 yr[2][NPART][BN * D];
    __shared__ __bf16 ytr[2][NYT][D * BN];
    __shared__ float bt[2][BN];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * ROWS + wave * (QB * 16);

    bf8 ub[QB][NPART][KS];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb)
        scaled_row_operand<D, NPART>(Xq, nq, d, row0 + qb * 16 + li, lq, scale2, ub[qb]);

    // A operand of the normaliser: a row of ones (output row 0)
    bf8 ones = bf8_zero();
    h8 ones16 = as_h8(bf8_zero());
    if (li == 0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            ones[e] = (__bf16)1.f;
            ones16[e] = (_Float16)1.f;
        }
    }

    float m_used[QB];
    f4 o[QB][NDB], on[QB];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        m_used[qb] = kNegBig;
        on[qb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int db = 0; db < NDB; ++db) o[qb][db] = f4{0.f, 0.f, 0.f, 0.f};
    }

    const int ntiles = (int)((m + BN - 1) / BN);
    u4 pre[NPART][PER_T];
    u4 pret[NYT][PER_T];
    // column biases: raw values with the tile, combined where stored
    int64_t jpre = 0;
    float gpre = 0.f, ypre = 0.f;
    auto fetch = [&](int t) {
        const int64_t j0 = (int64_t)t * BN;
#pragma unroll
        for (int r = 0; r < PER_T; ++r) {
            const int c = tid + 256 * r;
            if (NCH % 256 == 0 || c < NCH) {
#pragma unroll
                for (int p = 0; p < NPART; ++p)
                    pre[p][r] = *reinterpret_cast<const u4 *>(Ylp + (p * mp + j0) * D + c * 8);
#pragma unroll
                for (int p = 0; p < NYT; ++p)
                    pret[p][r] = *reinterpret_cast<const u4 *>(YTlp + (p * mp + j0) * D + c * 8);
            }
        }
        jpre = j0 + tid;
        if (tid < BN) {
            const int64_t jc = jpre < m ? jpre : m - 1;
            gpre = g[jc];
            ypre = ysq[jc];
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int r = 0; r < PER_T; ++r) {
            const int c = tid + 256 * r;
            if (NCH % 256 == 0 || c < NCH) {
#pragma unroll
                for (int p = 0; p < NPART; ++p) *reinterpret_cast<u4 *>(&yr[buf][p][c * 8]) = pre[p][r];
#pragma unroll
                for (int p = 0; p < NYT; ++p) *reinterpret_cast<u4 *>(&ytr[buf][p][c * 8]) = pret[p][r];
            }
        }
        if (tid < BN) bt[buf][tid] = jpre < m ? (gpre - ypre) * bscale : kNegBig;
    };

    if (ntiles > 0) {
        fetch(0);
        store(0);
    }
    __syncthreads();

    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        const bool more = t + 1 < ntiles;
        if (more) fetch(t + 1);
        f4 acc[QB][NS];
#pragma unroll
        for (int sub = 0; sub < NS; ++sub) {
            const f4 beta = *reinterpret_cast<const f4 *>(&bt[buf][sub * 16 + lq * 4]);
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) acc[qb][sub] = beta;
        }
        // k outer with the next step's fragments read ahead; each product
        // term sweeps the NS x QB accumulators (independent consecutive MFMAs)
        bf8 a[2][NPART][NS];
        auto read_a = [&](int s, bf8 (&dst)[NPART][NS]) {
#pragma unroll
            for (int p = 0; p < NPART; ++p)
#pragma unroll
                for (int sub = 0; sub < NS; ++sub)
                    dst[p][sub] = *reinterpret_cast<const bf8 *>(
                        &yr[buf][p][tile_chunk(sub, C, lq * KS + s, li) * 8]);
        };
        read_a(0, a[0]);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (s + 1 < KS) read_a(s + 1, a[(s + 1) & 1]);
            const int cs = s & 1;
#pragma unroll
            for (int sub = 0; sub < NS; ++sub)
#pragma unroll
                for (int qb = 0; qb < QB; ++qb)
                    acc[qb][sub] = mfma_bf(a[cs][0][sub], ub[qb][0][s], acc[qb][sub]);
            if constexpr (NPART == 2) {
#pragma unroll
                for (int sub = 0; sub < NS; ++sub)
#pragma unroll
                    for (int qb = 0; qb < QB; ++qb)
                        acc[qb][sub] = mfma_bf(a[cs][0][sub], ub[qb][1][s], acc[qb][sub]);
#pragma unroll
                for (int sub = 0; sub < NS; ++sub)
#pragma unroll
                    for (int qb = 0; qb < QB; ++qb)
                        acc[qb][sub] = mfma_bf(a[cs][1][sub], ub[qb][0][s], acc[qb][sub]);
            }
        }
        bf8 pb[QB][NG], pl[NPART == 2 ? QB : 1][NG];
        h8 p16[QB][NG];
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            float mx = kNegBig;
#pragma unroll
            for (int sub = 0; sub < NS; ++sub)
#pragma unroll
                for (int r = 0; r < 4; ++r) mx = fmaxf(mx, acc[qb][sub][r]);
            mx = max_lane_groups(mx);
            const bool up = mx > m_used[qb] + kLazy;
            if (__builtin_amdgcn_ballot_w64(up)) {
                const float mn = up ? mx : m_used[qb];
                const float cs = ex2(m_used[qb] - mn);
                m_used[qb] = mn;
                on[qb] *= cs;
#pragma unroll
                for (int db = 0; db < NDB; ++db) o[qb][db] *= cs;
            }
#pragma unroll
            for (int g2 = 0; g2 < NG; ++g2) {
                const f4 pair[2] = {acc[qb][2 * g2], acc[qb][2 * g2 + 1]};
                if constexpr (NPART == 1) {
                    p16[qb][g2] = weights_f16(pair, m_used[qb] - kF16Shift);
                } else {
                    float v[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) v[e] = ex2(pair[e >> 2][e & 3] - m_used[qb]);
                    split_weights(v, pb[qb][g2], pl[qb][g2]);
                }
            }
        }
        // O^T += Y^T P^T per 32-column group: each Y^T fragment (16 dims x 32
        // columns) is read once and feeds the QB row blocks; the hi part of
        // every dimension block is applied before the lo part, so an
        // accumulator is not touched by consecutive MFMAs
#pragma unroll
        for (int g2 = 0; g2 < NG; ++g2) {
            const int goff = g2 * D * kMapBN;
            if constexpr (NPART == 1) {
                // one FP16 product against the scaled FP16 copy
#pragma unroll
                for (int db = 0; db < NDB; ++db) {
                    const h8 av = as_h8(
                        *reinterpret_cast<const bf8 *>(&ytr[buf][0][goff + tile_chunk(db, 4, lq, li) * 8]));
#pragma unroll
                    for (int qb = 0; qb < QB; ++qb) o[qb][db] = mfma_h(av, p16[qb][g2], o[qb][db]);
                }
#pragma unroll
                for (int qb = 0; qb < QB; ++qb) on[qb] = mfma_h(ones16, p16[qb][g2], on[qb]);
            } else {
#pragma unroll
                for (int p2 = 0; p2 < 2; ++p2)
#pragma unroll
                    for (int db = 0; db < NDB; ++db) {
                        const bf8 av = *reinterpret_cast<const bf8 *>(
                            &ytr[buf][p2][goff + tile_chunk(db, 4, lq, li) * 8]);
#pragma unroll
                        for (int qb = 0; qb < QB; ++qb) o[qb][db] = mfma_bf(av, pb[qb][g2], o[qb][db]);
                        if (p2 == 0)
#pragma unroll
                            for (int qb = 0; qb < QB; ++qb) o[qb][db] = mfma_bf(av, pl[qb][g2], o[qb][db]);
                    }
#pragma unroll
                for (int qb = 0; qb < QB; ++qb) {
                    on[qb] = mfma_bf(ones, pb[qb][g2], on[qb]);
                    on[qb] = mfma_bf(ones, pl[qb][g2], on[qb]);
                }
            }
        }
        if (more) store(buf ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        // the normaliser of row li sits in output row 0: lane li, register 0
        const float l = __shfl(on[qb][0], li);
        // the FP16 copy holds Y scaled by a power of two: undo it exactly
        const float inv = (NPART == 1 ? *yt_unscale : 1.f) / l;
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

// Warp-specialised form of the map kernel (D = 128 and 256).  A workgroup of
// 8 waves maps 64 NQB queries in two roles that run one column tile apart
// (NG groups of 32 columns: one for BF16X3, two for plain BF16, whose
// one-product tiles leave the fixed costs of an interval a larger share):
//   score waves 0-3 each hold NQB blocks of 16 queries (rows in registers,
//     hi/lo for BF16X3) and, for tile t, compute the exponent-valued scores
//     and the softmax (running maximum, weights -- BF16 hi/lo, or FP16 for
//     plain BF16 -- and normaliser), and publish the weights and rescale
//     factors in LDS buffer t & 1;
//   projection waves 4-7 each own D/4 output dimensions of every query and,
//     in the same interval, apply the weights of tile t - 1 with their own
//     fragments of the transposed copy (read from global memory into
//     registers a tile ahead: each fragment is used by one wave only), and
//     load tile t + 1's rows straight from global memory into LDS.
// Waves w and w + 4 share a SIMD, so its matrix core is fed by one role while
// the other runs its softmax or waits on memory; the score waves issue at a
// raised priority so that their products, which the softmax waits for, go
// first.  One barrier per tile orders the roles through the double buffers.
// A score wave reads each tile fragment for NQB query blocks, and no wave
// stages anything through registers.  The products, normaliser and rescale
// rule are those of entropic_map_bf16, in one fixed order per accumulator.
// Measured at n = m = 65536 against the previous kernels: BF16X3 D = 256
// 8.9-9.4 ms instead of 12.5 (one role per wave, 16 queries per wave, 8
// waves in lockstep; same bits), D = 128 4.65-4.8 ms instead of 5.45-5.55
// (the narrow kernel); plain BF16 D = 256 3.5 ms instead of 5.8 (the narrow
// kernel; 3.7-3.9 ms, and its bits, with 32-column tiles), D = 128 1.95-2.0
// ms instead of 2.26-2.49 (the narrow kernel with the same 64-column tiles,
// same bits); at D = 64 (BF16X3) the narrow kernel with 64-column tiles
// stays faster.  Interval structure of
// BF16X3 at D = 256 from per-wave clock stamps: the projection waves are the
// critical path (products of both roles plus the softmax issue on the
// SIMD), the score waves wait ~1200 cycles of ~4850 at the barrier.
template <int D, int NQB, int NPART, int NG>
__global__ __launch_bounds__(512) void entropic_map_bf16_ws(
    const float *Xq, int64_t nq, int d, const __bf16 *__restrict__ Ylp,
    const __bf16 *__restrict__ YTlp, int64_t m, int64_t mp, const float *__restrict__ ysq,
    const float *__restrict__ g, float scale2, float bscale, float alpha, float *Xout,
    const float *__restrict__ yt_unscale) {
    static_assert(NPART == 1 || NG == 1, "BF16X3 tiles are one group of 32 columns");
    constexpr int BN = kMapBN * NG;        // NG groups of 32 columns per tile
    constexpr int NS = 2 * NG;             // 16-column score subtiles
    constexpr int NYG = NPART == 2 ? 2 : NG;  // transposed fragments per dims block: parts or groups
    constexpr int KS = D / 32, C = D / 8;
    constexpr int NSW = 4;                 // score waves; as many projection waves
    constexpr int NQ = NSW * NQB;          // query blocks of 16 per workgroup
    constexpr int ROWS = 16 * NQ;
    constexpr int NDB = D / 16 / NSW;      // output dimension blocks per projection wave
    constexpr int NCH = BN * C;            // 16-byte chunks per part of a tile
    constexpr int PER_T = NCH / 256;       // of them per projection thread
    static_assert(NDB >= 1 && NCH % 256 == 0, "projection waves need D >= 64");
    __shared__ __bf16 yr[2][NPART][BN * D];
    __shared__ float bt[2][BN];
    __shared__ bf8 pw[2][NPART * NG][NQ][64];  // weights of every block (hi/lo, or per group)
    __shared__ float csw[2][NQ][16];       // rescale factor of each query
    __shared__ __align__(16) int upw[2][NQ];  // block rescaled this tile
    __shared__ float lw[ROWS];             // normalisers at the end

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int64_t blk0 = (int64_t)blockIdx.x * ROWS;
    const int ntiles = (int)((m + BN - 1) / BN);
    const bool score_role = wave < NSW;
    const int rw = score_role ? wave : wave - NSW;

    if (score_role) {
        const int wave = rw;
        __builtin_amdgcn_s_setprio(1);    // 1-3 % over equal priority
        bf8 ub[NQB][NPART][KS];
#pragma unroll
        for (int b = 0; b < NQB; ++b)
            scaled_row_operand<D, NPART>(Xq, nq, d, blk0 + (wave * NQB + b) * 16 + li, lq, scale2, ub[b]);
        bf8 ones = bf8_zero();
        h8 ones16 = as_h8(bf8_zero());
        if (li == 0) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                ones[e] = (__bf16)1.f;
                ones16[e] = (_Float16)1.f;
            }
        }
        float m_used[NQB];
        f4 on[NQB];
#pragma unroll
        for (int b = 0; b < NQB; ++b) {
            m_used[b] = kNegBig;
            on[b] = f4{0.f, 0.f, 0.f, 0.f};
        }
        __syncthreads();                   // tile 0 staged
        for (int t = 0; t < ntiles; ++t) {
            const int buf = t & 1;
            f4 acc[NQB][NS];
#pragma unroll
            for (int sub = 0; sub < NS; ++sub) {
                const f4 bias = *reinterpret_cast<const f4 *>(&bt[buf][sub * 16 + lq * 4]);
#pragma unroll
                for (int b = 0; b < NQB; ++b) acc[b][sub] = bias;
            }
            bf8 a[2][NPART][NS];
            auto read_a = [&](int s, bf8 (&dst)[NPART][NS]) {
#pragma unroll
                for (int p = 0; p < NPART; ++p)
#pragma unroll
                    for (int sub = 0; sub < NS; ++sub)
                        dst[p][sub] = *reinterpret_cast<const bf8 *>(
                            &yr[buf][p][tile_chunk(sub, C, lq * KS + s, li) * 8]);
            };
            read_a(0, a[0]);
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                if (s + 1 < KS) read_a(s + 1, a[(s + 1) & 1]);
                const int cs = s & 1;
#pragma unroll
                for (int b = 0; b < NQB; ++b)
#pragma unroll
                    for (int sub = 0; sub < NS; ++sub) acc[b][sub] = mfma_bf(a[cs][0][sub], ub[b][0][s], acc[b][sub]);
                if constexpr (NPART == 2) {
#pragma unroll
                    for (int b = 0; b < NQB; ++b)
#pragma unroll
                        for (int sub = 0; sub < 2; ++sub)
                            acc[b][sub] = mfma_bf(a[cs][0][sub], ub[b][1][s], acc[b][sub]);
#pragma unroll
                    for (int b = 0; b < NQB; ++b)
#pragma unroll
                        for (int sub = 0; sub < 2; ++sub)
                            acc[b][sub] = mfma_bf(a[cs][1][sub], ub[b][0][s], acc[b][sub]);
                }
            }
#pragma unroll
            for (int b = 0; b < NQB; ++b) {
                const int qb = wave * NQB + b;
                float mx = kNegBig;
#pragma unroll
                for (int sub = 0; sub < NS; ++sub)
#pragma unroll
                    for (int r = 0; r < 4; ++r) mx = fmaxf(mx, acc[b][sub][r]);
                mx = max_lane_groups(mx);
                const bool up = mx > m_used[b] + kLazy;
                const bool any = __builtin_amdgcn_ballot_w64(up) != 0;
                float csf = 1.f;
                if (any) {
                    const float mn = up ? mx : m_used[b];
                    csf = ex2(m_used[b] - mn);
                    m_used[b] = mn;
                    on[b] *= csf;
                }
                if constexpr (NPART == 1) {
                    // FP16 weights scaled by 2^kF16Shift (normaliser alike),
                    // one B operand per group of 32 columns
#pragma unroll
                    for (int g2 = 0; g2 < NG; ++g2) {
                        const f4 pair[2] = {acc[b][2 * g2], acc[b][2 * g2 + 1]};
                        const h8 p16 = weights_f16(pair, m_used[b] - kF16Shift);
                        on[b] = mfma_h(ones16, p16, on[b]);
                        pw[buf][g2][qb][lane] = __builtin_bit_cast(bf8, p16);
                    }
                } else {
                    float v[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) v[e] = ex2(acc[b][e >> 2][e & 3] - m_used[b]);
                    bf8 pb, pl;
                    split_weights(v, pb, pl);
                    on[b] = mfma_bf(ones, pb, on[b]);
                    on[b] = mfma_bf(ones, pl, on[b]);
                    pw[buf][0][qb][lane] = pb;
                    pw[buf][1][qb][lane] = pl;
                }
                if (lq == 0) csw[buf][qb][li] = csf;
                if (lane == 0) upw[buf][qb] = any;
            }
            __syncthreads();
        }
        __syncthreads();                   // the interval that applies the last tile's weights
        // normalisers: output row 0 of each block's ones product
#pragma unroll
        for (int b = 0; b < NQB; ++b)
            if (lq == 0) lw[(wave * NQB + b) * 16 + li] = on[b][0];
        __syncthreads();
    } else {
        const int pv = __builtin_amdgcn_readfirstlane(rw);  // dimension blocks pv NDB .. + NDB - 1
        const int pt = pv * 64 + lane;     // loader thread 0..255
        // global addresses: a wave-uniform base (scalar registers) plus one
        // per-lane byte offset shared by every part
        const char *const yrow = reinterpret_cast<const char *>(Ylp);
        const char *const ycol = reinterpret_cast<const char *>(YTlp);
        const uint32_t loff = (uint32_t)lane * 16u;
        f4 o[NQ][NDB];
#pragma unroll
        for (int qb = 0; qb < NQ; ++qb)
#pragma unroll
            for (int db = 0; db < NDB; ++db) o[qb][db] = f4{0.f, 0.f, 0.f, 0.f};
        constexpr int NLD = NPART * PER_T;  // row chunks per loader thread and tile
        // rows of tile t straight from global memory into LDS buffer buf:
        // lane l of a wave writes its 16 bytes at the wave's base + 16 l, so
        // thread pt's chunk pt + 256 r lands at its place in the tile layout
        auto load_rows_part = [&](int t, int buf, int k) {
            const int p = k % NPART, r = k / NPART;
            const char *base = yrow + ((p * mp + (int64_t)t * BN) * D + (256 * r + 64 * pv) * 8) * 2;
            __builtin_amdgcn_global_load_lds(
                (const void *)(base + loff), (lds_ptr)&yr[buf][p][(256 * r + 64 * pv) * 8], 16, 0, 0);
        };
        // column biases of the next tile: loaded at the start of an interval,
        // combined and stored at its end (index clamped into the cloud, the
        // value replaced for columns past m)
        int64_t jb = 0;
        float gpre = 0.f, ypre = 0.f;
        auto fetch_bias = [&](int t) {
            jb = (int64_t)t * BN + pt;
            if (pt < BN) {
                const int64_t jc = jb < m ? jb : m - 1;
                gpre = g[jc];
                ypre = ysq[jc];
            }
        };
        auto store_bias = [&](int buf) {
            if (pt < BN) bt[buf][pt] = jb < m ? (gpre - ypre) * bscale : kNegBig;
        };
        // this wave's fragments of the transposed tile (hi and lo parts of
        // its one group, or the one FP16 part of each group): 1 KiB each,
        // contiguous in the tile layout; two sets, one in use and one loading
        bf8 yv[NYG][NDB], yw[NYG][NDB];
        auto load_yv_part = [&](int t, bf8 (&dst)[NYG][NDB], int k) {
            const int p2 = k / NDB, db = k % NDB;
            const int part = NPART == 2 ? p2 : 0, grp = NPART == 2 ? 0 : p2;
            const char *base =
                ycol + ((part * mp + (int64_t)t * BN + grp * kMapBN) * D + (pv * NDB + db) * 64 * 8) * 2;
            dst[p2][db] = *reinterpret_cast<const bf8 *>(base + loff);
        };
        // tile indices below clamp to the last tile (m >= 1): its repeated
        // loads land where nothing reads them again
        const int last = ntiles - 1;
#pragma unroll
        for (int k = 0; k < NLD; ++k) load_rows_part(0, 0, k);
        fetch_bias(0);
        store_bias(0);
        __builtin_amdgcn_s_waitcnt(kWaitVmem);
        __syncthreads();                   // tile 0 staged
        // Interval t: tile t's fragments (into ynew) and tile t + 1's column
        // biases load first, then the projection of tile t - 1 with the
        // fragments in yold, with the loads of tile t + 1's rows into LDS
        // buffer (t + 1) & 1 issued between the products of the first query
        // blocks: the copies run while the matrix cores work, and every load
        // of the wave must be complete at the barrier that ends the interval.
        auto body = [&](int t, bf8 (&ynew)[NYG][NDB], bf8 (&yold)[NYG][NDB]) {
            const int tn = min(t, last), tr = min(t + 1, last), sb = (t + 1) & 1;
            fetch_bias(tr);
#pragma unroll
            for (int k = 0; k < NYG * NDB; ++k) load_yv_part(tn, ynew, k);
            {
                // O^T[this wave's dims] += Y^T P^T for the weights of tile t - 1
                const int buf = (t - 1) & 1;
                // the rescale flags of all blocks in one LDS round trip
                int mask = 0;
#pragma unroll
                for (int k = 0; k < NQ / 4; ++k) {
                    const i4 f = *reinterpret_cast<const i4 *>(&upw[buf][4 * k]);
                    mask |= (f[0] << (4 * k)) | (f[1] << (4 * k + 1)) | (f[2] << (4 * k + 2)) |
                            (f[3] << (4 * k + 3));
                }
                mask = __builtin_amdgcn_readfirstlane(mask);
                if (mask) {
                    // one branch for all blocks (a factor of 1 leaves a block's
                    // sums unchanged): per-block branches made the compiler
                    // copy the accumulators at every join
#pragma unroll
                    for (int qb = 0; qb < NQ; ++qb) {
                        const float c = ((mask >> qb) & 1) ? csw[buf][qb][li] : 1.f;
#pragma unroll
                        for (int db = 0; db < NDB; ++db) o[qb][db] *= c;
                    }
                }
                // weights read one block ahead; the scheduling barrier at the
                // end of each block keeps the compiler from hoisting every
                // block's reads (64 more registers) above the products
                // ph, pl: the hi and lo weights (BF16X3) or those of groups 0, 1
                bf8 ph = pw[buf][0][0][lane], pl = pw[buf][NPART * NG - 1][0][lane];
#pragma unroll
                for (int qb = 0; qb < NQ; ++qb) {
                    bf8 phn = ph, pln = pl;
                    if (qb + 1 < NQ) {
                        phn = pw[buf][0][qb + 1][lane];
                        if (NPART * NG == 2) pln = pw[buf][1][qb + 1][lane];
                    }
                    if constexpr (NPART == 1) {
                        // one FP16 product against the scaled FP16 copy
#pragma unroll
                        for (int db = 0; db < NDB; ++db)
                            o[qb][db] = mfma_h(as_h8(yold[0][db]), as_h8(ph), o[qb][db]);
                        if constexpr (NG == 2) {
#pragma unroll
                            for (int db = 0; db < NDB; ++db)
                                o[qb][db] = mfma_h(as_h8(yold[1][db]), as_h8(pl), o[qb][db]);
                        }
                    } else {
#pragma unroll
                        for (int db = 0; db < NDB; ++db) o[qb][db] = mfma_bf(yold[0][db], ph, o[qb][db]);
#pragma unroll
                        for (int db = 0; db < NDB; ++db) o[qb][db] = mfma_bf(yold[1][db], ph, o[qb][db]);
                        // the lo weights against the hi copy: the third product of the split
#pragma unroll
                        for (int db = 0; db < NDB; ++db) o[qb][db] = mfma_bf(yold[0][db], pl, o[qb][db]);
                    }
                    // the rows go out over the first blocks
                    if (2 * qb < NLD) load_rows_part(tr, sb, 2 * qb);
                    if (2 * qb + 1 < NLD) load_rows_part(tr, sb, 2 * qb + 1);
                    ph = phn;
                    pl = pln;
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
                for (int k = 2 * NQ; k < NLD; ++k) load_rows_part(tr, sb, k);
            }
            store_bias(sb);
            // the rows must be in LDS before the score waves pass the barrier
            __builtin_amdgcn_s_waitcnt(kWaitVmem);
            __syncthreads();
        };
        // interval 0 stages only (tile 1's rows, tile 0's fragments); the
        // loop runs whole pairs, so no branch in it joins the accumulators
        fetch_bias(min(1, last));
#pragma unroll
        for (int k = 0; k < NLD; ++k) load_rows_part(min(1, last), 1, k);
#pragma unroll
        for (int k = 0; k < NYG * NDB; ++k) load_yv_part(0, yv, k);
        store_bias(1);
        __builtin_amdgcn_s_waitcnt(kWaitVmem);
        __syncthreads();
        int t = 1;
        for (; t + 1 <= ntiles; t += 2) {
            body(t, yw, yv);
            body(t + 1, yv, yw);
        }
        if (t <= ntiles) body(t, yw, yv);
        __syncthreads();                   // normalisers written
#pragma unroll
        for (int qb = 0; qb < NQ; ++qb) {
            const int64_t r = blk0 + qb * 16 + li;
            if (r >= nq) continue;
            // the FP16 copy holds Y scaled by a power of two: undo it exactly
            const float inv = (NPART == 1 ? *yt_unscale : 1.f) / lw[qb * 16 + li];
#pragma unroll
            for (int db = 0; db < NDB; ++db) {
                const int f0 = (pv * NDB + db) * 16 + 4 * lq;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (f0 + e < d) {
                        const float xo = Xq[r * d + f0 + e];
                        Xout[r * d + f0 + e] = (1.f - alpha) * xo + alpha * (o[qb][db][e] * inv);
                    }
                }
            }
        }
    }
}

// BF16 hi/lo copies of the rows of X in the tile layout, rows padded to
// np = bf16_mpad(n) and features to D with zeros: element (i, k) of part p
// at p np D + ((i / 16) (D / 8) + k / 8) 128 + (i % 16) 8 + k % 8.  One
// thread per destination element.
__global__ __launch_bounds__(256) void bf16_split_rows(const float *__restrict__ X, int64_t n, int d,
                                                       int D, int64_t np, __bf16 *__restrict__ lp) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= np * D) return;
    const int C = D / 8;
    const int64_t bc = e >> 7;                    // (i / 16) C + k / 8
    const int64_t i = (bc / C) * 16 + ((e >> 3) & 15);
    const int k = (int)(bc % C) * 8 + (int)(e & 7);
    const float x = (i < n && k < d) ? X[i * d + k] : 0.f;
    const __bf16 h = (__bf16)x;
    lp[e] = h;
    lp[np * D + e] = (__bf16)(x - (float)h);
}

// Transposed hi/lo copies of Y for the projection product, one block of
// D x 32 per group of 32 columns (tile t), in the tile layout with the
// dimensions as rows: element (dim, position q) of tile t of part p at
// p mp D + t 32 D + ((dim / 16) 4 + q / 8) 128 + (dim % 16) 8 + q % 8,
// holding column 32 t + perm32(q) (zero beyond m and d).
__global__ __launch_bounds__(256) void bf16_transpose(const float *__restrict__ Y, int64_t m, int d,
                                                      int D, int64_t mp, __bf16 *__restrict__ yt) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= mp * D) return;
    const int nblk = D / 4;                       // 16-chunk blocks per tile
    const int64_t rest = e >> 7;
    const int blk = (int)(rest % nblk);
    const int64_t t = rest / nblk;
    const int dim = (blk >> 2) * 16 + (int)((e >> 3) & 15);
    const int q = (blk & 3) * 8 + (int)(e & 7);
    const int64_t j = 32 * t + perm32(q);
    const float y = (j < m && dim < d) ? Y[j * d + dim] : 0.f;
    const __bf16 h = (__bf16)y;
    yt[e] = h;
    yt[mp * D + e] = (__bf16)(y - (float)h);
}

// max |y| over a cloud, as the bits of a non-negative float (which order like
// the floats): each workgroup reduces its grid-stride share and combines it
// with one atomicMax into *out (zeroed beforehand).
__global__ __launch_bounds__(256) void absmax_f32(const float *__restrict__ Y, int64_t count,
                                                  unsigned *__restrict__ out) {
    __shared__ float wmax[4];
    float v = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
        v = fmaxf(v, fabsf(Y[i]));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(out, __float_as_uint(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]))));
}

// The transposed copy of the plain BF16 form's projection: one FP16 part,
// Y scaled by 2^k with k the largest integer such that max |y| 2^k <= 2^14
// (exact scaling; far from FP16's overflow and subnormal ranges), in the
// layout of bf16_transpose.  unscale = 2^-k undoes it after the product.
__global__ __launch_bounds__(256) void f16_transpose(const float *__restrict__ Y, int64_t m, int d,
                                                     int D, int64_t mp, const unsigned *__restrict__ amax,
                                                     _Float16 *__restrict__ yt, float *__restrict__ unscale) {
    const float mx = __uint_as_float(*amax);
    int k = 0;
    if (mx > 0.f && mx < INFINITY) {
        int e;
        (void)frexpf(16384.f / mx, &e);   // 16384 / mx = f 2^e, f in [0.5, 1)
        k = min(e - 1, 126);
    }
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e == 0) *unscale = ldexpf(1.f, -k);
    if (e >= mp * D) return;
    const int nblk = D / 4;
    const int64_t rest = e >> 7;
    const int blk = (int)(rest % nblk);
    const int64_t t = rest / nblk;
    const int dim = (blk >> 2) * 16 + (int)((e >> 3) & 15);
    const int q = (blk & 3) * 8 + (int)(e & 7);
    const int64_t j = 32 * t + perm32(q);
    const float y = (j < m && dim < d) ? Y[j * d + dim] : 0.f;
    yt[e] = (_Float16)ldexpf(y, k);
}

// PROGOT_BF16_SHIFT (read at every launch): unset, the fixed exponent shift
// wherever the job carries the previous potential; "off", the running
// maximum only; "recheck", every fixed-shift sweep fails its range check and
// is redone with the running maximum (the fallback, which then computes the
// same bits as "off").
enum class ShiftMode { kAuto, kOff, kRecheck };
ShiftMode shift_mode() {
    const char *e = std::getenv("PROGOT_BF16_SHIFT");
    if (!e) return ShiftMode::kAuto;
    if (!std::strcmp(e, "off")) return ShiftMode::kOff;
    if (!std::strcmp(e, "recheck")) return ShiftMode::kRecheck;
    return ShiftMode::kAuto;
}

template <int D, int NPART>
hipError_t lse_bf16_t(const LseJob &a, hipStream_t s) {
    constexpr int QB = lse_shape(D, NPART).qb, BN = lse_shape(D, NPART).bn;
    // the plan must cover every row tile of this kernel variant, and splits
    // must start on the 64-column boundaries of the padded copy
    if (a.blocks != (a.nu + 64 * QB - 1) / (64 * QB) * a.S || a.cps % 64 != 0)
        return hipErrorInvalidValue;
    const int64_t vstride = bf16_mpad(a.nv) * D;
    const ShiftMode mode = shift_mode();
    const float *shift = mode == ShiftMode::kOff ? nullptr : a.shift_pot;
    const float sum_hi = mode == ShiftMode::kRecheck ? -1.f : kSumHi;
    timed_launch(0, lse_partial_bf16<D, QB, NPART, BN>, dim3((unsigned)a.blocks), dim3(256), 0, s, a.U,
                 a.nu, a.d, (const __bf16 *)a.V_lp, a.nv, vstride, a.vsq, a.vpot, a.gamma, a.scale2,
                 a.bscale, a.S, a.cps, a.part_m, a.part_s, shift, a.usq, a.logw, a.eps, sum_hi,
                 a.shift_gamma);
    return hipGetLastError();
}

template <int D, int NQB, int NPART, int NG = 1>
hipError_t map_bf16_ws_t(const MapArgs &a, float scale2, float bscale, hipStream_t s) {
    if (a.m < 1 || a.mp != bf16_mpad(a.m) || a.out_sqn || (NPART == 1 && !a.yt_unscale))
        return hipErrorInvalidValue;
    // every column tile the kernel reads must lie in the padded copies
    constexpr int64_t BN = (int64_t)kMapBN * NG;
    if ((a.m + BN - 1) / BN * BN > a.mp) return hipErrorInvalidValue;
    constexpr int ROWS = 64 * NQB;
    const int64_t tiles = (a.nq + ROWS - 1) / ROWS;
    timed_launch(1, entropic_map_bf16_ws<D, NQB, NPART, NG>, dim3((unsigned)tiles), dim3(512), 0, s, a.Xq,
                 a.nq, a.d, (const __bf16 *)a.Y_lp, (const __bf16 *)a.YT_lp, a.m, a.mp, a.ysq, a.g,
                 scale2, bscale, a.alpha, a.Xout, a.yt_unscale);
    return hipGetLastError();
}

template <int D, int QB, int NPART, int NG>
hipError_t map_bf16_t(const MapArgs &a, float scale2, float bscale, hipStream_t s) {
    if (a.mp != bf16_mpad(a.m)) return hipErrorInvalidValue;
    // every column tile the kernel reads must lie in the padded copies
    constexpr int64_t BN = (int64_t)kMapBN * NG;
    if ((a.m + BN - 1) / BN * BN > a.mp) return hipErrorInvalidValue;
    const int64_t tiles = (a.nq + 64 * QB - 1) / (64 * QB);
    if (NPART == 1 && !a.yt_unscale) return hipErrorInvalidValue;
    timed_launch(1, entropic_map_bf16<D, QB, NPART, NG>, dim3((unsigned)tiles), dim3(256), 0, s, a.Xq,
                 a.nq, a.d, (const __bf16 *)a.Y_lp, (const __bf16 *)a.YT_lp, a.m, a.mp, a.ysq, a.g,
                 scale2, bscale, a.alpha, a.Xout, a.out_sqn, a.yt_unscale);
    return hipGetLastError();
}

}  // namespace

int bf16_dim(int d) {
    if (d <= 32) return 32;
    if (d <= 64) return 64;
    if (d <= 128) return 128;
    return 256;
}

// Rows of the BF16 copies: a multiple of 128, so that every column tile the
// kernels read (potential tiles of up to 64 columns from 64-column split
// boundaries, map tiles of up to 128 columns from 0) lies in the copy.
int64_t bf16_mpad(int64_t m) { return (m + 127) / 128 * 128; }

// Rows per workgroup: 4 waves x QB x 16 (lse_shape).
int lse_bf16_rows_per_block(int d, int precision) {
    return 64 * lse_shape(bf16_dim(d), precision == 2 ? 2 : 1).qb;
}

hipError_t launch_lse_partial_bf16(const LseJob &a, hipStream_t s) {
    const bool x3 = a.precision == 2;
    switch (bf16_dim(a.d)) {
        case 32: return x3 ? lse_bf16_t<32, 2>(a, s) : lse_bf16_t<32, 1>(a, s);
        case 64: return x3 ? lse_bf16_t<64, 2>(a, s) : lse_bf16_t<64, 1>(a, s);
        case 128: return x3 ? lse_bf16_t<128, 2>(a, s) : lse_bf16_t<128, 1>(a, s);
        default: return x3 ? lse_bf16_t<256, 2>(a, s) : lse_bf16_t<256, 1>(a, s);
    }
}

hipError_t launch_map_bf16(const MapArgs &a, float scale2, float bscale, hipStream_t s) {
    const bool x3 = a.precision == 2;
    switch (bf16_dim(a.d)) {
        // D <= 64: the narrow kernel, two 16-row blocks per wave (four
        // measured 23-27 % slower: two waves per SIMD instead of three or
        // four).  Columns per tile (32 NG): every tile pays one dependent
        // score -> softmax -> projection chain, a cross-lane maximum and a
        // barrier, so wider tiles win where the registers allow; measured at
        // 65536^2 against 32 columns: plain BF16 128 columns (-36 % at D = 32,
        // -24 % at D = 64), BF16X3 64 (-6 %, -1 %)
        case 32: return x3 ? map_bf16_t<32, 2, 2, 2>(a, scale2, bscale, s) : map_bf16_t<32, 2, 1, 4>(a, scale2, bscale, s);
        case 64: return x3 ? map_bf16_t<64, 2, 2, 2>(a, scale2, bscale, s) : map_bf16_t<64, 2, 1, 4>(a, scale2, bscale, s);
        // D = 128 and 256: the warp-specialised kernel (it writes no
        // |Xout_i|^2, which the library asks of the FP32 maps only), 65536^2:
        // BF16X3 4.65-4.8 ms instead of 5.45-5.55 for the narrow kernel at
        // D = 128, 8.9-9.4 ms instead of 12.5 for the previous D = 256 kernel;
        // plain BF16 with 64-column tiles 1.95-2.0 ms instead of 2.26-2.49 at
        // D = 128 (the narrow kernel's 64-column tiles, same bits) and 3.5 ms
        // instead of 5.8 at D = 256 (3.7-3.9 with 32-column tiles)
        case 128: return x3 ? map_bf16_ws_t<128, 4, 2>(a, scale2, bscale, s) : map_bf16_ws_t<128, 4, 1, 2>(a, scale2, bscale, s);
        default: return x3 ? map_bf16_ws_t<256, 2, 2>(a, scale2, bscale, s) : map_bf16_ws_t<256, 2, 1, 2>(a, scale2, bscale, s);
    }
}

hipError_t launch_bf16_rows(const float *X, int64_t n, int d, void *lp, hipStream_t s) {
    const int D = bf16_dim(d);
    const int64_t np = bf16_mpad(n);
    const int64_t tot = np * D;
    hipLaunchKernelGGL(bf16_split_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, X, n, d, D,
                       np, (__bf16 *)lp);
    return hipGetLastError();
}

hipError_t launch_f16_transpose(const float *Y, int64_t m, int d, void *yt, float *scale2, hipStream_t s) {
    const int D = bf16_dim(d);
    const int64_t mp = bf16_mpad(m);
    const int64_t tot = mp * D;
    unsigned *amax = reinterpret_cast<unsigned *>(scale2);
    hipError_t e = hipMemsetAsync(amax, 0, sizeof(unsigned), s);
    if (e != hipSuccess) return e;
    const int64_t cnt = m * (int64_t)d;
    const int64_t blocks = std::min<int64_t>((cnt + 255) / 256, 1024);
    hipLaunchKernelGGL(absmax_f32, dim3((unsigned)blocks), dim3(256), 0, s, Y, cnt, amax);
    hipLaunchKernelGGL(f16_transpose, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Y, m, d, D, mp,
                       amax, (_Float16 *)yt, scale2 + 1);
    return hipGetLastError();
}

hipError_t launch_bf16_transpose(const float *Y, int64_t m, int d, void *yt, hipStream_t s) {
    const int D = bf16_dim(d);
    const int64_t mp = bf16_mpad(m);
    const int64_t tot = mp * D;
    hipLaunchKernelGGL(bf16_transpose, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, Y, m, d, D,
                       mp, (__bf16 *)yt);
    return hipGetLastError();
}

}  // namespace pot
