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
#include "progot_device.h"

#include <algorithm>
#include <cmath>

namespace pot {
namespace {

// LDS tile layout.  A tile of BN columns x D features is stored as 16-byte
// chunks (4 features): chunk c of tile row j sits at chunk index
//   ((j / 16) * C + c) * 16 + ((j % 16) ^ (c % 4)),   C = D / 4,
// i.e. 16 rows per chunk column with the rows of chunk column c permuted by
// an XOR with c % 4.  On gfx950 a ds_read_b128 is conflict-free when each
// group of 16 consecutive lanes reads 16 chunks of one 256-byte block (padded
// row strides measured 2-way conflicted): the cross-term operand read -- lane
// (li, lq) takes chunk c of row 16 s + li -- is one such block per lane group.
// The XOR makes the map's projection read conflict-free as well: there lane
// (li, lq) takes feature 16 db + li of row 16 s + 4 lq + r (a ds_read_b32),
// and the permuted row 4 lq + (r ^ (li / 4)) puts the 64 lanes on 64
// distinct banks.
//
// The loader (TileSlot) gives each wave whole row segments: a wave reads
// 4 rows x 256 bytes (D >= 64), 8 rows x 128 or 16 rows x 64 bytes of
// consecutive rows (D = 32, 16), and each group of 16 lanes stores 4 rows x 4
// chunks, i.e. 4 blocks of LDS (4-way).  Reading 16 rows x 64 bytes per wave
// instead, with conflict-free stores, measured 1 % slower for the potential
// kernel and 6 % slower for the map at d = 64, 7-8 % slower for the potential
// kernel at d = 128 and 256: the tiles stream from L2 on every workgroup, and
// their cache-line efficiency counts for more than the stores, which are a
// quarter of the LDS instructions.
template <int D, int BN_ = (D >= 256 ? 32 : 64)> struct Tile {
    static constexpr int BN = BN_;                 // columns per LDS tile
    static constexpr int NSUB = BN / 16;           // 16-column subtiles
    static constexpr int KD = D / 4;               // features per lane group
    static constexpr int C = D / 4;                // 16-byte chunks per row
    static constexpr int NCH = BN * C;             // chunks per tile
    static constexpr int FLOATS = BN * D;          // LDS floats per tile
    static constexpr int PER_T = (NCH + 255) / 256;
};

// Float offset of chunk c of tile row j (layout above).
template <int D>
__device__ __forceinline__ int tchunk(int j, int c) {
    return (((j >> 4) * (D / 4) + c) * 16 + ((j & 15) ^ (c & 3))) * 4;
}

// Loader slot (thread tid, round r): tile row row0 + row_step(r), chunk
// cc0 + chunk_step(r).  Wave w covers whole row segments, each quarter of it
// 4 rows x 4 chunks (layout comment above); the round only adds compile-time
// offsets, so one base address per thread serves every round.
template <int D> struct TileSlot {
    static constexpr int C = D / 4;
    int row0, cc0;
    __device__ __forceinline__ explicit TileSlot(int tid) {
        if constexpr (C >= 16) {       // 16-row blocks of 16 C chunks, 256 chunks per round
            row0 = 4 * (tid >> 6) + ((tid & 15) >> 2);
            cc0 = 4 * ((tid >> 4) & 3) + (tid & 3);
        } else if constexpr (C == 8) { // waves of 8 rows x 8 chunks
            row0 = 16 * (tid >> 7) + 8 * ((tid >> 6) & 1) + 4 * ((tid >> 5) & 1) + ((tid & 15) >> 2);
            cc0 = 4 * ((tid >> 4) & 1) + (tid & 3);
        } else {                       // C == 4: waves of 16 rows x 4 chunks
            row0 = 16 * (tid >> 6) + 4 * ((tid >> 4) & 3) + ((tid & 15) >> 2);
            cc0 = tid & 3;
        }
    }
    static constexpr int row_step(int r) {
        return C >= 16 ? 16 * (r / (C / 16)) : C == 8 ? 32 * r : 64 * r;
    }
    static constexpr int chunk_step(int r) { return C >= 16 ? 16 * (r % (C / 16)) : 0; }
    // LDS float offset of round r relative to round 0 (row steps are whole
    // 16-row blocks and chunk steps multiples of 4, so the XOR term is fixed)
    static constexpr int lds_step(int r) { return ((row_step(r) >> 4) * C + chunk_step(r)) * 64; }
};

// Load one BN x D column tile (rows j0.., zero-padded beyond nv and beyond
// feature d) into registers: thread t takes loader slots t, t + 256, ...
template <int D, int BN>
__device__ __forceinline__ void tile_fetch(const float *__restrict__ V, int64_t nv, int d,
                                           int64_t j0, int tid, f4 (&pre)[Tile<D, BN>::PER_T]) {
    using T = Tile<D, BN>;
    using S = TileSlot<D>;
    static_assert(T::NCH % 256 == 0, "a tile is whole loader rounds");
    const S slot(tid);
    const int64_t jb = j0 + slot.row0;
    const int cb = 4 * slot.cc0;
#pragma unroll
    for (int r = 0; r < T::PER_T; ++r) {
        f4 v = {0.f, 0.f, 0.f, 0.f};
        const int64_t j = jb + S::row_step(r);
        const int c = cb + 4 * S::chunk_step(r);
        if (j < nv) {
            if (d == D) {
                v = ldg(reinterpret_cast<const f4 *>(V + jb * D + cb) +
                        (S::row_step(r) * D + 4 * S::chunk_step(r)) / 4);
            } else {
                const float *p = V + j * d;
                v.x = c + 0 < d ? ldg(p + c + 0) : 0.f;
                v.y = c + 1 < d ? ldg(p + c + 1) : 0.f;
                v.z = c + 2 < d ? ldg(p + c + 2) : 0.f;
                v.w = c + 3 < d ? ldg(p + c + 3) : 0.f;
            }
        }
        pre[r] = v;
    }
}

// The loads of tile_fetch with the full-width test taken once for the
// tile: with the two forms side by side in every round, the map's register
// allocation at D <= 64 had the narrow form's targets share registers with
// the wide form's address, and the compiler waited for every earlier load
// before each round's 16-byte load, one round trip per round.
template <int D, int BN>
__device__ __forceinline__ void tile_fetch_wide_first(const float *__restrict__ V, int64_t nv, int d,
                                                      int64_t j0, int tid,
                                                      f4 (&pre)[Tile<D, BN>::PER_T]) {
    using T = Tile<D, BN>;
    using S = TileSlot<D>;
    const S slot(tid);
    const int64_t jb = j0 + slot.row0;
    const int cb = 4 * slot.cc0;
    if (d == D) {
        const f4 *base = reinterpret_cast<const f4 *>(V + jb * D + cb);
#pragma unroll
        for (int r = 0; r < T::PER_T; ++r) {
            f4 v = {0.f, 0.f, 0.f, 0.f};
            if (jb + S::row_step(r) < nv) v = ldg(base + (S::row_step(r) * D + 4 * S::chunk_step(r)) / 4);
            pre[r] = v;
        }
    } else {
        tile_fetch<D, BN>(V, nv, d, j0, tid, pre);
    }
}

template <int D, int BN>
__device__ __forceinline__ void tile_store(float *__restrict__ lds, int tid,
                                           const f4 (&pre)[Tile<D, BN>::PER_T]) {
    using T = Tile<D, BN>;
    using S = TileSlot<D>;
    const S slot(tid);
    float *base = lds + tchunk<D>(slot.row0, slot.cc0);
#pragma unroll
    for (int r = 0; r < T::PER_T; ++r) *reinterpret_cast<f4 *>(base + S::lds_step(r)) = pre[r];
}

// The thread id, hidden from loop-invariant code motion: in the persistent
// kernels the bodies run once per work item, and without this the compiler
// hoists every lane-dependent address out of the item loop and keeps it live
// across items, which pushed the D = 128 kernels into register spills.
template <int NT = 256>
__device__ __forceinline__ int item_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    __builtin_assume(t >= 0 && t < NT);
    return t;
}

// Partial log-sum-exp of t_ij over one column split, for ROWS = 64*QB rows
// (row tile `tile`, column split `split` of job J).
// Output: part_m/part_s[split*nu + i] = (max, sum 2^{t - max}) in log2 units.
// Column tile of the potential kernel (128 columns at D = 64 measured 6 %
// slower than 64: one workgroup fewer per CU by LDS).
constexpr int lse_bn(int D) { return D >= 256 ? 32 : 64; }
template <int D> using LseTile = Tile<D, lse_bn(D)>;

template <int D, int QB>
__device__ __forceinline__ void lse_partial_body(const LseJob &J, int64_t tile, int split,
                                                 float (&vt)[2][LseTile<D>::FLOATS],
                                                 float (&bt)[2][LseTile<D>::BN]) {
    using T = LseTile<D>;
    constexpr int ROWS = 64 * QB;
    const float *__restrict__ U = J.U;
    const float *__restrict__ V = J.V;
    const float *__restrict__ vsq = J.vsq;
    const float *__restrict__ vpot = J.vpot;
    const int64_t nu = J.nu, nv = J.nv;
    const int d = J.d;
    const float gamma = J.gamma, scale2 = J.scale2, bscale = J.bscale;
    const int64_t cols_per_split = J.cps;
    float *__restrict__ part_m = J.part_m;
    float *__restrict__ part_s = J.part_s;

    const int tid = item_tid();
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int64_t row0 = tile * ROWS + wave * (QB * 16);

    // rows held already multiplied by scale2 (and kept in registers: the
    // empty asm stops the compiler from re-deriving them inside the loop)
    float ub[QB][T::KD];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        row_fetch<D>(U, nu, d, row0 + qb * 16 + li, lq, ub[qb]);
#pragma unroll
        for (int k = 0; k < T::KD; ++k) {
            ub[qb][k] *= scale2;
            asm volatile("" : "+v"(ub[qb][k]));
        }
    }

    float run_m[QB], run_s[QB];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) { run_m[qb] = kNegBig; run_s[qb] = 0.f; }

    const int64_t c0 = (int64_t)split * cols_per_split;
    const int64_t c1 = c0 + cols_per_split < nv ? c0 + cols_per_split : nv;
    const int ntiles = c0 < c1 ? (int)((c1 - c0 + T::BN - 1) / T::BN) : 0;

    f4 pre[T::PER_T];
    // Column biases of the next tile: the raw values load with the tile and
    // are combined where they are stored, after the tile's products, so that
    // no wave waits on its loads (nor on the tile's, issued before them)
    // ahead of its MFMAs.  Index clamped into the split; past it the bias is
    // -inf.  The product is rounded on its own, as the plain expression is.
    int64_t jpre = 0;
    float gpre = 0.f, ypre = 0.f;
    auto fetch_beta = [&](int64_t j0) {
        jpre = j0 + tid;
        if (tid < T::BN) {
            const int64_t jc = jpre < c1 ? jpre : c1 - 1;
            gpre = vpot ? ldg(vpot + jc) : 0.f;
            ypre = ldg(vsq + jc);
        }
    };
    auto beta_pre = [&]() {
        return jpre < c1 ? ((vpot ? __fmul_rn(gamma, gpre) : 0.f) - ypre) * bscale : -INFINITY;
    };
    if (ntiles > 0) {
        tile_fetch<D, T::BN>(V, c1, d, c0, tid, pre);
        fetch_beta(c0);
        tile_store<D, T::BN>(vt[0], tid, pre);
        if (tid < T::BN) bt[0][tid] = beta_pre();
    }
    __syncthreads();

    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        const bool more = t + 1 < ntiles;
        if (more) {
            const int64_t jn = c0 + (int64_t)(t + 1) * T::BN;
            tile_fetch<D, T::BN>(V, c1, d, jn, tid, pre);
            fetch_beta(jn);
        }
        const float *vb = vt[buf];
        // raised wave priority while the products issue, so that a SIMD's
        // other wave, in its exponentials, yields the issue slot to them
        // (same bits; d = 256 1.7 % faster, d = 64 0-0.3 %)
        __builtin_amdgcn_s_setprio(1);
        // accumulators start at beta_j: the MFMA output is the exponent t_ij
        f4 acc[QB][T::NSUB];
#pragma unroll
        for (int sub = 0; sub < T::NSUB; ++sub) {
            const f4 beta = *reinterpret_cast<const f4 *>(&bt[buf][sub * 16 + lq * 4]);
            float a[T::KD];
#pragma unroll
            for (int k = 0; k < T::KD / 4; ++k) {
                const f4 v = *reinterpret_cast<const f4 *>(vb + tchunk<D>(sub * 16 + li, lq * (T::KD / 4) + k));
                a[4 * k + 0] = v.x; a[4 * k + 1] = v.y; a[4 * k + 2] = v.z; a[4 * k + 3] = v.w;
            }
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) {
                f4 c = beta;
#pragma unroll
                for (int k = 0; k < T::KD; ++k) c = mfma4(a[k], ub[qb][k], c);
                acc[qb][sub] = c;
            }
        }
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            float mx = kNegBig;
#pragma unroll
            for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
                for (int r = 0; r < 4; ++r) mx = fmaxf(mx, acc[qb][sub][r]);
            const float mn = fmaxf(run_m[qb], mx);
            // partial sums start at the first subtile's terms (an add to 0
            // cannot be dropped by the compiler; the terms are never -0)
            float s4[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) s4[r] = ex2(acc[qb][0][r] - mn);
#pragma unroll
            for (int sub = 1; sub < T::NSUB; ++sub)
#pragma unroll
                for (int r = 0; r < 4; ++r) s4[r] += ex2(acc[qb][sub][r] - mn);
            run_s[qb] = fmaf(run_s[qb], ex2(run_m[qb] - mn), (s4[0] + s4[1]) + (s4[2] + s4[3]));
            run_m[qb] = mn;
        }
        if (more) {
            tile_store<D, T::BN>(vt[buf ^ 1], tid, pre);
            if (tid < T::BN) bt[buf ^ 1][tid] = beta_pre();
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
            stg(part_m + split * nu + row, m);
            stg(part_s + split * nu + row, s);
        }
    }
}

// One job.  Block b runs on XCD b mod 8, and each XCD's L2 fetches the rows
// and columns its blocks touch.  When the grid divides evenly (an even
// number of row tiles, S a multiple of 4), XCD x takes the row tiles of half
// x / 4 and the splits of quarter x % 4, row tile major: its L2 streams half
// the rows and a quarter of the columns.  Otherwise block b takes row tile
// b / S and split b mod S, which with S a multiple of 8 gives each XCD every
// row tile and an eighth of the columns (at n = m, 4.5 instead of 3 eighths
// of both clouds per XCD).  Either way each (row tile, split) pair is one
// block, so the partials are the same.
template <int D, int QB>
__global__ __launch_bounds__(256) void lse_partial_f32(LseJob J) {
    __shared__ float vt[2][LseTile<D>::FLOATS];
    __shared__ float bt[2][LseTile<D>::BN];
    const int64_t b = blockIdx.x, tiles = J.blocks / J.S;
    int64_t rt;
    int split;
    if (tiles % 2 == 0 && J.S % 4 == 0) {
        const int64_t x = b % 8, i = b / 8, sq = J.S / 4;
        rt = (x / 4) * (tiles / 2) + i / sq;
        split = (int)((x % 4) * sq + i % sq);
    } else {
        rt = b / J.S;
        split = (int)(b % J.S);
    }
    lse_partial_body<D, QB>(J, rt, split, vt, bt);
}

// Persistent grouped kernels.  A grouped launch covers the work list of many
// jobs (problems of different sizes, or the grid points of Alg. 4): item i of
// the list is workgroup-sized work of the job whose [begin, begin + blocks)
// range holds i.  The grid is at most the number of workgroups the chip holds
// at once, and workgroup w walks the items w, w + G, w + 2G, ... (G the grid
// size), a static walk every workgroup finishes.  Workgroup w runs on XCD
// w mod 8 and G is a multiple of 8, so an XCD always gets the items with one
// residue mod 8; the potential kernel's jobs start on multiples of 8 in the
// list and split their columns S ways (S a power of two), so with S >= 8 an
// XCD streams a fixed subset of the column splits through its own L2, as a
// flat launch of one job would.  Items run the same device body as the
// single-problem kernels, so a problem gets the same bits alone or grouped,
// whichever workgroup runs an item.

// The control word of a problem's Sinkhorn loop is nonzero once it stopped
// (written by an earlier launch on the stream; read as global memory).
__device__ __forceinline__ bool stopped(const int *ctl) {
    return *(volatile const __attribute__((address_space(1))) int *)ctl != 0;
}

template <int D, int QB>
__global__ __launch_bounds__(256) void lse_partial_f32_group(const LseJob *__restrict__ jobs, int njobs,
                                                             int64_t total) {
    __shared__ float vt[2][LseTile<D>::FLOATS];
    __shared__ float bt[2][LseTile<D>::BN];
    int j = 0;   // the walk's items increase, so the owning job only advances
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        while (j + 1 < njobs && jobs[j + 1].blk_begin <= item) ++j;
        const LseJob &J = jobs[j];
        const int64_t local = item - J.blk_begin;
        if (local >= J.blocks) continue;                 // alignment gap before the next job
        if (J.ctl && stopped(J.ctl)) continue;           // loop already stopped
        lse_partial_body<D, QB>(J, local / J.S, (int)(local % J.S), vt, bt);
        __syncthreads();
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
__device__ __forceinline__ void lse_merge_body(const LseJob &J, int64_t blk, float *red) {
    const float *__restrict__ part_m = J.part_m;
    const float *__restrict__ part_s = J.part_s;
    const int S = J.S;
    const int64_t nu = J.nu;
    const float eps = J.eps;
    const int64_t i = blk * 256 + threadIdx.x;
    float e = 0.f;
    if (i < nu) {
        // one pass over the splits, running (max, sum); unrolled so the
        // loads of several splits are in flight together
        float M = kNegBig, sum = 0.f;
#pragma unroll 8
        for (int s = 0; s < S; ++s) {
            const float m = ldg(part_m + s * nu + i), v = ldg(part_s + s * nu + i);
            const float Mn = fmaxf(M, m);
            sum = sum * exp2f(M - Mn) + v * exp2f(m - Mn);
            M = Mn;
        }
        const float L = M + log2f(sum);
        const float lw = ldg(J.logw + i);
        const float pot = fmaf(eps, lw, J.usq ? ldg(J.usq + i) : 0.f) - eps * kLn2 * L;
        if (J.pot_old) e = expf(lw) * fabsf(expm1f((ldg(J.pot_old + i) - pot) / eps));
        stg(J.pot_out + i, pot);
    }
    if (J.pot_old) {
        const float tot = block_sum_256(e, red);
        if (threadIdx.x == 0) stg(J.err_part + blk, tot);
    }
}

__global__ __launch_bounds__(256) void lse_merge(LseJob J) {
    __shared__ float red[256];
    lse_merge_body(J, blockIdx.x, red);
}

__global__ __launch_bounds__(256) void lse_merge_group(const LseJob *__restrict__ jobs, int njobs,
                                                      int64_t total) {
    __shared__ float red[256];
    int j = 0;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        while (j + 1 < njobs && jobs[j + 1].mblk_begin <= item) ++j;
        const LseJob &J = jobs[j];
        if (J.ctl && stopped(J.ctl)) continue;   // loop already stopped
        lse_merge_body(J, item - J.mblk_begin, red);
        __syncthreads();
    }
}

__device__ __forceinline__ void sum_body(const float *__restrict__ part, int n, float *out,
                                         float *red) {
    float v = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) v += part[i];
    const float tot = block_sum_256(v, red);
    if (threadIdx.x == 0) out[0] = tot;
}

// Error sums of the jobs that carry pot_old, one block each, in job order;
// with a control word, also the device-side stop rule of the Sinkhorn loop.
__global__ __launch_bounds__(256) void sum_group(const LseJob *__restrict__ jobs, int njobs,
                                                 float *__restrict__ out) {
    __shared__ float red[256];
    __shared__ float tot;
    int k = 0, b = blockIdx.x;
    for (int j = 0; j < njobs; ++j) {
        const LseJob &J = jobs[j];
        if (!J.pot_old) continue;
        if (k == b) {
            if (J.ctl && *(volatile const int *)J.ctl != 0) return;
            sum_body(J.err_part, (int)J.mblocks, &tot, red);
            if (threadIdx.x == 0) {
                const float err = tot;
                if (out) out[k] = err;
                if (J.ctl && ((J.tau > 0.f && err <= J.tau) || J.iter >= J.max_iter || !(err == err))) {
                    J.ctl[1] = __float_as_int(err);
                    J.ctl[0] = J.iter;
                }
            }
            return;
        }
        ++k;
    }
}

__global__ __launch_bounds__(256) void sum_f32(const float *__restrict__ part, int n, float *__restrict__ out) {
    __shared__ float red[256];
    sum_body(part, n, out, red);
}

// Squared norms (FP64 accumulation), optional BF16 copy.
__global__ __launch_bounds__(256) void cloud_norms(const float *__restrict__ X, int64_t n, int d,
                                                   float *__restrict__ sqn) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float *x = X + i * d;
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
        const double v = x[k];
        s += v * v;
    }
    sqn[i] = (float)s;
}

// Per-block FP64 sums of every feature and of |x|^2 over a contiguous row
// range.  The 256 threads form G = 256/d groups of d threads (1 <= d <= 256):
// thread f of group g adds feature f of rows r0 + g, r0 + g + G, ... (a group
// reads whole rows, so the loads are contiguous), and the G group sums are
// folded in LDS in group order, so the result is deterministic.
__global__ __launch_bounds__(256) void cloud_stats(const float *__restrict__ X, int64_t n, int d,
                                                   const float *__restrict__ sqn, int64_t rows_per_blk,
                                                   double *__restrict__ part) {
    __shared__ double red[256];
    const int tid = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
    const int64_t r1 = r0 + rows_per_blk < n ? r0 + rows_per_blk : n;
    const int G = 256 / d;
    const int g = tid / d, f = tid - g * d;
    double s = 0.0;
    if (g < G)
        for (int64_t r = r0 + g; r < r1; r += G) s += X[r * d + f];
    red[tid] = s;
    __syncthreads();
    if (tid < d) {
        double t = 0.0;
        for (int k = 0; k < G; ++k) t += red[k * d + tid];
        part[(int64_t)blockIdx.x * (d + 1) + tid] = t;
    }
    __syncthreads();
    double q = 0.0;
    for (int64_t r = r0 + tid; r < r1; r += 256) q += sqn[r];
    red[tid] = q;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) part[(int64_t)blockIdx.x * (d + 1) + d] = red[0];
}

// Fold nblk x (d+1) partials (nblk <= 256) into the first row: workgroup f
// folds column f, thread t taking partial t, then a halving tree in LDS, so
// the order is fixed.  Each workgroup writes only the element of the first
// row that it alone reads.
__global__ __launch_bounds__(256) void stats_fold(double *__restrict__ part, int nblk, int d) {
    __shared__ double red[256];
    const int f = blockIdx.x, tid = threadIdx.x;
    red[tid] = tid < nblk ? part[(int64_t)tid * (d + 1) + f] : 0.0;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
    }
    if (tid == 0) part[f] = red[0];
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
// As in the potential kernel the query rows are held already multiplied by
// scale2 and the column bias beta_j is the accumulator's initial value, so
// the score MFMA yields the log2-domain exponent t_ij itself.  The online
// softmax keeps a running maximum per query (shared by the 4 lane groups).
// With KS = 2 the workgroup is two groups of four waves on the same queries,
// each streaming every other column tile through LDS tiles of its own, and
// their online-softmax states merge at the end: twice the waves per query
// tile, for maps whose query count alone gives the chip one wave per SIMD
// (16384 queries are 256 workgroups).
template <int D, int QB, int KS>
__device__ __forceinline__ void entropic_map_body(const float *Xq, int64_t nq, int d,
                                                  const float *__restrict__ Y,
                                                  const float *__restrict__ ysq,
                                                  const float *__restrict__ g, int64_t m,
                                                  float scale2, float bscale, float alpha, float *Xout,
                                                  float *__restrict__ out_sqn, int64_t tile,
                                                  float (&vts)[KS][2][Tile<D>::FLOATS],
                                                  float (&bts)[KS][2][Tile<D>::BN]) {
    using T = Tile<D>;
    constexpr int ROWS = 64 * QB;
    constexpr int NDB = D / 16;   // 16-feature blocks of the output
    static_assert(KS == 1 || (KS == 2 && QB == 1), "two column groups, one row block per wave");
    static_assert(KS == 1 || (2 + 4 * NDB) * 256 <= KS * 2 * T::FLOATS, "the group exchange fits in the tiles");

    // column group (KS = 2: threads 256 grp .. 256 grp + 255) and its tiles
    const int tid_all = item_tid<256 * KS>();
    const int grp = KS == 1 ? 0 : __builtin_amdgcn_readfirstlane(tid_all >> 8);   // wave-uniform
    const int tid = tid_all & 255;
    float (&vt)[2][T::FLOATS] = vts[grp];
    float (&bt)[2][T::BN] = bts[grp];
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lq = lane >> 4;
    const int64_t row0 = tile * ROWS + wave * (QB * 16);

    float ub[QB][T::KD];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        row_fetch<D>(Xq, nq, d, row0 + qb * 16 + li, lq, ub[qb]);
#pragma unroll
        for (int k = 0; k < T::KD; ++k) {
            ub[qb][k] *= scale2;
            asm volatile("" : "+v"(ub[qb][k]));
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
    // lane part of the projection read: row 4 lq + (r ^ (li / 4)) of a
    // 16-row block, feature li of a 16-feature block (layout of tchunk)
    int pv_off[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        pv_off[r] = ((li >> 2) * 16 + 4 * lq + (r ^ (li >> 2))) * 4 + (li & 3);

    // group grp takes column tiles grp, grp + KS, grp + 2 KS, ...; both
    // groups run niter iterations (one barrier each), a group past its last
    // tile idling through them
    const int ntiles = (int)((m + T::BN - 1) / T::BN);
    const int niter = (ntiles + KS - 1) / KS;
    auto has_tile = [&](int t) { return KS * t + grp < ntiles; };
    auto tile_col = [&](int t) { return (int64_t)(KS * t + grp) * T::BN; };
    f4 pre[T::PER_T];
    // column biases of the next tile, combined where they are stored (as in
    // the potential kernel)
    int64_t jpre = 0;
    float gpre = 0.f, ypre = 0.f;
    auto fetch_beta = [&](int64_t j0) {
        jpre = j0 + tid;
        if (tid < T::BN) {
            const int64_t jc = jpre < m ? jpre : m - 1;
            gpre = ldg(g + jc);
            ypre = ldg(ysq + jc);
        }
    };
    auto beta_pre = [&]() { return jpre < m ? (gpre - ypre) * bscale : -INFINITY; };
    if (has_tile(0)) {
        tile_fetch_wide_first<D, T::BN>(Y, m, d, tile_col(0), tid, pre);
        fetch_beta(tile_col(0));
        tile_store<D, T::BN>(vt[0], tid, pre);
        if (tid < T::BN) bt[0][tid] = beta_pre();
    }
    __syncthreads();

    for (int t = 0; t < niter; ++t) {
        const int buf = t & 1;
        const bool more = has_tile(t + 1);
        if (more) {
            const int64_t jn = tile_col(t + 1);
            tile_fetch_wide_first<D, T::BN>(Y, m, d, jn, tid, pre);
            fetch_beta(jn);
        }
        // KS = 1: always true (t < niter = ntiles)
        if (KS == 1 || has_tile(t)) {
        const float *vb = vt[buf];
        // accumulators start at beta_j; k outer, (column subtile, row block)
        // inner: NSUB x QB independent accumulation chains
        f4 acc[QB][T::NSUB];
#pragma unroll
        for (int sub = 0; sub < T::NSUB; ++sub) {
            const f4 beta = *reinterpret_cast<const f4 *>(&bt[buf][sub * 16 + lq * 4]);
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) acc[qb][sub] = beta;
        }
#pragma unroll
        for (int k4 = 0; k4 < T::KD / 4; ++k4) {
            f4 a[T::NSUB];
#pragma unroll
            for (int sub = 0; sub < T::NSUB; ++sub)
                a[sub] = *reinterpret_cast<const f4 *>(vb + tchunk<D>(sub * 16 + li, lq * (T::KD / 4) + k4));
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
                    for (int qb = 0; qb < QB; ++qb)
                        acc[qb][sub] = mfma4(a[sub][kk], ub[qb][4 * k4 + kk], acc[qb][sub]);
        }
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            float mx = kNegBig;
#pragma unroll
            for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
                for (int r = 0; r < 4; ++r) mx = fmaxf(mx, acc[qb][sub][r]);
            mx = max_lane_groups(mx);
            const float mn = fmaxf(run_m[qb], mx);
            // rescale every tile: a wave-uniform test to skip it when no
            // maximum rose measured 2 % slower than the multiplies it saves
            const float c = ex2(run_m[qb] - mn);
            run_l[qb] *= c;
#pragma unroll
            for (int db = 0; db < NDB; ++db) o[qb][db] *= c;
            run_m[qb] = mn;
            float p[T::NSUB * 4];
            float s = 0.f;
#pragma unroll
            for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    p[sub * 4 + r] = ex2(acc[qb][sub][r] - mn);
                    s += p[sub * 4 + r];
                }
            run_l[qb] += s;
#pragma unroll
            for (int sub = 0; sub < T::NSUB; ++sub)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float *yb = vb + sub * 16 * D + pv_off[r];
#pragma unroll
                    for (int db = 0; db < NDB; ++db)
                        o[qb][db] = mfma4(yb[db * 256], p[sub * 4 + r], o[qb][db]);
                }
        }
        }
        if (more) {
            tile_store<D, T::BN>(vt[buf ^ 1], tid, pre);
            if (tid < T::BN) bt[buf ^ 1][tid] = beta_pre();
        }
        __syncthreads();
    }

    if constexpr (KS == 2) {
        // group 1 hands its (max, sum, output) to group 0 through the tiles,
        // free after the loop's last barrier; group 0 rescales both to the
        // larger maximum and adds them
        float *xch = &vts[0][0][0];
        if (grp == 1) {
            xch[tid] = run_m[0];
            xch[256 + tid] = run_l[0];
#pragma unroll
            for (int db = 0; db < NDB; ++db)
#pragma unroll
                for (int r = 0; r < 4; ++r) xch[(2 + 4 * db + r) * 256 + tid] = o[0][db][r];
        }
        __syncthreads();
        if (grp == 0) {
            const float m1 = xch[tid];
            const float mn = fmaxf(run_m[0], m1);
            const float c0 = ex2(run_m[0] - mn), c1 = ex2(m1 - mn);
            run_l[0] = run_l[0] * c0 + xch[256 + tid] * c1;
#pragma unroll
            for (int db = 0; db < NDB; ++db)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    o[0][db][r] = o[0][db][r] * c0 + xch[(2 + 4 * db + r) * 256 + tid] * c1;
            run_m[0] = mn;
        }
    }

    if (grp != 0) return;   // the merged state is group 0's; no barrier follows
    // the epilogue's lane coordinates, taken afresh so that no lane address
    // formed before the loop stays live through it
    const int etid = item_tid<256 * KS>() & 255;
    const int eli = etid & 15, elq = (etid & 63) >> 4;
    const int64_t erow0 = tile * ROWS + (etid >> 6) * (QB * 16);
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        float l = run_l[qb];
        l += __shfl_xor(l, 16);
        l += __shfl_xor(l, 32);
        const float inv = 1.f / l;
        const int64_t row = erow0 + qb * 16 + eli;
        double sq = 0.0;
        if (row < nq) {
            // the row's features of every block load first, together
            float xo[NDB][4];
            if (d == D) {
#pragma unroll
                for (int db = 0; db < NDB; ++db) {
                    const f4 v = ldg(reinterpret_cast<const f4 *>(Xq + row * D + db * 16 + 4 * elq));
                    xo[db][0] = v.x; xo[db][1] = v.y; xo[db][2] = v.z; xo[db][3] = v.w;
                }
            } else {
#pragma unroll
                for (int db = 0; db < NDB; ++db)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int f = db * 16 + 4 * elq + r;
                        xo[db][r] = f < d ? ldg(Xq + row * d + f) : 0.f;
                    }
            }
#pragma unroll
            for (int db = 0; db < NDB; ++db) {
                const int f0 = db * 16 + 4 * elq;
                if (f0 >= d) continue;
                float xn[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    xn[r] = (1.f - alpha) * xo[db][r] + alpha * (o[qb][db][r] * inv);
                    if (f0 + r < d) sq += (double)xn[r] * xn[r];
                }
                if (f0 + 3 < d && (d & 3) == 0) {
                    stg(reinterpret_cast<f4 *>(Xout + row * d + f0), f4{xn[0], xn[1], xn[2], xn[3]});
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (f0 + r < d) stg(Xout + row * d + f0 + r, xn[r]);
                }
            }
        }
        sq += __shfl_xor(sq, 16);
        sq += __shfl_xor(sq, 32);
        if (out_sqn && elq == 0 && row < nq) stg(out_sqn + row, (float)sq);
    }
}

// Column groups of the FP32 map per padded dimension: two at D <= 64, held
// to 128 VGPRs (4 waves per SIMD: two 8-wave workgroups per CU hold as many
// waves as four of 4 waves did); one at D = 128 and 256, whose 240-252
// VGPRs leave no room for the 512-thread launch bound.
constexpr int map_ks(int D) { return D <= 64 ? 2 : 1; }
constexpr int map_waves_per_simd(int D) { return D <= 64 ? 4 : 1; }

template <int D, int QB>
__global__ __launch_bounds__(256 * map_ks(D), map_waves_per_simd(D)) void entropic_map_f32(
    const float *Xq, int64_t nq, int d, const float *__restrict__ Y,
    const float *__restrict__ ysq, const float *__restrict__ g, int64_t m, float scale2,
    float bscale, float alpha, float *Xout, float *__restrict__ out_sqn) {
    __shared__ float vt[map_ks(D)][2][Tile<D>::FLOATS];
    __shared__ float bt[map_ks(D)][2][Tile<D>::BN];
    entropic_map_body<D, QB, map_ks(D)>(Xq, nq, d, Y, ysq, g, m, scale2, bscale, alpha, Xout, out_sqn,
                                        blockIdx.x, vt, bt);
}

// Grouped map: the (job, 64-query tile) items of many maps in one launch
// (the McCann steps and final maps of the serving form).
template <int D>
__global__ __launch_bounds__(256 * map_ks(D), map_waves_per_simd(D)) void entropic_map_f32_group(const MapJob *__restrict__ jobs,
                                                                         int njobs, int64_t total) {
    __shared__ float vt[map_ks(D)][2][Tile<D>::FLOATS];
    __shared__ float bt[map_ks(D)][2][Tile<D>::BN];
    int j = 0;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        while (j + 1 < njobs && jobs[j + 1].blk_begin <= item) ++j;
        const MapJob &J = jobs[j];
        entropic_map_body<D, 1, map_ks(D)>(J.Xq, J.nq, J.d, J.Y, J.ysq, J.g, J.m, J.scale2, J.bscale, J.alpha,
                                J.Xout, J.out_sqn, item - J.blk_begin, vt, bt);
        __syncthreads();
    }
}

// Workgroups of `kernel` the chip holds at once (the grid of a persistent
// launch), for the current device; computed once per kernel.
template <typename K>
int64_t resident_blocks(K kernel, int threads = 256) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        cus < 1 || per_cu < 1)
        return 1024;   // a safe default; any grid size gives the same results
    return (int64_t)cus * per_cu;
}

template <int D, int QB>
hipError_t lse_launch_t(const LseJob &j, hipStream_t s) {
    // the plan must cover every row tile of this kernel variant
    if (j.blocks != (j.nu + 64 * QB - 1) / (64 * QB) * j.S) return hipErrorInvalidValue;
    timed_launch(0, lse_partial_f32<D, QB>, dim3((unsigned)j.blocks), dim3(256), 0, s, j);
    return hipGetLastError();
}

// Grid of a persistent launch: the workgroups the chip holds at once, or
// fewer when the list is short.
inline unsigned group_grid(int64_t total, int64_t cap) { return (unsigned)std::min(total, cap); }

template <int D, int QB>
hipError_t lse_group_launch_t(const LseJob *jobs_dev, int njobs, int64_t total, hipStream_t s) {
    static const int64_t cap = resident_blocks(lse_partial_f32_group<D, QB>);
    timed_launch(0, lse_partial_f32_group<D, QB>, dim3(group_grid(total, cap)), dim3(256), 0, s, jobs_dev,
                 njobs, total);
    return hipGetLastError();
}

template <int D>
hipError_t map_group_launch_t(const MapJob *jobs_dev, int njobs, int64_t total, hipStream_t s) {
    static const int64_t cap = resident_blocks(entropic_map_f32_group<D>, 256 * map_ks(D));
    timed_launch(1, entropic_map_f32_group<D>, dim3(group_grid(total, cap)), dim3(256 * map_ks(D)), 0, s, jobs_dev,
                 njobs, total);
    return hipGetLastError();
}

template <int D, int QB>
hipError_t map_launch_t(const MapArgs &a, float scale2, float bscale, hipStream_t s) {
    const int64_t tiles = (a.nq + 64 * QB - 1) / (64 * QB);
    timed_launch(1, entropic_map_f32<D, QB>, dim3((unsigned)tiles), dim3(256 * map_ks(D)), 0, s, a.Xq, a.nq, a.d,
                 a.Y, a.ysq, a.g, a.m, scale2, bscale, a.alpha, a.Xout, a.out_sqn);
    return hipGetLastError();
}

int padded_dim(int d) {
    if (d <= 16) return 16;
    if (d <= 32) return 32;
    if (d <= 64) return 64;
    if (d <= 128) return 128;
    return 256;
}

// Row blocks per wave of the potential kernel: four for D <= 64 (each column
// fragment read from LDS feeds four MFMA chains; measured 5 % faster on the
// benchmark workload than two, at two waves per SIMD instead of three, and
// 13 % faster than three, at two waves per SIMD or, with the registers
// capped, three).
constexpr int lse_qb(int D) { return D <= 64 ? 4 : (D >= 256 ? 1 : 2); }

}  // namespace

int lse_rows_per_block(int d) { return 64 * lse_qb(padded_dim(d)); }

int padded_dim_f32(int d) { return padded_dim(d); }

// Workgroups per potential update.  The chip holds ~512-1024 of the BF16
// workgroups at once; with ~8 rounds the last, partly filled round costs
// little (measured: 1024 -> 8192 made the BF16 update 26% faster at
// n = 65536, d = 128, and changed nothing where the grid was already
// large).  The FP32 kernel measured the same at both, so it keeps the
// smaller merge.
constexpr int64_t kSplitTargetBf16 = 8192;
constexpr int64_t kSplitTargetF32 = 1024;

void plan_lse_job(LseJob &j) {
    const int rows = j.precision == 0 ? lse_rows_per_block(j.d) : lse_bf16_rows_per_block(j.d, j.precision);
    const int64_t tiles = (j.nu + rows - 1) / rows;
    // Split the columns so that the grid holds >= target workgroups,
    // keeping >= one LDS column tile per split in FP32 (64 columns; small
    // problems such as the 1024-point grid solves of the eps-scheduler need
    // the splits to fill the chip) and >= 256 columns in BF16.  S is a power
    // of two, so from S = 4 on (with an even number of row tiles) the FP32
    // kernel can hand each XCD half of the row tiles and a quarter of the
    // splits, and from S = 8 on the BF16 blocks an XCD receives (block b goes
    // to XCD b mod 8, split b mod S) stream a fixed subset of the column
    // splits through that XCD's L2.
    const int64_t target = j.precision == 0 ? kSplitTargetF32 : kSplitTargetBf16;
    int64_t S = tiles >= target ? 1 : (target + tiles - 1) / tiles;
    const int64_t min_cols = j.precision == 0 ? 64 : 256;
    const int64_t max_by_cols = (j.nv + min_cols - 1) / min_cols;
    if (S > max_by_cols) S = max_by_cols;
    if (S > 1) {
        int64_t q = 1;
        while (q < S) q <<= 1;
        S = q;
        if (S > max_by_cols) S = max_by_cols;
    }
    // the split partials hold kMaxSplit x max(n, m) floats: up to
    // kMaxSplit max(nu, nv) / nu splits of nu rows (a flat cap of kMaxSplit
    // left the update of a pair with nu << nv a fraction of the chip)
    const int64_t cap = kMaxSplit * std::max(j.nu, j.nv) / std::max<int64_t>(j.nu, 1);
    if (S > cap) S = cap;
    if (S < 1) S = 1;
    j.S = (int)S;
    j.cps = (j.nv + S - 1) / S;
    // BF16 splits start on the 64-row boundaries of the padded column copy
    if (j.precision != 0) j.cps = (j.cps + 63) / 64 * 64;
    j.scale2 = 2.f * kLog2e / j.eps;
    j.bscale = kLog2e / j.eps;
    j.blocks = tiles * S;
    j.mblocks = (j.nu + 255) / 256;
}

hipError_t launch_lse_update(const LseArgs &a, hipStream_t s, int *n_err_part) {
    if (a.esum_out && !lse_update_folds_sum(a)) return hipErrorInvalidValue;
    LseJob j = a;
    if (j.cost_p != 0.f) plan_pcost_job(j);
    else plan_lse_job(j);
    hipError_t e;
    if (j.cost_p != 0.f) {
        e = launch_pcost_partial(j, s);
    } else if (j.precision != 0) {
        e = launch_lse_partial_bf16(j, s);
    } else switch (padded_dim(j.d)) {
        case 16: e = lse_launch_t<16, lse_qb(16)>(j, s); break;
        case 32: e = lse_launch_t<32, lse_qb(32)>(j, s); break;
        case 64: e = lse_launch_t<64, lse_qb(64)>(j, s); break;
        case 128: e = lse_launch_t<128, lse_qb(128)>(j, s); break;
        default: e = lse_launch_t<256, lse_qb(256)>(j, s); break;
    }
    if (e != hipSuccess) return e;
    if (j.cost_p != 0.f) {
        if (!pcost_fused(j) && (e = launch_pcost_merge(j, s)) != hipSuccess) return e;
        if (n_err_part) *n_err_part = j.pot_old ? (int)j.mblocks : 0;
        return hipGetLastError();
    }
    hipLaunchKernelGGL(lse_merge, dim3((unsigned)j.mblocks), dim3(256), 0, s, j);
    if (n_err_part) *n_err_part = j.pot_old ? (int)j.mblocks : 0;
    return hipGetLastError();
}

hipError_t plan_lse_update_group(LseJob *jobs, int njobs, GroupPlan *gp) {
    if (njobs <= 0) return hipErrorInvalidValue;
    int64_t blk = 0, mblk = 0;
    int nerr = 0;
    const int D = padded_dim(jobs[0].d);
    for (int k = 0; k < njobs; ++k) {
        if (jobs[k].cost_p != 0.f || jobs[k].esum_out) return hipErrorInvalidValue;
        plan_lse_job(jobs[k]);
        if (jobs[k].precision != 0 || padded_dim(jobs[k].d) != D) return hipErrorInvalidValue;
    }
    // largest items first (an item is a row tile times cps columns): every
    // workgroup's share of the static walk starts with the long items and
    // the walk ends on short ones
    std::stable_sort(jobs, jobs + njobs, [](const LseJob &a, const LseJob &b) { return a.cps > b.cps; });
    for (int k = 0; k < njobs; ++k) {
        blk = (blk + 7) / 8 * 8;   // jobs start on multiples of 8 (XCD affinity of the splits)
        jobs[k].blk_begin = blk;
        jobs[k].mblk_begin = mblk;
        blk += jobs[k].blocks;
        mblk += jobs[k].mblocks;
        if (jobs[k].pot_old) ++nerr;
    }
    *gp = GroupPlan{blk, mblk, nerr, D};
    return hipSuccess;
}

hipError_t enqueue_lse_update_group(const LseJob *jobs_dev, int njobs, const GroupPlan &gp,
                                    float *err_out, hipStream_t s) {
    hipError_t e;
    switch (gp.D) {
        case 16: e = lse_group_launch_t<16, lse_qb(16)>(jobs_dev, njobs, gp.blocks, s); break;
        case 32: e = lse_group_launch_t<32, lse_qb(32)>(jobs_dev, njobs, gp.blocks, s); break;
        case 64: e = lse_group_launch_t<64, lse_qb(64)>(jobs_dev, njobs, gp.blocks, s); break;
        case 128: e = lse_group_launch_t<128, lse_qb(128)>(jobs_dev, njobs, gp.blocks, s); break;
        default: e = lse_group_launch_t<256, lse_qb(256)>(jobs_dev, njobs, gp.blocks, s); break;
    }
    if (e != hipSuccess) return e;
    static const int64_t mcap = resident_blocks(lse_merge_group);
    hipLaunchKernelGGL(lse_merge_group, dim3(group_grid(gp.mblocks, mcap)), dim3(256), 0, s, jobs_dev, njobs,
                       gp.mblocks);
    if (gp.nerr > 0)
        hipLaunchKernelGGL(sum_group, dim3(gp.nerr), dim3(256), 0, s, jobs_dev, njobs, err_out);
    return hipGetLastError();
}

MapJob map_job(const MapArgs &a) {
    MapJob j{};
    j.Xq = a.Xq; j.nq = a.nq; j.Y = a.Y; j.m = a.m; j.ysq = a.ysq; j.g = a.g;
    j.scale2 = 2.f * kLog2e / a.eps;   // as launch_entropic_map
    j.bscale = kLog2e / a.eps;
    j.alpha = a.alpha; j.d = a.d; j.Xout = a.Xout; j.out_sqn = a.out_sqn;
    return j;
}

hipError_t plan_map_group(MapJob *jobs, int njobs, MapGroupPlan *gp) {
    if (njobs <= 0) return hipErrorInvalidValue;
    const int D = padded_dim(jobs[0].d);
    for (int k = 0; k < njobs; ++k)
        if (padded_dim(jobs[k].d) != D || jobs[k].nq < 1) return hipErrorInvalidValue;
    // largest items (most targets) first, as for the potential updates
    std::stable_sort(jobs, jobs + njobs, [](const MapJob &a, const MapJob &b) { return a.m > b.m; });
    int64_t blk = 0;
    for (int k = 0; k < njobs; ++k) {
        jobs[k].blk_begin = blk;
        blk += (jobs[k].nq + 63) / 64;   // 64 queries per workgroup (one 16-row block per wave)
    }
    *gp = MapGroupPlan{blk, D};
    return hipSuccess;
}

hipError_t enqueue_map_group(const MapJob *jobs_dev, int njobs, const MapGroupPlan &gp, hipStream_t s) {
    switch (gp.D) {
        case 16: return map_group_launch_t<16>(jobs_dev, njobs, gp.blocks, s);
        case 32: return map_group_launch_t<32>(jobs_dev, njobs, gp.blocks, s);
        case 64: return map_group_launch_t<64>(jobs_dev, njobs, gp.blocks, s);
        case 128: return map_group_launch_t<128>(jobs_dev, njobs, gp.blocks, s);
        default: return map_group_launch_t<256>(jobs_dev, njobs, gp.blocks, s);
    }
}

hipError_t launch_sum_f32(const float *part, int n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(sum_f32, dim3(1), dim3(256), 0, s, part, n, out);
    return hipGetLastError();
}

// Workgroups of the moments pass: >= 64 rows each, at most 256 (the fold
// reads nblk x (d + 1) partials in one workgroup).
int cloud_stat_blocks(int64_t n) {
    const int64_t b = (n + 63) / 64;
    return (int)(b < 256 ? (b < 1 ? 1 : b) : 256);
}

hipError_t launch_cloud_prep(const float *X, int64_t n, int d, float *sqn, void *lp,
                             double *stats_part, int nblk, hipStream_t s, bool norms_ready) {
    if (!norms_ready)
        hipLaunchKernelGGL(cloud_norms, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, n, d, sqn);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && lp) e = launch_bf16_rows(X, n, d, lp, s);
    if (e != hipSuccess || !stats_part) return e;
    const int64_t rpb = (n + nblk - 1) / nblk;
    hipLaunchKernelGGL(cloud_stats, dim3(nblk), dim3(256), 0, s, X, n, d, sqn, rpb, stats_part);
    if (nblk > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(stats_fold, dim3(d + 1), dim3(256), 0, s, stats_part, nblk, d);
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
    hipError_t e;
    if (a.precision != 0) {
        e = launch_map_bf16(a, scale2, bscale, s);
    } else switch (padded_dim(a.d)) {
        // one 16-row block per wave at every width: two (at D <= 64, and
        // at D = 128 with 164 AGPRs spilled over) measured 32-35 % slower at
        // D = 16, 32, 64 and 3.5 % at D = 128, for the lower occupancy
        case 16: e = map_launch_t<16, 1>(a, scale2, bscale, s); break;
        case 32: e = map_launch_t<32, 1>(a, scale2, bscale, s); break;
        case 64: e = map_launch_t<64, 1>(a, scale2, bscale, s); break;
        case 128: e = map_launch_t<128, 1>(a, scale2, bscale, s); break;
        default: e = map_launch_t<256, 1>(a, scale2, bscale, s); break;
    }
    return e;
}

}  // namespace pot
