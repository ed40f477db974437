// Internal interface between the C ABI driver and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstddef>
#include <cstdint>

namespace pot {

// Rows handled by one workgroup of the log-sum-exp kernel.
int lse_rows_per_block(int d);
constexpr int kMaxSplit = 32;       // column splits of the log-sum-exp kernel
constexpr int kReduceBlock = 256;   // threads of the per-row kernels

// One potential update (the f-update or the g-update of Alg. 1) of one
// problem, as the kernels see it:
//   out_i = eps*logw_i + usq_i - eps*ln2*log2 sum_j 2^(scale2*<u_i,v_j> + beta_j)
//   beta_j = (gamma*vpot_j - vsq_j) * log2(e)/eps,  scale2 = 2*log2(e)/eps.
// The columns are split S ways (cps columns each); the partial kernel writes
// per-split (max, sum) partials, the merge kernel the potential and, when
// pot_old is set, the per-block row-marginal error partials.
struct LseJob {
    const float *U;        // rows (nu x d)
    const void *U_lp;      // BF16 [hi | lo] copy of U (BF16 forms; unused by the kernels,
                           // which split the scaled FP32 rows themselves)
    int64_t nu;
    const float *usq;      // |u_i|^2
    const float *logw;     // log weights of the rows
    const float *V;        // columns (nv x d)
    const void *V_lp;      // BF16 [hi | lo] copy of V, bf16_mpad(nv) rows per part
    int64_t nv;
    const float *vsq;      // |v_j|^2
    const float *vpot;     // potential of the columns (NULL = 0)
    float gamma;           // warm-start factor on vpot
    float eps;
    int d;
    int precision;
    const float *pot_old;  // previous potential of the rows (NULL: no error)
    float *pot_out;        // new potential (nu)
    float *part_m, *part_s;  // split partials (kMaxSplit x nu each)
    float *err_part;       // per-block error partials (ceil(nu/256))
    // filled by plan_lse_job
    int S;                 // column splits
    int64_t cps;           // columns per split
    float scale2, bscale;
    int64_t blocks;        // workgroups of the partial kernel
    int64_t mblocks;       // workgroups of the merge kernel
    // grouped launches: first workgroup of this job in the flattened grid
    int64_t blk_begin, mblk_begin;
    // serving: device control word of the problem's current Sinkhorn loop.
    // ctl[0] = 0 while running; the error sum of the f-update that carries
    // err(iter) sets ctl[0] = iter (and ctl[1] = err bits) once err <= tau or
    // iter == max_iter, and every later update of the job is skipped, so the
    // loop stops on the device at the same iterate as the host-checked loop.
    int *ctl;
    int iter;
    int max_iter;
    float tau;
    // general costs h = (1/p)|.|_p^p (cost_p = p; 0 for the squared-Euclidean
    // cost): usq is NULL.  With the pair's cost matrix (n x ldc, row-major,
    // rows = source points) the update reads C: the f-update reduces rows of
    // C (cmat_cols = 0), the g-update columns (cmat_cols = 1), and cps counts
    // columns (rows) of C per split.  Without it (cmat NULL) the update forms
    // h(u_i - v_j) on the fly from U and V.
    float cost_p;
    const float *cmat;
    int64_t ldc;
    int cmat_cols;
    // The previous f-update's error sum, folded into this update where
    // lse_update_folds_sum(job) holds (esum_out NULL: none): workgroup 0 adds
    // the esum_n partials at esum_in into *esum_out in the order of
    // launch_sum_f32, so the value is the same bits as the separate sum.
    const float *esum_in;
    int esum_n;
    float *esum_out;
    // An estimate of the rows' new potential, times shift_gamma (NULL: none):
    // the previous iterate's at the same eps and clouds, or at the first
    // iteration of a ProgOT step the warm start (1 - alpha_k) times the
    // previous step's.  The BF16 partial kernels take the log-sum-exp it
    // implies as a fixed exponent shift instead of a running maximum; a
    // workgroup whose sums leave the safe range redoes its split with the
    // running maximum, so the estimate decides speed, never the result's
    // validity.
    const float *shift_pot;
    float shift_gamma;
};

typedef LseJob LseArgs;

// Choose S, the scales and the workgroup counts of a job.  Depends only on
// the job's own sizes, so a problem computes the same bits alone, in a
// single-problem launch, or inside a grouped launch.
void plan_lse_job(LseJob &j);

// Enqueue one potential update (partials + merge).  Returns the number of
// error partials written to err_part (0 if pot_old is NULL).
hipError_t launch_lse_update(const LseArgs &a, hipStream_t s, int *n_err_part);

// Grouped potential updates: every job of a host array (FP32, all of one
// padded dimension) in one partial launch and one merge launch, both
// persistent kernels (a static walk of the jobs' work list), plus one
// error-sum launch for the jobs that
// carry pot_old.  plan_lse_update_group plans the host array in place --
// reordering it, largest items first, and filling the work-list offsets --
// and the totals; enqueue_lse_update_group launches on a device copy of that
// planned array (callers upload the tables of several updates in one copy).
// Error sums go to err_out[k] for the k-th job with pot_old in the planned
// order (err_out may be NULL when the jobs carry control words).
struct GroupPlan {
    int64_t blocks, mblocks;
    int nerr;
    int D;
};
hipError_t plan_lse_update_group(LseJob *jobs, int njobs, GroupPlan *gp);
hipError_t enqueue_lse_update_group(const LseJob *jobs_dev, int njobs, const GroupPlan &gp,
                                    float *err_out, hipStream_t s);
int padded_dim_f32(int d);

// Deterministic sum of n float partials into *out (device).
hipError_t launch_sum_f32(const float *part, int n, float *out, hipStream_t s);

// True when the update of `j` can carry the previous f-update's error sum
// (the general-cost column kernel on a kept cost matrix), saving the launch
// of launch_sum_f32.
bool lse_update_folds_sum(const LseJob &j);

// Per-point squared norms in FP64 (rounded to FP32; skipped when
// norms_ready: the entropic map that produced X wrote them), optional BF16
// hi/lo copies (lp != NULL), and FP64 partial sums of (sum_i x_i,
// sum_i |x_i|^2) into stats (nblk x (d+1)).
hipError_t launch_cloud_prep(const float *X, int64_t n, int d, float *sqn, void *lp,
                             double *stats_part, int nblk, hipStream_t s, bool norms_ready = false);
int cloud_stat_blocks(int64_t n);

// log of probability weights (w == NULL: uniform).
hipError_t launch_log_weights(const float *w, int64_t n, float *logw, hipStream_t s);

// out = gamma * in (n floats); in == NULL writes zeros.
hipError_t launch_scale(const float *in, float gamma, int64_t n, float *out, hipStream_t s);

struct MapArgs {
    const float *Xq;       // queries (nq x d)
    int64_t nq;
    const float *Y;        // targets (m x d)
    const void *Y_lp;
    int64_t m;
    const float *ysq;      // |y_j|^2
    const float *g;        // target potential
    float eps, alpha;
    int d, precision;
    const void *YT_lp;     // transposed BF16 copy of Y (BF16 forms)
    int64_t mp;            // bf16_mpad(m): rows of Y_lp per part, row stride of YT_lp
    const float *yt_unscale;  // plain BF16 form: 2^-k of the FP16 copy YT_lp = Y 2^k
    float *Xout;           // may alias Xq
    float *out_sqn;        // |Xout_i|^2 (nullable)
};
hipError_t launch_entropic_map(const MapArgs &a, hipStream_t s);

// Grouped FP32 maps (one launch for many maps of one padded dimension, each
// computing exactly what launch_entropic_map computes for it).  plan_map_group
// reorders the host array (largest first) and fills the work-list offsets;
// enqueue_map_group launches on a device copy of the planned array.
struct MapJob {
    const float *Xq;
    int64_t nq;
    const float *Y;
    int64_t m;
    const float *ysq, *g;
    float scale2, bscale, alpha;
    int d;
    float *Xout, *out_sqn;
    int64_t blk_begin;
};
struct MapGroupPlan {
    int64_t blocks;
    int D;
};
MapJob map_job(const MapArgs &a);   // FP32 args, squared-Euclidean cost
hipError_t plan_map_group(MapJob *jobs, int njobs, MapGroupPlan *gp);
hipError_t enqueue_map_group(const MapJob *jobs_dev, int njobs, const MapGroupPlan &gp,
                             hipStream_t s);

// General costs h(z) = (1/p) sum_k |z_k|^p (FP32 on the VALU).
int pcost_pad_dim(int d);                 // padded dimension of the map kernel
int64_t pcost_ldc(int64_t m);             // row stride of the cost matrix (m rounded up to 4)
int64_t pcost_matrix_blocks(int64_t n, int64_t m);
int pcost_map_max_split();
// C_ij = h(x_i - y_j) for all pairs into Cm (Cm NULL: not stored), and
// sum_ij C_ij (FP64) into *sum_out; part holds pcost_matrix_blocks(n, m)
// doubles.
hipError_t launch_pcost_matrix(const float *X, int64_t n, const float *Y, int64_t m, int d, float p,
                               float *Cm, int64_t ldc, double *part, double *sum_out,
                               hipStream_t s);
void plan_pcost_job(LseJob &j);
// The row update over the cost matrix with one split writes the potential
// and the error partials itself (no merge launch; mblocks error partials).
bool pcost_fused(const LseJob &j);
hipError_t launch_pcost_partial(const LseJob &j, hipStream_t s);   // planned job
hipError_t launch_pcost_merge(const LseJob &j, hipStream_t s);     // planned, not fused
// Xout_i = Xq_i - alpha grad h*(sum_j p_j grad h(Xq_i - y_j)),
// p_j = softmax_j((g_j - h(Xq_i - y_j))/eps).  With few queries the targets
// are split and the partials go to pm/ps (pcost_map_max_split() x cap_q
// floats each) and pacc (that many x pcost_pad_dim(d) floats); more than
// cap_q queries are processed in chunks.  Xout may alias Xq.
struct PcostMapArgs {
    const float *Xq;
    int64_t nq;
    const float *Y;
    int64_t m;
    const float *g;
    float eps, alpha, p;
    int d;
    float *Xout;
    float *pm, *ps, *pacc;
    int64_t cap_q;
};
hipError_t launch_pcost_map(const PcostMapArgs &a, hipStream_t s);
// FP64 check for the cost h: the same partials as launch_fp64_check, with
// C_ij = h(x_i - y_j) by FP64 direct differences.
hipError_t launch_fp64_check_pcost(const float *X, int64_t n, const float *Y, int64_t m, int d,
                                   float p, const float *f, const float *g, const float *a,
                                   const float *b, float eps, double *part_rows,
                                   double *part_cols, hipStream_t s);

// BF16 forms (precision 1: one BF16 product; 2: hi/lo split, three products).
int bf16_dim(int d);                 // padded dimension of the BF16 copies
int64_t bf16_mpad(int64_t m);        // padded row count of the BF16 copies (multiple of 128)
int lse_bf16_rows_per_block(int d, int precision);
hipError_t launch_lse_partial_bf16(const LseJob &a, hipStream_t s);  // planned job
hipError_t launch_map_bf16(const MapArgs &a, float scale2, float bscale, hipStream_t s);
// [hi | lo] BF16 copies of the rows of X (each bf16_mpad(n) x bf16_dim(d),
// zero padded, in the tile layout of the BF16 kernels).
hipError_t launch_bf16_rows(const float *X, int64_t n, int d, void *lp, hipStream_t s);
// [hi^T | lo^T] of Y, each bf16_dim(d) x bf16_mpad(m) in blocks of 32
// columns (permuted into the projection product's order, tile layout).
hipError_t launch_bf16_transpose(const float *Y, int64_t m, int d, void *yt, hipStream_t s);
// The plain BF16 form's projection copy: one FP16 part of the same layout
// holding Y 2^k (k from max |y|, so max |y| 2^k <= 2^14); scale2 is two
// floats of device scratch: [0] max |y| (bits), [1] receives 2^-k.
hipError_t launch_f16_transpose(const float *Y, int64_t m, int d, void *yt, float *scale2, hipStream_t s);

// FP64 check: FP64 norms of X and Y into xsq64/ysq64 (n and m doubles),
// then row sums and column sums of P in FP64 reduced to per-block partials
// part[0..kCheckParts*nb) of (sum |r_i - a_i|, sum r_i, sum f_i a_i,
// sum P_ij C_ij, sum P_ij log P_ij) and the same over columns (|c_j - b_j|,
// c_j, g_j b_j, ...).  Weights a, b: caller arrays or NULL (uniform, 1/n in
// FP64).
hipError_t launch_fp64_check(const float *X, int64_t n, const float *Y, int64_t m, int d,
                             const float *f, const float *g, const float *a,
                             const float *b, float eps, double *xsq64, double *ysq64,
                             double *part_rows, double *part_cols, hipStream_t s);
int fp64_check_blocks(int64_t n);
constexpr int kCheckParts = 5;
// FP64 per-block partials of sum_i v_i w_i (w NULL: uniform 1/n) into part
// (weighted_sum_blocks(n) <= 256 doubles).
int weighted_sum_blocks(int64_t n);
hipError_t launch_weighted_sum(const float *v, const float *w, int64_t n, double *part,
                               hipStream_t s);
// Diagonal of the coupling (n == m): per-block partials (sum P_ii,
// sum log P_ii), diag_blocks(n) blocks of 2 doubles; cost_p = 0 is the
// squared-Euclidean cost, cost_p > 1 the cost (1/p)|.|_p^p.
hipError_t launch_diag_sums(const float *X, const float *Y, int64_t n, int d, const float *f,
                            const float *g, float eps, float cost_p, double *part, hipStream_t s);
int diag_blocks(int64_t n);

// Launch timing (see pot_timing_enable): kind 0 = potential (cost +
// log-sum-exp) partial kernel, kind 1 = entropic-map kernel.  When timing is
// on, timed_launch hands a start and a stop event to the dispatch itself
// (hipExtLaunchKernelGGL), so each interval is the kernel's execution alone,
// without the gap to the previous command on the stream.
struct TimedEvents {
    hipEvent_t start, stop;
};
TimedEvents timing_events(int kind);          // both null when timing is off
void timing_commit(int kind, TimedEvents t);  // after the launch that records them

template <typename... KArgs, typename... Args>
void timed_launch(int kind, void (*kernel)(KArgs...), dim3 grid, dim3 block, uint32_t shmem,
                  hipStream_t s, Args... args) {
    const TimedEvents t = timing_events(kind);
    if (t.start) {
        hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, t.start, t.stop, 0, args...);
        timing_commit(kind, t);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
    }
}

}  // namespace pot
