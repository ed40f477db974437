// Internal interface between the C ABI driver and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace pot {

// Rows handled by one workgroup of the log-sum-exp kernel and the map kernel.
int lse_rows_per_block(int d);
int map_rows_per_block(int d);
constexpr int kMaxSplit = 32;       // column splits of the log-sum-exp kernel
constexpr int kReduceBlock = 256;   // threads of the per-row kernels

// Arguments of one potential update (the f-update or the g-update of Alg. 1):
//   out_i = eps*logw_i + usq_i - eps*ln2*log2 sum_j 2^(scale2*<u_i,v_j> + beta_j)
//   beta_j = (gamma*vpot_j - vsq_j) * log2(e)/eps,  scale2 = 2*log2(e)/eps.
struct LseArgs {
    const float *U;        // rows (nu x d)
    const void *U_lp;      // BF16 copy of U (BF16 form)
    int64_t nu;
    const float *usq;      // |u_i|^2
    const float *logw;     // log weights of the rows
    const float *V;        // columns (nv x d)
    const void *V_lp;
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
};

// Enqueue one potential update (partials + merge).  Returns the number of
// error partials written to err_part (0 if pot_old is NULL).
hipError_t launch_lse_update(const LseArgs &a, hipStream_t s, int *n_err_part);

// Deterministic sum of n float partials into *out (device).
hipError_t launch_sum_f32(const float *part, int n, float *out, hipStream_t s);

// Per-point squared norms in FP64 (rounded to FP32), optional BF16 copy, and
// FP64 partial sums of (sum_i x_i, sum_i |x_i|^2) into stats (nblk x (d+1)).
hipError_t launch_cloud_prep(const float *X, int64_t n, int d, float *sqn, void *lp,
                             double *stats_part, int nblk, hipStream_t s);
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
    float *Xout;           // may alias Xq
    float *out_sqn;        // |Xout_i|^2 (nullable)
    void *out_lp;          // BF16 copy of Xout (nullable)
};
hipError_t launch_entropic_map(const MapArgs &a, hipStream_t s);

// FP64 check: row sums and column sums of P in FP64, reduced to
// part[0..3*nb) per-block partials of (|r_i - a_i|, r_i, f_i a_i) and
// (|c_j - b_j|, c_j, g_j b_j).  Weights a, b: caller arrays or NULL (uniform,
// 1/n in FP64).
hipError_t launch_fp64_check(const float *X, int64_t n, const float *Y, int64_t m, int d,
                             const float *f, const float *g, const float *a,
                             const float *b, float eps, double *part_rows,
                             double *part_cols, hipStream_t s);
int fp64_check_blocks(int64_t n);

// Launch timing (see pot_timing_enable): kind 0 = cost + log-sum-exp
// partial kernel, kind 1 = entropic-map kernel.  timing_begin returns an
// opaque slot (or -1 when timing is off); timing_end closes it.
int64_t timing_begin(int kind, hipStream_t s);
void timing_end(int64_t slot, hipStream_t s);

}  // namespace pot
