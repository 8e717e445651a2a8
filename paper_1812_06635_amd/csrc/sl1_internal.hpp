// Internal device-side definitions shared by the stablel1 kernels and the host
// orchestration.  CDNA4 (gfx950): wave64, 256 threads per block.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/stablel1.h"

namespace sl1 {

constexpr int kBlock = 256;         // threads per block (4 waves)
constexpr int kWave = 64;
constexpr int kSeg = 256;           // atoms per segment of a compacted list (one update block)
constexpr int kFwdRows = 1024;      // rows per forward item: 4 sub-chunks of 256 (4 per lane), 2 waves each
constexpr int kFwdBlock = 512;      // forward block: 8 waves share the nonzeros of x
constexpr int kFwdFacLds = 48 * 1024;   // largest Kronecker factor set staged in the forward LDS
constexpr int kFwdFacNnz = 32;          // nonzeros from which a block stages the factors
constexpr int kFwdWaves = kFwdBlock / 64;
constexpr int kMaxSeg = 1024;       // segments of a compacted list (K <= 262144)
constexpr int kKronVLds = 96 * 1024; // largest V region (the item's intermediate) of a Kronecker tile shape
constexpr int kMaxN = 8192;
constexpr int kWgBlock = 512;       // whole-solve engine: one 8-wave workgroup per signal
constexpr int kWgWaves = kWgBlock / 64;
constexpr int kWgRows = 1024;       // rows per forward pass of that engine (16 per lane of a wave)
constexpr int kWgStage = 512;       // nonzeros of x staged in LDS per forward step
constexpr int kWgPhases = 4;        // profiled phases: forward, dense correlations, Kronecker correlations, update

enum Kind { kDense = 0, kKron = 1, kFaust = 2 };

// FAuST stage A~ = S_1 S_2 ... S_J (sparse factors, S_l of size dim[l-1] x dim[l],
// dim[0] = N, dim[J] = K): every factor in CSR and its transpose in CSR, the
// arrays of all factors concatenated (device).  Values in the stage's dtype
// (FP64 or FP32), products accumulated in FP64.
constexpr int kFaustMax = 8;          // factors
constexpr int kFaustMaxDim = 1024;    // N and every inner dimension
constexpr int kFaustAtoms = 64;       // atoms per correlation tile (one block: all its signals)
struct FaustDesc {
    int J;
    int dim[kFaustMax + 1];
    int maxd;                          // largest of dim[0 .. J-1]
    int q;                             // nonzeros of x per scatter chunk of the forward
    long long fp[kFaustMax], fz[kFaustMax];   // S_l: offsets of its row pointers / entries
    long long tp[kFaustMax], tz[kFaustMax];   // S_l^T: offsets of its row pointers / entries
    const int* ptr;
    const int* idx;
    const void* val;
    const int* tptr;
    const int* tidx;
    const void* tval;
};

struct StageDesc {
    int kind, dtype;
    int R, n1, k1, n2, k2;
    int kt2, kt1;             // Kronecker correlation item: kt2 x kt1 atoms (j2 x j1), multiples of 16
    int vec;                  // dense: elements per lane per load (4, 8 or 16)
    const void* A;            // dense storage
    const float* scale;       // dense per-column scale or nullptr
    const void* B;            // kron factors (device copies)
    const void* C;
    const double* eps;        // eps_j enlarged by the library's rounding bound
    const double* at_norm;    // ||a~_j||_2 (look-ahead estimate K_t)
    const FaustDesc* fa;      // FAuST factors (device) or nullptr
    int fa_items;             // FAuST: correlation tiles (kFaustAtoms atoms each)
    int fa_maxd;              // FAuST: largest of N and the inner dimensions
    int fa_dlast;             // FAuST: rows of the last factor (length of w = S_{J-1}^T ... S_1^T z)
    double L, invL, rc;
    double at_norm_max, eps_max;
    // norm q of the bounds eps (Lemma 1 with an l_q zone): qmode 0 for q = 2, 1 for
    // other finite q > 1, 2 for q = 1 (dual norm: max), 3 for q = inf (dual norm: sum);
    // qd the dual exponent q*, cq = N^((1/2 - 1/q)_+), the l2 constant of the bounds
    int qmode, qpad;
    double qd, cq;
};

// Iteration state C_t of one signal.  Double-buffered by iteration parity:
// the forward kernel of iteration t reads C_{t-1} from slot (t-1)%2, folds in
// the per-block results of iteration t-1 and (block 0 only) writes C_t to slot
// t%2; every later kernel of iteration t reads slot t%2.
struct Control {
    int stage, iter, done, status;
    int ksince, par, advance;         // advance: the next iteration folds this one's results
    int nslot;                        // correlation-partial slots of the iteration (4 per item)
    int n_act, n_nz, nseg_act, nseg_nz;
    double lam, tau, l1;              // lambda, FISTA momentum sequence, ||x_t||_1
    long long t0;
};

// FP64 quantities of iteration t (Section III-C, Theorem 1, Section IV-A),
// computed identically by every block of the update kernel; block 0 stores them.
struct Scalars {
    double r2, zz, yz;                // ||y - A~x||^2, ||z||^2, y^T z (z: stored residual direction)
    double mp, mt, E;                 // max(|g|+eps||z||), max|g|, max eps over A_t
    double sp, st;                    // theta' = s' z, theta~ = s~ z
    double P, Gp, Gt, delta, Rp, gamma;
    double c1, c2;                    // |s'| and |s'| ||z||
    double beta, tau_next;
    double Rd, ny;                    // stable Dynamic Safe radius ||theta' - y/lambda|| (bounded), ||y||
    double Rdl, dcut;                 // GAP dome: lower bound of that radius, normalised cut level
    int conv, pad0;                   // 1 converged on A, 2 iteration cap
    long long tconv;
};

// Outcome of a finished signal.
struct Final {
    double gap, gap_cert;
    int iters, stage, status, par;
    long long t0, tconv;
};

struct SolveParams {
    int n_stages, N, K, batch;
    int max_iter, trace_cap, y_f64, lambda_only;
    int ista, rule;           // update: 0 FISTA, 1 ISTA; test: 0 stable GAP Safe, 1 stable Dynamic Safe
    int screen_every;         // rejections only at iterations t with t % screen_every == 0
    double Gamma, tol, margin;
    StageDesc st[SL1_MAX_STAGES];
    const double* atom_norm;
    const void* y;            // batch x N, FP32 or FP64 (y_f64)
    const double* lam;        // batch
    const double* cy;         // stable Dynamic Safe: [batch][K] a_j^T y with the exact dictionary
    const double* yy;         // [batch] ||y||^2 (FP64)
    double* trace;
    // workspace (per signal b)
    Control* ctrl;            // [batch][2]
    Scalars* sc;              // [batch]
    Final* fin;               // [batch]
    double* x;                // [batch][2][K]
    double* g;                // [batch][2][K]
    uint8_t* mask;            // [batch][K]
    int* act;                 // [batch][2][K]
    int* nz;                  // [batch][2][K]
    double* nzx;              // [batch][2][K] values of the nonzero list (same positions)
    int* act_pre;             // [batch][2][nseg_max+1]
    int* nz_pre;              // [batch][2][nseg_max+1]
    double* z;                // [batch][N]
    double* res_part;         // [batch][nrc][3]
    double* zq;               // [batch] ||z||_{q*} of the iteration (stages with l_q bounds)
    double* adj_part;         // [batch][nadj_max][4 waves][3] per-wave maxima of the correlation items
    double* upd_part;         // [batch][nseg_max][4]
    int* cnt_fwd;             // [2][batch] work items of the forward launch of the iteration with parity s
    int* cnt_adj;             // [batch] work items of the dense correlation launch (current iteration)
    int* cnt_adjk;            // [batch] work items of the Kronecker correlation launch
    int* cnt_upd;             // [batch] work items of the update launch (current iteration)
    int* cnt_gemm;            // [batch] 1: the signal's correlations go through the batched product
    int* cnt_adjf;            // [batch] stage + 1 while the signal's correlations are a FAuST stage's (0: not)
    double* fw;               // [batch][kFaustMaxDim] FAuST stages: w = S_{J-1}^T ... S_1^T z of the iteration
    double* gemm_part;        // [kGemmSplitUnits][64 * 64] partial tiles of a split product launch
    int gemm_min;             // |A_t| from which a signal on the exact dense stage qualifies (0: never)
    int gemm_on;              // the batched product runs (set by the host between chunks)
    int* active_signals;      // [0] signals not yet done; [8] signals that reached the park stage
                              // in the whole-solve kernel during the current solve
    int* sig_stat;            // [batch][4] per live signal, written by each forward launch (zero
                              // once done): |A_t|, |A_t|, not yet on the last stage, qualifies
                              // for the batched correlation product
    int* stat;                // [4] reduction of sig_stat after a chunk: max and sum of |A_t|,
                              // count of signals not on the last stage, count that qualify
    int nseg_max, nrc, nadj_max, n1_max;
    int fwd_fac_lds;          // bytes of the forward kernel's LDS region for a Kronecker stage's
                              // factors (0: none); a stage whose factors fit is staged there
                              // for signals with many nonzeros
    // whole-solve engine: byte offsets of its dynamic LDS regions (-1: absent):
    // z in FP64 and FP32, y, the current stage's Kronecker factors, the scratch
    // (staging, cross-wave sums, Kronecker intermediate), the nonzero list (index
    // and value) and the preserved list, with the two list capacities (entries);
    // the tail kernel's per-position state of the preserved set (8 FP64 arrays
    // and one int array of wg_cap_act entries) and its Gram region (G, c and the
    // atom of each row, wg_cap_gram rows; 0: columns only); optional per-signal
    // phase clocks [batch][kWgPhases] (wall-clock ticks)
    int wo_zd, wo_zf, wo_y, wo_fac, wo_scr, wo_lnj, wo_lnx, wo_lact, wo_tail, wo_gram;
    int wg_cap_nz, wg_cap_act, wg_cap_gram;
    long long* wg_prof;
    // whole-solve kernel: a signal whose stage reaches wg_park stops at the top of
    // that iteration and keeps its state for another engine (-1: never); once at
    // most wg_park_allow live signals are still short of it (0: never), those stop
    // as well
    int wg_park;
    int wg_park_allow;
    int wg_absent_only;       // whole-solve launch for the signals marked absent only
    // [batch] 1 while the signal's iterations run in a whole-solve launch beside the
    // grid kernels, which then leave its state alone
    int* absent;
};

struct LaunchCfg {
    int batch, nseg_max, nrc, nadj_max;
    int g_fwd, g_adj, g_adjk, g_upd, g_gemm;  // persistent grid sizes (blocks; 0: launch skipped)
    int g_lq;                                  // l_q dual norms: batch, or 0 when every stage has q = 2
    int dome;                                  // the update kernel of the dome rule
    int step;                                  // per-signal step launches instead of forward + update
    int adjf_x, adjf_y, adjf_z;                // FAuST correlations: tiles x signal groups x stages (0: none)
    size_t lds_fwd, lds_adj, lds_adjk, lds_upd, lds_gemm, lds_step, lds_adjf;
};

// grid kernels (profile order): forward, dense correlations, Kronecker correlations,
// update, batched correlations, their finishing pass, per-signal step; launch order
// within an iteration (the step, or the forward, first; the update last)
constexpr int kGridKernels = 7;
constexpr int kIterOrder[kGridKernels] = {6, 0, 1, 4, 5, 2, 3};

// batched correlation tiles: 64 atoms x 64 signals per block
constexpr int kGemmAtoms = 64;
constexpr int kGemmSig = 64;
constexpr int kGemmMaxSplit = 8;     // row splits of one product tile
constexpr int kGemmSplitUnits = 512; // partial tiles of one split launch at most
#ifndef SL1_GEMM_MIN_SIGNALS
#define SL1_GEMM_MIN_SIGNALS 64
#endif
constexpr int kGemmMinSignals = SL1_GEMM_MIN_SIGNALS;   // fewer qualifying signals: streaming is faster

constexpr int kMaxBatch = 4096;     // per-launch work map lives in LDS

// FAuST correlations: signals per block (their w vectors in LDS, rows padded to dl + 1
// doubles, at most 96 KB) and the block's LDS bytes (the vectors, the signal list, and
// each signal's iterate parity and ||z||)
__host__ __device__ inline int faust_group(int dl) {
    const int sg = (64 * 1024) / ((dl + 1) * 8);
    return sg < 1 ? 1 : (sg > 64 ? 64 : sg);
}
// + per wave 4 atoms x 64 staged entries (index and value)
constexpr int kFaustStage = 4 * 64 * 12;
__host__ __device__ inline size_t faust_lds_bytes(int dl, int sg, int batch) {
    return (size_t)sg * (size_t)(dl + 1) * 8 + (((size_t)batch + 1) * 4 + 15) / 16 * 16 + (size_t)64 * 16 +
           (size_t)4 * kFaustStage;
}

// atoms per wave of the streaming correlation kernel: 4, 3, 2 or 1 by the stored size
// of a column (4 atoms of up to 3 KB, 3 of up to 4 KB, 2 of up to 6 KB, else 1)
__host__ __device__ __forceinline__ int dense_apw(int N, int dtype) {
    const int es = dtype == SL1_F64 ? 8 : (dtype == SL1_F32 ? 4 : (dtype == SL1_BF16 ? 2 : 1));
    const int cb = N * es;
    return cb <= 3072 ? 4 : (cb <= 4096 ? 3 : (cb <= 6144 ? 2 : 1));
}


// Rejections that zero a nonzero coefficient of x_t are counted in the same FP64
// sum as the look-ahead count K_t, scaled by 2^20 > K (the two stay separable):
// after such a rejection the FISTA momentum restarts, because the gradient at the
// extrapolated point is formed by linearity from g_t, which was taken at x_t before
// the zeroing.
constexpr double kRejNz = 1048576.0;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// bfloat16 bits -> float (exact)
__device__ __forceinline__ float bf16_to_f(uint16_t b) {
    return __uint_as_float(((uint32_t)b) << 16);
}

// Index i of a segmented compacted list: pre[] (in LDS) holds nseg+1 prefix counts.
__device__ __forceinline__ int seg_find(const int* pre, int nseg, int i) {
    int lo = 0, hi = nseg;   // invariant pre[lo] <= i < pre[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pre[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int list_pos(const int* pre, int nseg, int i) {
    const int s = seg_find(pre, nseg, i);
    return s * kSeg + (i - pre[s]);
}

__device__ __forceinline__ int list_get(const int* idx, const int* pre, int nseg, int i) {
    return idx[list_pos(pre, nseg, i)];
}

}  // namespace sl1
