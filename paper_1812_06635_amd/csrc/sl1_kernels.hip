// Per-iteration kernels of the stable-screening FISTA solver (gfx950).
//
// One iteration t of Algorithm 1 (FastL1) for every live signal of a batch is
// three steps, each a persistent launch over a work list of (signal, item) pairs:
//   k_fwd        forward product u = A~ x_t as a gather over the nonzeros of x_t,
//                residual rho = y - u and its norms (FP64), stored direction z;
//                also folds the previous iteration's partials into C_t
//                (Algorithm 2, momentum, list prefixes).
//   k_adj_dense  correlations g = A~^T z over the preserved set A_t on dense
//   k_adj_kron   stages (each wavefront streams a few atoms) or Kronecker stages
//                (MFMA tiles of sum_r C_r^T P B_r), and per-wave maxima of the
//                stable dual scaling.
//   k_upd        FP64 scalar block (dual points, gaps, delta, stable GAP radius,
//                gap ratio, stop decision), per-atom stable GAP test, look-ahead
//                count, FISTA step with soft thresholding, compaction of the
//                preserved set and of the nonzeros (wavefront ballot + prefix).
// No block communicates with another block of the same launch: every block
// writes its partial results, and the consumers in the NEXT launch reduce them
// in a fixed order (deterministic; the kernel boundary makes them visible
// across the chip's XCDs without any in-kernel cache write-back).  Quantities
// needed by every block of a launch (the FP64 scalar block, the prefix counts
// of the compacted lists, the switching decision) are recomputed identically by
// each block; one designated block stores them.  No block ever waits for
// another, so no launch can hang.
#include <algorithm>

#include "sl1_device.hpp"

namespace sl1 {

// ---------------------------------------------------------------------------
// work map: every launch covers the flattened list of (signal, item) pairs
// of the live signals; the per-signal item counts were written by the previous
// launch.  Each block scans the counts in LDS and takes a contiguous range of
// the list, so no block is launched without work.
// ---------------------------------------------------------------------------
__device__ int build_work_map(const int* cnt, int batch, int* s_pre, int* s_tmp) {
    int run = 0;
    for (int base = 0; base < batch; base += blockDim.x) {
        const int b = base + threadIdx.x;
        const int v = b < batch ? cnt[b] : 0;
        int ex;
        const int tot = block_excl_scan(v, ex, s_tmp);
        if (b < batch) s_pre[b] = run + ex;
        run += tot;
    }
    if (threadIdx.x == 0) s_pre[batch] = run;
    __syncthreads();
    return run;
}

__device__ __forceinline__ int find_signal(const int* s_pre, int batch, int g) {
    int lo = 0, hi = batch;      // s_pre[lo] <= g < s_pre[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_pre[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// initialisation: x_0 = 0, A_0 = {1..K}, stage 0 (Algorithm 1, Initialize).
// C_0 goes to both control slots with advance = 0, so the forward launch of
// iteration 0 (slot 0) takes it as is.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_init(const SolveParams* __restrict__ P) {
    const int b = blockIdx.y, c = blockIdx.x, K = P->K;
    const int j = c * kSeg + threadIdx.x;
    if (j < K) {
        xbuf(P, b, 0)[j] = 0.0;
        xbuf(P, b, 1)[j] = 0.0;
        gbuf(P, b, 0)[j] = 0.0;
        gbuf(P, b, 1)[j] = 0.0;
        P->mask[(size_t)b * K + j] = 1;
        actbuf(P, b, 0)[j] = j;
    }
    if (c != 0) return;
    const int nseg = (K + kSeg - 1) / kSeg;
    int* ap = actpre(P, b, 0);
    for (int s = threadIdx.x; s <= nseg; s += kBlock) ap[s] = min(s * kSeg, K);
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    int bad = 0;
    for (int i = threadIdx.x; i < P->N; i += kBlock) bad |= !isfinite(yval(P, b, i));
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double lam = P->lam ? P->lam[b] : 1.0;
        const bool ok = !s_bad && lam > 0.0 && isfinite(lam);
        Control C;
        C.stage = 0;
        C.iter = 0;
        C.done = ok ? 0 : 1;
        C.status = ok ? SL1_OK : SL1_EINVAL;
        C.ksince = 0;
        C.par = 0;
        C.advance = 0;
        C.nslot = 0;
        C.n_act = K;
        C.n_nz = 0;
        C.nseg_act = nseg;
        C.nseg_nz = 0;
        C.lam = lam;
        C.tau = 1.0;
        C.l1 = 0.0;
        C.t0 = wall_clock64();
        P->ctrl[2 * b + 0] = C;
        P->ctrl[2 * b + 1] = C;
        P->absent[b] = 0;
        nzpre(P, b, 0)[0] = 0;
        Final F;
        F.gap = 0.0;
        F.gap_cert = 0.0;
        F.iters = 0;
        F.stage = 0;
        F.status = C.status;
        F.par = 0;
        F.t0 = C.t0;
        F.tconv = 0;
        P->fin[b] = F;
        P->cnt_fwd[b] = ok ? P->nrc : 0;                 // slot 0
        P->cnt_fwd[P->batch + b] = 0;                    // slot 1
        P->cnt_adj[b] = 0;
        P->cnt_adjk[b] = 0;
        P->cnt_adjf[b] = 0;
        P->cnt_upd[b] = 0;
        P->cnt_gemm[b] = 0;
        for (int k = 0; k < 4; ++k) P->sig_stat[4 * b + k] = 0;
        if (ok) atomicAdd(P->active_signals, 1);
        if (b == 0) {
            for (int k = 0; k < 4; ++k) P->stat[k] = 0;
        }
    }
}

__device__ __forceinline__ int adj_items(const StageDesc& st, int n_act, int N) {
    if (st.kind == kDense) {
        const int per = 4 * dense_apw(N, st.dtype);
        return max(1, (n_act + per - 1) / per);
    }
    if (st.kind == kFaust) return st.fa_items;
    return (st.k2 / st.kt2) * (st.k1 / st.kt1);
}

// C_t from C_{t-1}, the scalars of iteration t-1 and the update launch's
// per-block partials; also the prefix counts of the two new compacted lists
// (into LDS).  Identical in every block; returns 1 when the signal finished.
// Sp and up0 were fetched together with C_{t-1}: the signal's scalars and this
// thread's first update partial (valid for threadIdx.x < min(nseg_max, blockDim)).
__device__ int advance_control(const SolveParams* P, int b, const Control& Cp, const Scalars& Sp,
                               const double (&up0)[4], Control& C, int* s_apre, int* s_zpre, double* s_red,
                               int* s_tmp, Scalars& S, double& kt_out) {
    C = Cp;
    if (!Cp.advance) return 0;
    S = Sp;
    if (S.conv) return 1;
    const int nblk = max(1, (Cp.n_act + kSeg - 1) / kSeg);
    int ak_tot = 0, az_tot = 0;
    double kt = 0.0, l1 = 0.0;
    for (int base = 0; base < nblk; base += blockDim.x) {
        const int k = base + threadIdx.x;
        int ck = 0, cz = 0;
        double a = 0.0, d = 0.0;
        if (k < nblk) {
            if (base == 0) {
                ck = (int)up0[0];
                cz = (int)up0[1];
                a = up0[2];
                d = up0[3];
            } else {
                const double* up = P->upd_part + ((size_t)b * P->nseg_max + k) * 4;
                ck = (int)up[0];
                cz = (int)up[1];
                a = up[2];
                d = up[3];
            }
        }
        int ek, ez;
        const int tk = block_excl_scan(ck, ek, s_tmp);
        const int tz = block_excl_scan(cz, ez, s_tmp);
        if (k < nblk) {
            s_apre[k] = ak_tot + ek;
            s_zpre[k] = az_tot + ez;
        }
        ak_tot += tk;
        az_tot += tz;
        double v[2] = {a, d};
        block_sum<2>(v, s_red);
        kt += v[0];
        l1 += v[1];
    }
    if (threadIdx.x == 0) {
        s_apre[nblk] = ak_tot;
        s_zpre[nblk] = az_tot;
    }
    __syncthreads();
    // rejected nonzero coefficients travel above the look-ahead count
    const double rnz = floor(kt / kRejNz);
    kt -= rnz * kRejNz;
    const int I = P->n_stages - 1;
    const StageDesc& st = P->st[Cp.stage];
    const int i_new = switch_dictionary(Cp.stage, I, S.gamma, P->Gamma, kt, st.rc, (double)P->K);
    if (i_new != Cp.stage || rnz > 0.0) {   // a switch, or a rejection that zeroed x_t[j]: restart
        C.stage = i_new;
        C.ksince = 0;
        C.tau = 1.0;
    } else {
        C.ksince = Cp.ksince + 1;
        C.tau = S.tau_next;
    }
    C.iter = Cp.iter + 1;
    C.par = 1 - Cp.par;
    C.n_act = ak_tot;
    C.n_nz = az_tot;
    C.nseg_act = nblk;
    C.nseg_nz = nblk;
    C.l1 = l1;
    kt_out = kt;
    return 0;
}

// ---------------------------------------------------------------------------
// forward gathers for one lane's rows r0..r0+3 over the staged nonzeros [k0, k1)
// (same per-element arithmetic as fwd_accumulate).  Dense: G columns per step,
// every load issued before the first product.  Kronecker: staged entries are
// (j1 << 16) | j2; four atoms generated together, term by term.
// ---------------------------------------------------------------------------
// G: column loads in flight per lane per step (the forward launch keeps 2 or 4 to
// stay within its registers; the per-signal step, 4 or 8)
template <int DT, int G = (DT == SL1_F64 ? 2 : 4)>
__device__ __forceinline__ void fwd_dense_gather(const StageDesc& st, int N, int r0, const int* s_j, const double* s_x,
                                                 int k0, int k1, double (&acc)[4]) {
    constexpr bool kScaled = DT == SL1_BF16 || DT == SL1_FP8_E4M3;
    const float* scale = kScaled ? st.scale : nullptr;
    for (int k = k0; k < k1; k += G) {
        Raw4<DT> r[G];
        double xs[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int kk = min(k + g, k1 - 1);
            const int j = s_j[kk];
            r[g] = raw_load<DT>(st.A, (size_t)j * N + r0);
            xs[g] = k + g < k1 ? s_x[kk] : 0.0;
            if (scale) xs[g] *= (double)scale[j];
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (k + g < k1) {
                double a[4];
                raw_get<DT>(r[g], a);
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v] += xs[g] * a[v];
            }
        }
    }
}

// Bsrc / Csrc: the stage's factors, in global memory or staged in LDS (same layout)
template <int DT>
__device__ __forceinline__ void fwd_kron_gather(const StageDesc& st, const void* Bsrc, const void* Csrc, int r0,
                                                const int* s_j, const double* s_x, int k0, int k1,
                                                double (&acc)[4]) {
    constexpr int G = DT == SL1_F64 ? 2 : 4;
    const int n1 = st.n1, k1d = st.k1, n2 = st.n2, k2 = st.k2, R = st.R;
    const int i1 = r0 / n2, i2 = r0 - i1 * n2;
    for (int k = k0; k < k1; k += G) {
        int j1[G], j2[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int jp = s_j[min(k + g, k1 - 1)];
            j1[g] = jp >> 16;
            j2[g] = jp & 0xFFFF;
        }
        if constexpr (DT == SL1_F64) {
            const double* Bf = (const double*)Bsrc;
            const double* Cf = (const double*)Csrc;
            double a[G][4];
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int v = 0; v < 4; ++v) a[g][v] = 0.0;
            for (int r = 0; r < R; ++r) {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const double bv = Bf[((size_t)r * k1d + j1[g]) * n1 + i1];
                    const f64v2* cp = (const f64v2*)(Cf + ((size_t)r * k2 + j2[g]) * n2 + i2);
                    const f64v2 c0 = cp[0], c1 = cp[1];
                    a[g][0] += bv * c0[0]; a[g][1] += bv * c0[1]; a[g][2] += bv * c1[0]; a[g][3] += bv * c1[1];
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (k + g < k1) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[v] += s_x[k + g] * a[g][v];
                }
        } else {
            float a[G][4];
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int v = 0; v < 4; ++v) a[g][v] = 0.f;
            for (int r = 0; r < R; ++r) {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    float bv, cv[4];
                    if constexpr (DT == SL1_F32) {
                        bv = ((const float*)Bsrc)[((size_t)r * k1d + j1[g]) * n1 + i1];
                        const f32v4 c = *(const f32v4*)((const float*)Csrc + ((size_t)r * k2 + j2[g]) * n2 + i2);
                        cv[0] = c[0]; cv[1] = c[1]; cv[2] = c[2]; cv[3] = c[3];
                    } else if constexpr (DT == SL1_FP8_E4M3) {
                        // four consecutive rows i2 .. i2+3 of C_r (i2 % 4 == 0: one aligned word)
                        const uint32_t bq = ((const uint8_t*)Bsrc)[((size_t)r * k1d + j1[g]) * n1 + i1];
                        bv = __builtin_amdgcn_cvt_pk_f32_fp8((int)bq, false)[0];
                        const uint32_t cq = *(const uint32_t*)((const uint8_t*)Csrc + ((size_t)r * k2 + j2[g]) * n2 + i2);
                        const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)cq, false);
                        const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)cq, true);
                        cv[0] = lo[0]; cv[1] = lo[1]; cv[2] = hi[0]; cv[3] = hi[1];
                    } else {
                        bv = bf16_to_f(((const uint16_t*)Bsrc)[((size_t)r * k1d + j1[g]) * n1 + i1]);
                        const u16x4 c = *(const u16x4*)((const uint16_t*)Csrc + ((size_t)r * k2 + j2[g]) * n2 + i2);
                        cv[0] = bf16_to_f(c[0]); cv[1] = bf16_to_f(c[1]); cv[2] = bf16_to_f(c[2]); cv[3] = bf16_to_f(c[3]);
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) a[g][v] = fmaf(bv, cv[v], a[g][v]);
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (k + g < k1) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[v] += s_x[k + g] * (double)a[g][v];
                }
        }
    }
}

// ---------------------------------------------------------------------------
// FAuST stages (A~ = S_1 S_2 ... S_J, sparse factors): products through the chain
// with FP64 accumulation, every sum in a fixed order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double faust_val(const void* v, long long i, int dtype) {
    return dtype == SL1_F64 ? ((const double*)v)[i] : (double)((const float*)v)[i];
}

// out = S_l in (CSR rows of factor l, 0-based; out has dim[l] rows), one thread per row
__device__ __forceinline__ void faust_rows(const FaustDesc& F, int dtype, int l, const double* in, double* out) {
    const int rows = F.dim[l];
    const int* ptr = F.ptr + F.fp[l];
    const int* idx = F.idx + F.fz[l];
    for (int i = threadIdx.x; i < rows; i += blockDim.x) {
        const int e0 = ptr[i], e1 = ptr[i + 1];
        double s = 0.0;
#pragma unroll 4
        for (int e = e0; e < e1; ++e) s += faust_val(F.val, F.fz[l] + e, dtype) * in[idx[e]];
        out[i] = s;
    }
}

// out = S_l^T in (CSR rows of the transpose of factor l; out has dim[l+1] rows)
__device__ __forceinline__ void faust_trows(const FaustDesc& F, int dtype, int l, const double* in, double* out) {
    const int rows = F.dim[l + 1];
    const int* ptr = F.tptr + F.tp[l];
    const int* idx = F.tidx + F.tz[l];
    for (int i = threadIdx.x; i < rows; i += blockDim.x) {
        const int e0 = ptr[i], e1 = ptr[i + 1];
        double s = 0.0;
#pragma unroll 4
        for (int e = e0; e < e1; ++e) s += faust_val(F.tval, F.tz[l] + e, dtype) * in[idx[e]];
        out[i] = s;
    }
}

// w = S_{J-1}^T ... S_1^T z (z in va; va, vb: the chain's LDS vectors) into wg
// (global); called by the whole block after z is in va, ends with a barrier.
__device__ __forceinline__ void faust_chain_w(const StageDesc& st, double* va, double* vb, double* wg) {
    __syncthreads();
    const FaustDesc& F = *st.fa;
    double* in = va;
    double* out = vb;
    for (int l = 0; l + 1 < F.J; ++l) {
        faust_trows(F, st.dtype, l, in, out);
        __syncthreads();
        double* t = in;
        in = out;
        out = t;
    }
    for (int i = threadIdx.x; i < F.dim[F.J - 1]; i += blockDim.x) wg[i] = in[i];
    __syncthreads();       // the region is reused by the block's next signal
}

// Forward product u = A~ x_t of a FAuST stage for one signal (all N <= 1024 rows):
// v = S_J x from the nonzeros of x -- each nonzero's column of S_J (a row of S_J^T)
// is scattered, q nonzeros at a time, into column c of an LDS block M[row][q]
// (distinct rows within a column), whose rows are then summed in list order --
// then v <- S_l v for l = J-1 .. 1.  Region: two vectors of maxd doubles, M
// (dim[J-1] x q doubles), the chunk's column bounds (2 x kFwdBlock ints).
// Returns u in LDS.  Called by the whole block.
__device__ const double* fwd_faust(const StageDesc& st, int nnz, const int* nzi, const double* nzx,
                                   const int* s_zpre, int nseg_nz, int* s_j, double* s_x, char* region) {
    const FaustDesc& F = *st.fa;
    const int J = F.J, maxd = F.maxd, q = F.q, dl = F.dim[J - 1];
    double* va = (double*)region;
    double* vb = va + maxd;
    double* M = vb + maxd;
    int* s_e0 = (int*)(M + (size_t)dl * q);
    int* s_e1 = s_e0 + kFwdBlock;
    const int* tptr = F.tptr + F.tp[J - 1];
    const int* tidx = F.tidx + F.tz[J - 1];
    for (int i = threadIdx.x; i < dl; i += kFwdBlock) va[i] = 0.0;
    __syncthreads();
    for (int base = 0; base < nnz; base += kFwdBlock) {
        const int cnt = min(kFwdBlock, nnz - base);
        if ((int)threadIdx.x < cnt) {
            const int pos = list_pos(s_zpre, nseg_nz, base + threadIdx.x);
            const int j = nzi[pos];
            s_j[threadIdx.x] = j;
            s_x[threadIdx.x] = nzx[pos];
            s_e0[threadIdx.x] = tptr[j];
            s_e1[threadIdx.x] = tptr[j + 1];
        }
        for (int k0 = 0; k0 < cnt; k0 += q) {
            const int cc = min(q, cnt - k0);
            for (int i = threadIdx.x; i < dl * q; i += kFwdBlock) M[i] = 0.0;
            __syncthreads();
#pragma unroll 4
            for (int c = 0; c < cc; ++c) {
                const int e0 = s_e0[k0 + c], n = s_e1[k0 + c] - e0;
                const double xv = s_x[k0 + c];
                for (int e = threadIdx.x; e < n; e += kFwdBlock)
                    M[(size_t)tidx[e0 + e] * q + c] = faust_val(F.tval, F.tz[J - 1] + e0 + e, st.dtype) * xv;
            }
            __syncthreads();
            for (int i = threadIdx.x; i < dl; i += kFwdBlock) {
                double s = 0.0;
                for (int c = 0; c < cc; ++c) s += M[(size_t)i * q + c];
                va[i] += s;
            }
            __syncthreads();
        }
    }
    double* in = va;
    double* out = vb;
    for (int l = J - 2; l >= 0; --l) {
        faust_rows(F, st.dtype, l, in, out);
        __syncthreads();
        double* t = in;
        in = out;
        out = t;
    }
    return in;
}

// ---------------------------------------------------------------------------
// forward product and residual (Section III-C: rho~_t = y - A~ x_t)
// items: row chunks of 1024 rows; wave pair (2s, 2s + 1) covers rows
// 256 s .. 256 s + 255 of the chunk (4 per lane) and splits the nonzeros of x_t
// (staged once per item with their values); the odd wave's partial meets the
// even wave's in LDS.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kFwdBlock, 4) void k_fwd(const SolveParams* __restrict__ P, int slot) {
    extern __shared__ __align__(16) char smem[];
    const int prev = 1 - slot;
    const int N = P->N, batch = P->batch;
    const int nseg1 = P->nseg_max + 1;
    int* s_apre = (int*)smem;
    int* s_zpre = s_apre + nseg1;
    int* s_j = s_zpre + nseg1;
    int* s_wpre = s_j + kFwdBlock;                      // work map (batch + 1)
    double* s_x = (double*)(((uintptr_t)(s_wpre + batch + 1) + 15) & ~(uintptr_t)15);
    double* s_u = s_x + kFwdBlock;                      // [4 sub-chunks][256 rows]: odd waves' partials
    char* s_fac = (char*)(s_u + 4 * 256);               // a Kronecker stage's factors (fwd_fac_lds bytes)
    __shared__ double s_red[48];
    __shared__ int s_tmp[16];

    const int* cnt_cur = P->cnt_fwd + (size_t)slot * batch;
    const int total = build_work_map(cnt_cur, batch, s_wpre, s_tmp);
    // a signal without work in this slot is finished: clear its count in the
    // other slot too, so no later forward launch visits it (the other slot is
    // read only by the next forward launch; live signals have work here), and
    // mark this slot's control state done (no block of this launch reads it:
    // blocks read the other slot, and only live signals' blocks write this one)
    if (blockIdx.x == 0) {
        for (int b = threadIdx.x; b < batch; b += blockDim.x)
            if (s_wpre[b + 1] == s_wpre[b]) {
                P->cnt_fwd[(size_t)prev * batch + b] = 0;
                P->ctrl[2 * b + slot].done = 1;
            }
    }
    const int per = (total + gridDim.x - 1) / gridDim.x;
    const int g0 = blockIdx.x * per, g1 = min(total, g0 + per);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int cur_b = -1, finished = 0;
    Control C;
    __shared__ Control s_cp;
    for (int g = g0; g < g1; ++g) {
        const int b = uni(find_signal(s_wpre, batch, g));
        const int item = uni(g - s_wpre[b]);
        if (b != cur_b) {
            cur_b = b;
            // C_{t-1} read once for the whole block, so that every thread takes
            // the same path through the barriers below; the scalars of t-1 and the
            // update partials are fetched in the same round trip (they are only
            // used when C_{t-1} says so)
            __syncthreads();
            if (threadIdx.x == 0) s_cp = P->ctrl[2 * b + prev];
            double up0[4] = {0.0, 0.0, 0.0, 0.0};
            if ((int)threadIdx.x < P->nseg_max) {
                const double* up = P->upd_part + ((size_t)b * P->nseg_max + threadIdx.x) * 4;
                up0[0] = up[0];
                up0[1] = up[1];
                up0[2] = up[2];
                up0[3] = up[3];
            }
            const Scalars Sp = P->sc[b];
            __syncthreads();
            const Control Cp = s_cp;
            if (Cp.done) {           // finished in an earlier launch: nothing to do
                finished = 1;
                continue;
            }
            Scalars S;
            double kt = 0.0;
            finished = advance_control(P, b, Cp, Sp, up0, C, s_apre, s_zpre, s_red, s_tmp, S, kt);
            if (finished) {
                if (item == 0 && threadIdx.x == 0) {
                    Final F;
                    F.gap = S.Gt;
                    F.gap_cert = S.Gp + S.delta;
                    F.iters = Cp.iter;
                    F.stage = Cp.stage;
                    F.status = S.conv == 2 ? SL1_MAXITER : SL1_OK;
                    F.par = Cp.par;
                    F.t0 = Cp.t0;
                    F.tconv = S.tconv;
                    P->fin[b] = F;
                    // the other slot is read by this launch's other blocks of the
                    // signal: it is marked done by the next forward launch
                    Control D = Cp;
                    D.done = 1;
                    D.advance = 0;
                    P->ctrl[2 * b + slot] = D;
                    P->cnt_adj[b] = 0;
                    P->cnt_adjk[b] = 0;
                    P->cnt_adjf[b] = 0;
                    P->cnt_upd[b] = 0;
                    P->cnt_gemm[b] = 0;
                    P->cnt_fwd[(size_t)prev * batch + b] = 0;
                    *(int4*)(P->sig_stat + 4 * b) = make_int4(0, 0, 0, 0);
                    atomicSub(P->active_signals, 1);
                }
            } else {
                if (!Cp.advance) {
                    const int* zp = nzpre(P, b, C.par);
                    for (int s = threadIdx.x; s <= C.nseg_nz; s += kFwdBlock) s_zpre[s] = zp[s];
                    __syncthreads();
                }
                if (item == 0) {
                    if (Cp.advance) {
                        int* ap = actpre(P, b, C.par);
                        int* zp = nzpre(P, b, C.par);
                        for (int s = threadIdx.x; s <= C.nseg_act; s += kFwdBlock) {
                            ap[s] = s_apre[s];
                            zp[s] = s_zpre[s];
                        }
                    }
                    if (threadIdx.x == 0) {
                        const StageDesc& stn = P->st[C.stage];
                        const int items = adj_items(stn, C.n_act, N);
                        // large preserved sets on the exact dense stage join the batched product
                        // while enough signals qualify (the host decides between chunks)
                        const bool qual = P->gemm_min > 0 && C.stage == P->n_stages - 1 &&
                                          stn.kind == kDense && C.n_act >= P->gemm_min;
                        const bool gemm = qual && P->gemm_on;
                        Control D = C;
                        D.advance = 1;
                        // correlation-partial slots the update launch reduces: 4 per item, or
                        // the product's 4 per 64-atom tile
                        D.nslot = gemm ? 4 * ((P->K + kGemmAtoms - 1) / kGemmAtoms) : 4 * items;
                        P->ctrl[2 * b + slot] = D;
                        // per-signal statistics, plain stores (reduced once per chunk)
                        *(int4*)(P->sig_stat + 4 * b) =
                            make_int4(C.n_act, C.n_act, C.stage < P->n_stages - 1 ? 1 : 0, qual ? 1 : 0);
                        P->cnt_adj[b] = (stn.kind == kDense && !gemm) ? items : 0;
                        P->cnt_adjk[b] = stn.kind == kKron ? items : 0;
                        P->cnt_adjf[b] = stn.kind == kFaust ? C.stage + 1 : 0;
                        P->cnt_gemm[b] = gemm ? 1 : 0;
                        P->cnt_upd[b] = max(1, (C.n_act + kSeg - 1) / kSeg);
                        if (Cp.advance && P->trace && Cp.iter < P->trace_cap) {
                            double* tr = P->trace + ((size_t)b * P->trace_cap + Cp.iter) * SL1_TRACE_FIELDS;
                            tr[0] = Cp.iter; tr[1] = Cp.stage; tr[2] = Cp.n_act; tr[3] = C.n_act;
                            tr[4] = kt;
                            tr[5] = S.Gp; tr[6] = S.Gt; tr[7] = S.delta; tr[8] = P->rule ? S.Rd : S.Rp; tr[9] = S.gamma;
                            tr[10] = Cp.l1; tr[11] = S.P; tr[12] = Cp.n_nz;
                        }
                    }
                }
            }
        }
        if (finished) continue;

        const int stg = uni(C.stage), par = uni(C.par), nnz = uni(C.n_nz), nseg_nz = uni(C.nseg_nz);
        const StageDesc& st = P->st[stg];
        const bool kron = st.kind == kKron;
        // wave w: 256-row sub-chunk w / 2 of this 1024-row item, half w % 2 of the nonzeros
        const int sub = w >> 1, half = w & 1;
        const int r0 = item * kFwdRows + sub * 256 + lane * 4;
        const bool rows_ok = r0 < N;
        // y of the rows this lane finishes, fetched before the gather
        double yv[4] = {0.0, 0.0, 0.0, 0.0};
        if (half == 0 && rows_ok) {
#pragma unroll
            for (int v = 0; v < 4; ++v) yv[v] = yval(P, b, r0 + v);
        }
        const int* nzi = nzbuf(P, b, par);
        const double* nzx = nzxbuf(P, b, par);
        // with many nonzeros, a Kronecker stage's factors are read from LDS: the
        // block stages all R pairs (B_r, C_r) once (16-byte copies, same layout)
        const void* Bsrc = st.B;
        const void* Csrc = st.C;
        if (kron && nnz >= kFwdFacNnz) {
            const int es = st.dtype == SL1_F64 ? 8 : (st.dtype == SL1_F32 ? 4 : (st.dtype == SL1_BF16 ? 2 : 1));
            const size_t bb = (size_t)st.R * st.n1 * st.k1 * es, cb = (size_t)st.R * st.n2 * st.k2 * es;
            if (bb + cb <= (size_t)P->fwd_fac_lds) {
                // sizes are multiples of 16 bytes: factor dimensions are multiples of 16
                const uint4* gb = (const uint4*)st.B;
                const uint4* gc = (const uint4*)st.C;
                uint4* lb = (uint4*)s_fac;
                uint4* lc = (uint4*)(s_fac + bb);
                for (size_t q = threadIdx.x; q < bb / 16; q += kFwdBlock) lb[q] = gb[q];
                for (size_t q = threadIdx.x; q < cb / 16; q += kFwdBlock) lc[q] = gc[q];
                Bsrc = s_fac;
                Csrc = s_fac + bb;
            }
        }
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (st.kind == kFaust) {
            // the whole chain in this block (N <= 1024: one item); the even waves take their rows
            const double* u = fwd_faust(st, nnz, nzi, nzx, s_zpre, nseg_nz, s_j, s_x, s_fac);
            if (half == 0 && rows_ok) {
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v] = u[r0 + v];
            }
        }
        for (int base = 0; st.kind != kFaust && base < nnz; base += kFwdBlock) {
            const int cnt = min(kFwdBlock, nnz - base);
            if ((int)threadIdx.x < cnt) {
                const int pos = list_pos(s_zpre, nseg_nz, base + threadIdx.x);
                const int j = nzi[pos];
                if (kron) {
                    const int j1 = j / st.k2;
                    s_j[threadIdx.x] = (j1 << 16) | (j - j1 * st.k2);
                } else {
                    s_j[threadIdx.x] = j;
                }
                s_x[threadIdx.x] = nzx[pos];
            }
            __syncthreads();
            const int ph = (cnt + 1) >> 1;
            const int k0 = half ? ph : 0, k1 = half ? cnt : ph;
            if (rows_ok && k0 < k1) {
                switch (st.kind * 4 + st.dtype) {
                    case kDense * 4 + SL1_F64: fwd_dense_gather<SL1_F64>(st, N, r0, s_j, s_x, k0, k1, acc); break;
                    case kDense * 4 + SL1_F32: fwd_dense_gather<SL1_F32>(st, N, r0, s_j, s_x, k0, k1, acc); break;
                    case kDense * 4 + SL1_BF16: fwd_dense_gather<SL1_BF16>(st, N, r0, s_j, s_x, k0, k1, acc); break;
                    case kDense * 4 + SL1_FP8_E4M3: fwd_dense_gather<SL1_FP8_E4M3>(st, N, r0, s_j, s_x, k0, k1, acc); break;
                    case kKron * 4 + SL1_F64: fwd_kron_gather<SL1_F64>(st, Bsrc, Csrc, r0, s_j, s_x, k0, k1, acc); break;
                    case kKron * 4 + SL1_F32: fwd_kron_gather<SL1_F32>(st, Bsrc, Csrc, r0, s_j, s_x, k0, k1, acc); break;
                    case kKron * 4 + SL1_FP8_E4M3:
                        fwd_kron_gather<SL1_FP8_E4M3>(st, Bsrc, Csrc, r0, s_j, s_x, k0, k1, acc);
                        break;
                    default: fwd_kron_gather<SL1_BF16>(st, Bsrc, Csrc, r0, s_j, s_x, k0, k1, acc); break;
                }
            }
            __syncthreads();
        }
        if (half == 1) {
#pragma unroll
            for (int v = 0; v < 4; ++v) s_u[sub * 256 + lane * 4 + v] = acc[v];
        }
        __syncthreads();
        // rho = y - u and the stored direction z (rho itself, or its FP32 / BF16
        // rounding when the stage's matrix-core product takes that input type)
        const int zround = (st.kind == kKron && (st.dtype == SL1_BF16 || st.dtype == SL1_FP8_E4M3))
                               ? 2 : ((st.kind == kKron && st.dtype == SL1_F32) ? 1 : 0);
        double sums[3] = {0.0, 0.0, 0.0};
        if (half == 0 && rows_ok) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double u = acc[v] + s_u[sub * 256 + lane * 4 + v];
                const double rho = yv[v] - u;
                double zd = rho;
                if (zround == 1) zd = (double)(float)rho;
                else if (zround == 2) zd = (double)bf16_rne((float)rho);
                P->z[(size_t)b * N + r0 + v] = zd;
                sums[0] += rho * rho;
                sums[1] += zd * zd;
                sums[2] += yv[v] * zd;
            }
        }
        block_sum<3>(sums, s_red);
        if (threadIdx.x == 0) {
            double* rp = P->res_part + ((size_t)b * P->nrc + item) * 3;
            rp[0] = sums[0];
            rp[1] = sums[1];
            rp[2] = sums[2];
        }
        if (st.kind == kFaust) {
            // the FAuST correlations' chain w = S_{J-1}^T ... S_1^T z of this signal (one
            // item covers all N <= 1024 rows), for the launch that applies S_J^T to the
            // w of many signals at once; z and the two chain vectors reuse the factor region
            const FaustDesc& F = *st.fa;
            double* va = (double*)s_fac;
            double* vb = va + F.maxd;
            if (half == 0 && rows_ok) {
#pragma unroll
                for (int v = 0; v < 4; ++v) va[r0 + v] = yv[v] - (acc[v] + s_u[sub * 256 + lane * 4 + v]);
            }
            faust_chain_w(st, va, vb, P->fw + (size_t)b * kFaustMaxDim);
        }
    }
}

// ---------------------------------------------------------------------------
// adjoint: Kronecker correlations of one item, G[j2, j1] = sum_r (C_r^T P B_r)[j2, j1] for
// the atoms j = j1 k2 + j2 with j2 in [a0, a0 + TJ2) and j1 in [cb0, cb0 + TJ1), where
// P is the stored residual direction as an n2 x n1 matrix (in LDS) and (TJ2, TJ1) =
// (st.kt2, st.kt1), multiples of 16 chosen per stage (sl1_tune_kron measures them).
//   Phase 1: V_r = C_r[:, a0:a0+TJ2]^T P for every term: 16 x 16 MFMA output tiles over
//            (term, row block, column block), spread over the four waves; V in LDS as
//            [r][jj][i1] (BF16 stages: a hi and a lo BF16 part).
//   Phase 2: G = [V_1 .. V_R] [B_1; ..; B_R] restricted to the item's columns: the terms
//            are folded into one contraction of length R n1; every 16 x 16 output tile
//            belongs to one wave, which forms its whole contraction in a fixed order (no
//            cross-wave sums) and writes g and its maxima.
// MFMA operand layout (wave64, 16 x 16 shapes): lane l holds A[l % 16][k], B[k][l % 16]
// with k = l / 16 (x4 shapes) or 4 (l / 16) + v (x16 shapes); the FP32 and BF16 results
// are D[4 (l / 16) + v][l % 16], the FP64 16x16x4 result is D[4 v + l / 16][l % 16].
// ---------------------------------------------------------------------------

// one output tile's epilogue: g_j for its 16 x 16 atoms and the lane's maxima over the
// preserved ones (|g| + eps ||z||_{q*}, |g|, eps)
template <bool kF64Layout, typename D4>
__device__ __forceinline__ void kron_tile_out(const StageDesc& st, const uint8_t* mask, double* gvec, double rz,
                                              int j2b, int j1, const D4& d, double (&mx)[3]) {
    const int l = threadIdx.x & 63, lk = l >> 4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int row = kF64Layout ? 4 * v + lk : 4 * lk + v;
        const int j = j1 * st.k2 + j2b + row;
        const double sv = (double)d[v];
        gvec[j] = sv;
        if (mask[j]) {
            const double e = st.eps[j];
            mx[0] = fmax(mx[0], fabs(sv) + e * rz);
            mx[1] = fmax(mx[1], fabs(sv));
            mx[2] = fmax(mx[2], e);
        }
    }
}

__device__ __forceinline__ void kron_item_f64(const StageDesc& st, int a0, int cb0, const double* zs, double* V,
                                              const uint8_t* mask, double* gvec, double rz, double (&mx)[3]) {
    const int n1 = st.n1, n2 = st.n2, k1 = st.k1, k2 = st.k2, R = st.R, tj2 = st.kt2, tj1 = st.kt1;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const double* Bf = (const double*)st.B;
    const double* Cf = (const double*)st.C;
    const int nrb = tj2 >> 4, ncb = n1 >> 4;
    for (int t = w; t < nrb * ncb * R; t += 4) {
        const int r = t / (nrb * ncb), jt = (t / ncb) % nrb, it = t % ncb;
        const double* A = Cf + ((size_t)r * k2 + a0 + 16 * jt + li) * n2 + lk;
        const double* Bp = zs + (size_t)(16 * it + li) * n2 + lk;
        f64x4 d = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < n2; k0 += 4) d = __builtin_amdgcn_mfma_f64_16x16x4f64(A[k0], Bp[k0], d, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) V[((size_t)r * tj2 + 16 * jt + 4 * v + lk) * n1 + 16 * it + li] = d[v];
    }
    __syncthreads();
    const int nct = tj1 >> 4;
    for (int t = w; t < nrb * nct; t += 4) {
        const int jt = t / nct, ct = t % nct;
        f64x4 d = {0.0, 0.0, 0.0, 0.0};
        for (int r = 0; r < R; ++r) {
            const double* A = V + ((size_t)r * tj2 + 16 * jt + li) * n1 + lk;
            const double* Bp = Bf + ((size_t)r * k1 + cb0 + 16 * ct + li) * n1 + lk;
            for (int k0 = 0; k0 < n1; k0 += 4) d = __builtin_amdgcn_mfma_f64_16x16x4f64(A[k0], Bp[k0], d, 0, 0, 0);
        }
        kron_tile_out<true>(st, mask, gvec, rz, a0 + 16 * jt, cb0 + 16 * ct + li, d, mx);
    }
}

__device__ __forceinline__ void kron_item_f32(const StageDesc& st, int a0, int cb0, const float* zs, float* V,
                                              const uint8_t* mask, double* gvec, double rz, double (&mx)[3]) {
    const int n1 = st.n1, n2 = st.n2, k1 = st.k1, k2 = st.k2, R = st.R, tj2 = st.kt2, tj1 = st.kt1;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const float* Bf = (const float*)st.B;
    const float* Cf = (const float*)st.C;
    const int nrb = tj2 >> 4, ncb = n1 >> 4;
    for (int t = w; t < nrb * ncb * R; t += 4) {
        const int r = t / (nrb * ncb), jt = (t / ncb) % nrb, it = t % ncb;
        const float* A = Cf + ((size_t)r * k2 + a0 + 16 * jt + li) * n2 + lk;
        const float* Bp = zs + (size_t)(16 * it + li) * n2 + lk;
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < n2; k0 += 4) d = __builtin_amdgcn_mfma_f32_16x16x4f32(A[k0], Bp[k0], d, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) V[((size_t)r * tj2 + 16 * jt + 4 * lk + v) * n1 + 16 * it + li] = d[v];
    }
    __syncthreads();
    const int nct = tj1 >> 4;
    for (int t = w; t < nrb * nct; t += 4) {
        const int jt = t / nct, ct = t % nct;
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
        for (int r = 0; r < R; ++r) {
            const float* A = V + ((size_t)r * tj2 + 16 * jt + li) * n1 + lk;
            const float* Bp = Bf + ((size_t)r * k1 + cb0 + 16 * ct + li) * n1 + lk;
            for (int k0 = 0; k0 < n1; k0 += 4) d = __builtin_amdgcn_mfma_f32_16x16x4f32(A[k0], Bp[k0], d, 0, 0, 0);
        }
        kron_tile_out<false>(st, mask, gvec, rz, a0 + 16 * jt, cb0 + 16 * ct + li, d, mx);
    }
}

// four consecutive factor entries as BF16 bits: BF16 storage as is; FP8 E4M3 storage
// decoded (every E4M3 value has at most 4 significant bits, so its FP32 form ends in
// 16 zero bits and its BF16 form is exact)
__device__ __forceinline__ u16x4 bf16x4_of(const uint16_t* p) { return *(const u16x4*)p; }
__device__ __forceinline__ u16x4 bf16x4_of(const uint8_t* p) {
    const uint32_t q = *(const uint32_t*)p;
    const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)q, false);
    const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)q, true);
    u16x4 r;
    r[0] = (uint16_t)(__float_as_uint(lo[0]) >> 16);
    r[1] = (uint16_t)(__float_as_uint(lo[1]) >> 16);
    r[2] = (uint16_t)(__float_as_uint(hi[0]) >> 16);
    r[3] = (uint16_t)(__float_as_uint(hi[1]) >> 16);
    return r;
}

__device__ __forceinline__ s16x4 as_s16x4(const u16x4& u) {
    s16x4 s;
#pragma unroll
    for (int v = 0; v < 4; ++v) s[v] = (short)u[v];
    return s;
}

// BF16 (or FP8) factors: P (the stored residual, bf16-exact) and C_r enter the first
// product exactly; the FP32 intermediate V is split into hi + lo BF16 parts so the
// second product loses at most 2^-16 |V| (folded into eps by the library).
template <typename FT>
__device__ __forceinline__ void kron_item_bf16(const StageDesc& st, int a0, int cb0, const float* zs, uint16_t* Vh,
                                               const uint8_t* mask, double* gvec, double rz, double (&mx)[3]) {
    const int n1 = st.n1, n2 = st.n2, k1 = st.k1, k2 = st.k2, R = st.R, tj2 = st.kt2, tj1 = st.kt1;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    uint16_t* Vl = Vh + (size_t)R * tj2 * n1;
    const FT* Bf = (const FT*)st.B;
    const FT* Cf = (const FT*)st.C;
    const int nrb = tj2 >> 4, ncb = n1 >> 4;
    for (int t = w; t < nrb * ncb * R; t += 4) {
        const int r = t / (nrb * ncb), jt = (t / ncb) % nrb, it = t % ncb;
        const FT* A = Cf + ((size_t)r * k2 + a0 + 16 * jt + li) * n2 + 4 * lk;
        const float* Bp = zs + (size_t)(16 * it + li) * n2 + 4 * lk;
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < n2; k0 += 16) {
            const s16x4 a = as_s16x4(bf16x4_of(A + k0));
            s16x4 bb;
#pragma unroll
            for (int v = 0; v < 4; ++v) bb[v] = (short)bf16_bits(Bp[k0 + v]);
            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, d, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const float hi = bf16_rne(d[v]);
            const float lo = bf16_rne(d[v] - hi);
            const size_t o = ((size_t)r * tj2 + 16 * jt + 4 * lk + v) * n1 + 16 * it + li;
            Vh[o] = bf16_bits(hi);
            Vl[o] = bf16_bits(lo);
        }
    }
    __syncthreads();
    const int nct = tj1 >> 4;
    for (int t = w; t < nrb * nct; t += 4) {
        const int jt = t / nct, ct = t % nct;
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
        for (int r = 0; r < R; ++r) {
            const size_t vo = ((size_t)r * tj2 + 16 * jt + li) * n1 + 4 * lk;
            const FT* Bp = Bf + ((size_t)r * k1 + cb0 + 16 * ct + li) * n1 + 4 * lk;
            for (int k0 = 0; k0 < n1; k0 += 16) {
                const s16x4 h = as_s16x4(*(const u16x4*)(Vh + vo + k0));
                const s16x4 lo = as_s16x4(*(const u16x4*)(Vl + vo + k0));
                const s16x4 bb = as_s16x4(bf16x4_of(Bp + k0));
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(h, bb, d, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lo, bb, d, 0, 0, 0);
            }
        }
        kron_tile_out<false>(st, mask, gvec, rz, a0 + 16 * jt, cb0 + 16 * ct + li, d, mx);
    }
}

// dense correlation item: NA atoms of one wave (first = first list position);
// eps_j is fetched together with the columns.  ident: the list holds all K atoms,
// which is the identity (compactions keep the order), so positions are atoms and
// the list is not read before the columns.
template <int DT, int NA>
__device__ __forceinline__ void dense_item(const StageDesc& st, int N, const int* act, const int* s_pre, int nseg,
                                           int n_act, bool ident, int first, const double* zs, double rz, double* g, int lane,
                                           double (&mx)[3]) {
    int js[NA];
    int cnt = 0;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const int i = first + q;
        js[q] = i < n_act ? (ident ? i : list_get(act, s_pre, nseg, i)) : -1;
        cnt += i < n_act;
    }
    if (cnt == 0) return;
#pragma unroll
    for (int q = 0; q < NA; ++q)
        if (js[q] < 0) js[q] = js[0];
    double e[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) e[q] = st.eps[js[q]];
    double gv[NA];
    dense_dots_t<DT, NA>(st, N, js, zs, lane, gv);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            if (q < cnt) {
                g[js[q]] = gv[q];
                mx[0] = fmax(mx[0], fabs(gv[q]) + e[q] * rz);
                mx[1] = fmax(mx[1], fabs(gv[q]));
                mx[2] = fmax(mx[2], e[q]);
            }
        }
    }
}

// per-wave maxima of one correlation item into its slot (lane 0 holds them
// already for dense items; Kronecker items reduce over the wave first)
__device__ __forceinline__ void put_wave_max(const SolveParams* P, int b, int item, double (&mx)[3], bool reduce) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (reduce) {
#pragma unroll
        for (int k = 0; k < 3; ++k) mx[k] = wave_max(mx[k]);
    }
    if (lane == 0) {
        double* ap = P->adj_part + (((size_t)b * P->nadj_max + item) * 4 + w) * 3;
        ap[0] = mx[0];
        ap[1] = mx[1];
        ap[2] = mx[2];
    }
}

__device__ __forceinline__ void reduce_res(const SolveParams* P, int b, double* s_red, double& r2, double& zz,
                                           double& yz) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < P->nrc; k += blockDim.x) {
        const double* rp = P->res_part + ((size_t)b * P->nrc + k) * 3;
        v[0] += rp[0];
        v[1] += rp[1];
        v[2] += rp[2];
    }
    block_sum<3>(v, s_red);
    r2 = v[0];
    zz = v[1];
    yz = v[2];
}

// the residual sums together with three maxima already loaded by the caller:
// one pass of barriers (sums in the same fixed order as block_sum; red: 96 doubles)
__device__ __forceinline__ void reduce_res_max(const SolveParams* P, int b, double* red, double (&mx)[3], double& r2,
                                               double& zz, double& yz) {
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < P->nrc; k += blockDim.x) {
        const double* rp = P->res_part + ((size_t)b * P->nrc + k) * 3;
        v[0] += rp[0];
        v[1] += rp[1];
        v[2] += rp[2];
    }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[k] = wave_sum(v[k]);
        mx[k] = wave_max(mx[k]);
    }
    __syncthreads();
    if (l == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            red[k * 16 + w] = v[k];
            red[48 + k * 16 + w] = mx[k];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double a = 0.0, m = red[48 + k * 16];
        for (int q = 0; q < nw; ++q) a += red[k * 16 + q];
        for (int q = 1; q < nw; ++q) m = fmax(m, red[48 + k * 16 + q]);
        v[k] = a;
        mx[k] = m;
    }
    __syncthreads();
    r2 = v[0];
    zz = v[1];
    yz = v[2];
}

// ---------------------------------------------------------------------------
// correlations over the preserved set: g_j = a~_j^T z for j in A_t, and the
// per-wave maxima of the stable dual scaling (Section III-C).  Dense stages and
// Kronecker stages have kernels of their own (the dense one needs few registers
// and runs at high occupancy; the Kronecker one holds MFMA tiles).
// ---------------------------------------------------------------------------
template <int DT>
__device__ __forceinline__ void dense_item_any(const StageDesc& st, int N, const int* act, const int* s_pre, int nseg,
                                               int n_act, bool ident, int first, const double* zs, double rz, double* g,
                                               int lane, double (&mx)[3]) {
    const int apw = dense_apw(N, DT);
    if (apw == 4) dense_item<DT, 4>(st, N, act, s_pre, nseg, n_act, ident, first, zs, rz, g, lane, mx);
    else if (apw == 3) dense_item<DT, 3>(st, N, act, s_pre, nseg, n_act, ident, first, zs, rz, g, lane, mx);
    else if (apw == 2) dense_item<DT, 2>(st, N, act, s_pre, nseg, n_act, ident, first, zs, rz, g, lane, mx);
    else dense_item<DT, 1>(st, N, act, s_pre, nseg, n_act, ident, first, zs, rz, g, lane, mx);
}

__global__ __launch_bounds__(kBlock, 4) void k_adj_dense(const SolveParams* __restrict__ P, int slot) {
    extern __shared__ __align__(16) char smem[];
    const int N = P->N, batch = P->batch;
    const size_t zbytes = ((size_t)N * 8 + 15) & ~(size_t)15;
    int* s_pre = (int*)(smem + zbytes);
    int* s_wpre = s_pre + (P->nseg_max + 1);
    __shared__ double s_red[48];
    __shared__ int s_tmp[16];
    const int total = build_work_map(P->cnt_adj, batch, s_wpre, s_tmp);
    const int per = (total + gridDim.x - 1) / gridDim.x;
    const int g0 = blockIdx.x * per, g1 = min(total, g0 + per);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int cur_b = -1;
    Control C;
    double rz = 0.0;
    for (int g = g0; g < g1; ++g) {
        const int b = uni(find_signal(s_wpre, batch, g));
        const int c = uni(g - s_wpre[b]);
        if (b != cur_b) {
            cur_b = b;
            C = P->ctrl[2 * b + slot];
            double r2, zz, yz;
            reduce_res(P, b, s_red, r2, zz, yz);
            rz = dual_norm_z(P, P->st[C.stage], b, zz);
            const double* zg = P->z + (size_t)b * N;
            double* zsd = (double*)smem;
            for (int i = threadIdx.x * 2; i < N; i += kBlock * 2) *(f64v2*)(zsd + i) = *(const f64v2*)(zg + i);
            const int* ap = actpre(P, b, C.par);
            for (int s = threadIdx.x; s <= C.nseg_act; s += kBlock) s_pre[s] = ap[s];
            __syncthreads();
        }
        const int stg = uni(C.stage), par = uni(C.par), nseg = uni(C.nseg_act), n_act = uni(C.n_act);
        const StageDesc& st = P->st[stg];
        const double* zs = (const double*)smem;
        double* gvec = gbuf(P, b, par);
        const int* act = actbuf(P, b, par);
        const int first = (c * 4 + w) * dense_apw(N, st.dtype);
        double mx[3] = {0.0, 0.0, 0.0};   // max(|g|+eps*|z|), max|g|, max eps over the item
        switch (st.dtype) {
            case SL1_F64: dense_item_any<SL1_F64>(st, N, act, s_pre, nseg, n_act, n_act == P->K, first, zs, rz, gvec, lane, mx); break;
            case SL1_F32: dense_item_any<SL1_F32>(st, N, act, s_pre, nseg, n_act, n_act == P->K, first, zs, rz, gvec, lane, mx); break;
            case SL1_BF16: dense_item_any<SL1_BF16>(st, N, act, s_pre, nseg, n_act, n_act == P->K, first, zs, rz, gvec, lane, mx); break;
            default: dense_item_any<SL1_FP8_E4M3>(st, N, act, s_pre, nseg, n_act, n_act == P->K, first, zs, rz, gvec, lane, mx); break;
        }
        put_wave_max(P, b, c, mx, false);
    }
}

// ---------------------------------------------------------------------------
// batched correlations: the signals whose preserved set on the exact dense
// stage is large share one product G = A^T Z, tiled 64 atoms x 64 signals per
// block (FP64 MFMA 16x16x4; stored entries decoded to FP64 exactly, z in FP64),
// so a column is read once per 64 signals instead of once per signal.  Entries of
// atoms outside a signal's preserved set are discarded.  Rows go in chunks of 32:
// the block stages the chunk's A (stored type) and z (FP64) with coalesced loads
// into one of two LDS buffers while the waves multiply the other.  The four waves
// form a 2 x 2 grid of 32 atoms x 32 signals (2 x 2 MFMA tiles each).  MFMA
// operands: lane l gives A[atom l%16][row 4k + l/16] and z[signal l%16][same row];
// the FP64 accumulator holds D[4v + l/16][l%16] (atom, signal).  Per-16-atom
// maxima of the stable dual scaling go to the slots the update launch reduces
// (4 per 64-atom tile).
// One block's tile is bound by its waves' MFMA rate, so while the tiles are
// fewer than half the blocks each tile's rows are split over up to
// kGemmMaxSplit blocks: they store partial tiles, and k_gemm_fin, launched
// right after, sums each tile's partials in split order and finishes it.
// ---------------------------------------------------------------------------
constexpr int kGR = 32;                 // rows per chunk
constexpr int kGLdA = kGR + 1;          // LDS row length of a staged column (32-bit words)
constexpr int kGLdZ = kGR + 1;          // LDS row length of a staged z (doubles)
constexpr int kGBufA = kGemmAtoms * kGLdA;      // 32-bit words of one A buffer (F64: 2 words each)
constexpr int kGBufZ = kGemmSig * kGLdZ;        // doubles of one z buffer

template <int DT>
__device__ __forceinline__ double gemm_dec(const uint32_t* w, int i) {
    if constexpr (DT == SL1_F64) return __hiloint2double((int)w[2 * i + 1], (int)w[2 * i]);
    else if constexpr (DT == SL1_F32) return (double)__uint_as_float(w[i]);
    else if constexpr (DT == SL1_BF16) return (double)bf16_to_f((uint16_t)w[i]);
    else {
        const auto v = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], false);
        return (double)v[0];
    }
}

// rows r0..r0+kGR (zero past N) of the tile's 64 columns and 64 z vectors: the
// global loads go to registers first (gemm_fetch) and reach LDS later (gemm_put),
// so they are in flight while the previous chunk is multiplied
constexpr int kGQuads = kGemmAtoms * (kGR / 4) / kBlock;     // column quads per thread
constexpr int kGPairs = kGemmSig * (kGR / 2) / kBlock;       // z pairs per thread

template <int DT>
struct GemmRegs {
    Raw4<DT> a[kGQuads];
    f64v2 z[kGPairs];
};

template <int DT>
__device__ __forceinline__ void gemm_fetch(const SolveParams* P, const StageDesc& st, int N, int K, int j0,
                                           const int* sig, int ns, int r0, GemmRegs<DT>& g) {
#pragma unroll
    for (int t = 0; t < kGQuads; ++t) {
        const int e = threadIdx.x + t * kBlock;
        const int c = e / (kGR / 4), q = e - c * (kGR / 4);
        const int r = r0 + 4 * q;
        const int j = min(j0 + c, K - 1);
        g.a[t] = raw_load<DT>(st.A, (size_t)j * N + (r < N ? r : 0));
    }
#pragma unroll
    for (int t = 0; t < kGPairs; ++t) {
        const int e = threadIdx.x + t * kBlock;
        const int sl = e / (kGR / 2), p2 = e - sl * (kGR / 2);
        const int r = r0 + 2 * p2;
        f64v2 v = {0.0, 0.0};
        if (sl < ns && r < N) v = *(const f64v2*)(P->z + (size_t)sig[sl] * N + r);
        g.z[t] = v;
    }
}

template <int DT>
__device__ __forceinline__ void gemm_put(const GemmRegs<DT>& g, int N, int r0, uint32_t* sa, double* sz) {
    constexpr int wpe = DT == SL1_F64 ? 2 : 1;     // 32-bit words per stored entry
#pragma unroll
    for (int t = 0; t < kGQuads; ++t) {
        const int e = threadIdx.x + t * kBlock;
        const int c = e / (kGR / 4), q = e - c * (kGR / 4);
        const bool in = r0 + 4 * q < N;
        uint32_t wv[4 * wpe];
        if constexpr (DT == SL1_F64) {
            double v[4];
            raw_get<DT>(g.a[t], v);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                wv[2 * u] = (uint32_t)__double2loint(in ? v[u] : 0.0);
                wv[2 * u + 1] = (uint32_t)__double2hiint(in ? v[u] : 0.0);
            }
        } else if constexpr (DT == SL1_F32) {
#pragma unroll
            for (int u = 0; u < 4; ++u) wv[u] = in ? __float_as_uint(g.a[t].a[u]) : 0u;
        } else if constexpr (DT == SL1_BF16) {
#pragma unroll
            for (int u = 0; u < 4; ++u) wv[u] = in ? (uint32_t)g.a[t].a[u] : 0u;
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) wv[u] = in ? ((g.a[t].a >> (8 * u)) & 0xFFu) : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4 * wpe; ++u) sa[(c * kGLdA + 4 * q) * wpe + u] = wv[u];
    }
#pragma unroll
    for (int t = 0; t < kGPairs; ++t) {
        const int e = threadIdx.x + t * kBlock;
        const int sl = e / (kGR / 2), p2 = e - sl * (kGR / 2);
        sz[sl * kGLdZ + 2 * p2] = g.z[t][0];
        sz[sl * kGLdZ + 2 * p2 + 1] = g.z[t][1];
    }
}

template <int DT>
__device__ __forceinline__ void gemm_mul(const uint32_t* sa, const double* sz, int wa, int wsg, int li, int lk,
                                         f64x4 (&acc)[2][2]) {
#pragma unroll
    for (int k = 0; k < kGR / 4; ++k) {
        const int row = 4 * k + lk;
        double a[2], z[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) a[q] = gemm_dec<DT>(sa, (32 * wa + 16 * q + li) * kGLdA + row);
#pragma unroll
        for (int p = 0; p < 2; ++p) z[p] = sz[(32 * wsg + 16 * p + li) * kGLdZ + row];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int p = 0; p < 2; ++p) acc[q][p] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], z[p], acc[q][p], 0, 0, 0);
    }
}

// the tile's rows, chunk by chunk: while chunk c is multiplied from one LDS
// buffer, chunk c + 1 (already in registers) goes to the other and chunk c + 2
// is loaded, so every chunk's loads have two chunk periods to arrive
// chunks c0 .. c0 + nch - 1 of the tile (rows from 32 c0)
template <int DT>
__device__ void gemm_block_tile(const SolveParams* P, const StageDesc& st, int N, int K, int j0, const int* sig,
                                int ns, int c0, int nch, uint32_t* sa0, uint32_t* sa1, double* sz0, double* sz1,
                                int wa, int wsg, int li, int lk, f64x4 (&acc)[2][2]) {
    const int r0 = c0 * kGR;
    GemmRegs<DT> g0, g1;
    gemm_fetch<DT>(P, st, N, K, j0, sig, ns, r0, g0);
    if (nch > 1) gemm_fetch<DT>(P, st, N, K, j0, sig, ns, r0 + kGR, g1);
    gemm_put<DT>(g0, N, r0, sa0, sz0);
    __syncthreads();
    if (nch > 2) gemm_fetch<DT>(P, st, N, K, j0, sig, ns, r0 + 2 * kGR, g0);
    for (int c = 0; c < nch; ++c) {
        const bool odd = c & 1;
        gemm_mul<DT>(odd ? sa1 : sa0, odd ? sz1 : sz0, wa, wsg, li, lk, acc);
        if (c + 1 < nch) {
            // chunk c + 1 sits in g1 when c is even, in g0 when c is odd
            if (!odd) gemm_put<DT>(g1, N, r0 + (c + 1) * kGR, sa1, sz1);
            else gemm_put<DT>(g0, N, r0 + (c + 1) * kGR, sa0, sz0);
        }
        __syncthreads();
        if (c + 3 < nch) {
            if (!odd) gemm_fetch<DT>(P, st, N, K, j0, sig, ns, r0 + (c + 3) * kGR, g1);
            else gemm_fetch<DT>(P, st, N, K, j0, sig, ns, r0 + (c + 3) * kGR, g0);
        }
    }
}

// tiles and row splits of one product launch (identical in k_adj_gemm and k_gemm_fin)
struct GemmPlan {
    int nat, tiles, ks, cps, nch;
};
__device__ __forceinline__ GemmPlan gemm_plan(int S, int N, int K, int grid) {
    GemmPlan g;
    g.nat = (K + kGemmAtoms - 1) / kGemmAtoms;
    g.tiles = g.nat * ((S + kGemmSig - 1) / kGemmSig);
    g.nch = (N + kGR - 1) / kGR;
    int ks = 1;
    if (2 * g.tiles <= grid) ks = max(1, min(min(kGemmMaxSplit, g.nch), min(grid, kGemmSplitUnits) / g.tiles));
    g.cps = (g.nch + ks - 1) / ks;                      // chunks per split
    g.ks = (g.nch + g.cps - 1) / g.cps;                 // no empty split
    return g;
}

// g and the per-16-atom maxima of one finished tile (the update launch reduces
// exactly the 4 slots per 64-atom tile written here).  Everything the epilogue
// reads is loaded first (one memory round trip).
__device__ void gemm_epilogue(const SolveParams* P, const StageDesc& st, int slot, const int* s_sig, int s0, int ns,
                              int j0, int ta, int nat, int wa, int wsg, int li, int lk, const f64x4 (&acc)[2][2]) {
    const int K = P->K, nrc = P->nrc;
    // lane: signals s0 + 32 wsg + 16 p + li, atoms j0 + 32 wa + 16 q + 4 v + lk
    int bp[2], par[2];
    bool sv[2];
    double zz[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int sl = 32 * wsg + 16 * p + li;
        sv[p] = sl < ns;
        bp[p] = sv[p] ? s_sig[s0 + sl] : 0;
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        par[p] = P->ctrl[2 * bp[p] + slot].par;
        zz[p] = 0.0;
        for (int k = 0; k < nrc; ++k) zz[p] += P->res_part[((size_t)bp[p] * nrc + k) * 3 + 1];
    }
    double ev[2][4], scv[2][4];
    uint8_t mkv[2][2][4];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = j0 + 32 * wa + 16 * q + 4 * v + lk;
            const bool jin = j < K;
            ev[q][v] = jin ? st.eps[j] : 0.0;
            scv[q][v] = (jin && st.scale) ? (double)st.scale[j] : 1.0;
#pragma unroll
            for (int p = 0; p < 2; ++p) mkv[p][q][v] = (sv[p] && jin) ? P->mask[(size_t)bp[p] * K + j] : (uint8_t)0;
        }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const int b = bp[p];
        const double rz = dual_norm_z(P, st, b, zz[p]);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            double mx[3] = {0.0, 0.0, 0.0};
            if (sv[p]) {
                double* gv = gbuf(P, b, par[p]);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = j0 + 32 * wa + 16 * q + 4 * v + lk;
                    if (mkv[p][q][v]) {
                        double gval = acc[q][p][v];
                        if (st.scale) gval *= scv[q][v];
                        gv[j] = gval;
                        const double e = ev[q][v];
                        mx[0] = fmax(mx[0], fabs(gval) + e * rz);
                        mx[1] = fmax(mx[1], fabs(gval));
                        mx[2] = fmax(mx[2], e);
                    }
                }
            }
            // the four lanes of a signal (l % 16 equal) combine their atoms
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                mx[k] = fmax(mx[k], __shfl_xor(mx[k], 16, 64));
                mx[k] = fmax(mx[k], __shfl_xor(mx[k], 32, 64));
            }
            if (lk == 0 && sv[p]) {
                double* ap = P->adj_part + (((size_t)b * P->nadj_max + ta) * 4 + 2 * wa + q) * 3;
                ap[0] = mx[0];
                ap[1] = mx[1];
                ap[2] = mx[2];
            }
        }
    }
}

__global__ __launch_bounds__(kBlock, 2) void k_adj_gemm(const SolveParams* __restrict__ P, int slot) {
    extern __shared__ __align__(16) char smem[];
    const int N = P->N, K = P->K, batch = P->batch;
    const StageDesc& st = P->st[P->n_stages - 1];
    uint32_t* sa0 = (uint32_t*)smem;
    uint32_t* sa1 = sa0 + kGBufA * 2;                                    // room for FP64 entries
    double* sz0 = (double*)(sa1 + kGBufA * 2);
    double* sz1 = sz0 + kGBufZ;
    int* s_pre = (int*)(sz1 + kGBufZ);                                   // [batch + 1]
    int* s_sig = s_pre + batch + 1;                                      // compacted signal list
    __shared__ int s_tmp[16];
    const int S = build_work_map(P->cnt_gemm, batch, s_pre, s_tmp);
    if (S == 0) return;
    for (int b = threadIdx.x; b < batch; b += kBlock)
        if (s_pre[b + 1] > s_pre[b]) s_sig[s_pre[b]] = b;
    __syncthreads();
    const GemmPlan pl = gemm_plan(S, N, K, gridDim.x);
    const int nat = pl.nat, total = pl.tiles * pl.ks;
    const int per = (total + gridDim.x - 1) / gridDim.x;
    const int g0 = blockIdx.x * per, g1 = min(total, g0 + per);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const int wa = w & 1, wsg = w >> 1;                 // the wave's atom half and signal half
    for (int u = g0; u < g1; ++u) {
        const int g = u / pl.ks, ks = u - g * pl.ks;
        const int ts = g / nat, ta = g - ts * nat;      // signal tile outer, atom tile inner
        const int s0 = ts * kGemmSig, j0 = ta * kGemmAtoms;
        const int ns = min(kGemmSig, S - s0);
        const int c0 = ks * pl.cps, nc = min(pl.nch, c0 + pl.cps) - c0;
        f64x4 acc[2][2];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int p = 0; p < 2; ++p) acc[q][p] = f64x4{0.0, 0.0, 0.0, 0.0};
        switch (st.dtype) {
            case SL1_F64: gemm_block_tile<SL1_F64>(P, st, N, K, j0, s_sig + s0, ns, c0, nc, sa0, sa1, sz0, sz1, wa, wsg, li, lk, acc); break;
            case SL1_F32: gemm_block_tile<SL1_F32>(P, st, N, K, j0, s_sig + s0, ns, c0, nc, sa0, sa1, sz0, sz1, wa, wsg, li, lk, acc); break;
            case SL1_BF16: gemm_block_tile<SL1_BF16>(P, st, N, K, j0, s_sig + s0, ns, c0, nc, sa0, sa1, sz0, sz1, wa, wsg, li, lk, acc); break;
            default: gemm_block_tile<SL1_FP8_E4M3>(P, st, N, K, j0, s_sig + s0, ns, c0, nc, sa0, sa1, sz0, sz1, wa, wsg, li, lk, acc); break;
        }
        if (pl.ks > 1) {
            // partial tile, element-major (coalesced): [unit][16 accumulator entries][256 threads];
            // k_gemm_fin reads it after this launch
            double* part = P->gemm_part + (size_t)u * (kGemmAtoms * kGemmSig);
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int v = 0; v < 4; ++v) part[((q * 2 + p) * 4 + v) * kBlock + threadIdx.x] = acc[q][p][v];
            continue;
        }
        gemm_epilogue(P, st, slot, s_sig, s0, ns, j0, ta, nat, wa, wsg, li, lk, acc);
    }
}

// split product tiles: the partials summed in split order, then the tile's
// epilogue (one block per tile; nothing to do when the launch did not split)
__global__ __launch_bounds__(kBlock, 2) void k_gemm_fin(const SolveParams* __restrict__ P, int slot, int gemm_grid) {
    extern __shared__ __align__(16) char smem[];
    const int N = P->N, K = P->K, batch = P->batch;
    const StageDesc& st = P->st[P->n_stages - 1];
    int* s_pre = (int*)smem;                                              // [batch + 1]
    int* s_sig = s_pre + batch + 1;
    __shared__ int s_tmp[16];
    const int S = build_work_map(P->cnt_gemm, batch, s_pre, s_tmp);
    if (S == 0) return;
    const GemmPlan pl = gemm_plan(S, N, K, gemm_grid);
    if (pl.ks == 1) return;
    for (int b = threadIdx.x; b < batch; b += kBlock)
        if (s_pre[b + 1] > s_pre[b]) s_sig[s_pre[b]] = b;
    __syncthreads();
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const int wa = w & 1, wsg = w >> 1;
    for (int g = blockIdx.x; g < pl.tiles; g += gridDim.x) {
        const int ts = g / pl.nat, ta = g - ts * pl.nat;
        const int s0 = ts * kGemmSig, j0 = ta * kGemmAtoms;
        const int ns = min(kGemmSig, S - s0);
        const double* pt = P->gemm_part + (size_t)g * pl.ks * (kGemmAtoms * kGemmSig);
        f64x4 acc[2][2];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int p = 0; p < 2; ++p) acc[q][p] = f64x4{0.0, 0.0, 0.0, 0.0};
        // four splits' partials are loaded together, then added in split order
        constexpr int kStep = 4;
#pragma unroll 1
        for (int k0 = 0; k0 < pl.ks; k0 += kStep) {
            double part[kStep][16];
#pragma unroll
            for (int k = 0; k < kStep; ++k)
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    part[k][e] = k0 + k < pl.ks
                                     ? pt[(size_t)(k0 + k) * (kGemmAtoms * kGemmSig) + e * kBlock + threadIdx.x]
                                     : 0.0;
#pragma unroll
            for (int k = 0; k < kStep; ++k)
                if (k0 + k < pl.ks) {
#pragma unroll
                    for (int q = 0; q < 2; ++q)
#pragma unroll
                        for (int p = 0; p < 2; ++p)
#pragma unroll
                            for (int v = 0; v < 4; ++v) acc[q][p][v] += part[k][(q * 2 + p) * 4 + v];
                }
        }
        gemm_epilogue(P, st, slot, s_sig, s0, ns, j0, ta, pl.nat, wa, wsg, li, lk, acc);
    }
}

__global__ __launch_bounds__(kBlock, 3) void k_adj_kron(const SolveParams* __restrict__ P, int slot) {
    extern __shared__ __align__(16) char smem[];
    const int N = P->N, K = P->K, batch = P->batch;
    const size_t zbytes = ((size_t)N * 8 + 15) & ~(size_t)15;
    int* s_wpre = (int*)(smem + zbytes);
    char* extra = smem + zbytes + ((((size_t)batch + 1) * 4 + 15) & ~(size_t)15);
    __shared__ double s_red[48];
    __shared__ int s_tmp[16];
    const int total = build_work_map(P->cnt_adjk, batch, s_wpre, s_tmp);
    const int per = (total + gridDim.x - 1) / gridDim.x;
    const int g0 = blockIdx.x * per, g1 = min(total, g0 + per);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int cur_b = -1;
    Control C;
    double rz = 0.0;
    for (int g = g0; g < g1; ++g) {
        const int b = uni(find_signal(s_wpre, batch, g));
        const int c = uni(g - s_wpre[b]);
        if (b != cur_b) {
            cur_b = b;
            C = P->ctrl[2 * b + slot];
            double r2, zz, yz;
            reduce_res(P, b, s_red, r2, zz, yz);
            rz = dual_norm_z(P, P->st[C.stage], b, zz);
            const StageDesc& st0 = P->st[uni(C.stage)];
            const double* zg = P->z + (size_t)b * N;
            if (st0.kind == kKron && st0.dtype != SL1_F64) {
                float* zsf = (float*)smem;
                for (int i = threadIdx.x; i < N; i += kBlock) zsf[i] = (float)zg[i];
            } else {
                double* zsd = (double*)smem;
                for (int i = threadIdx.x * 2; i < N; i += kBlock * 2) *(f64v2*)(zsd + i) = *(const f64v2*)(zg + i);
            }
            __syncthreads();
        }
        const StageDesc& st = P->st[uni(C.stage)];
        const double* zs = (const double*)smem;
        double* gvec = gbuf(P, b, uni(C.par));
        double mx[3] = {0.0, 0.0, 0.0};
        const int ntc = st.k1 / st.kt1;
        const int a0 = (c / ntc) * st.kt2, cb0 = (c % ntc) * st.kt1;
        const uint8_t* mask = P->mask + (size_t)b * K;
        // tile skipping: once few atoms remain, an item whose atoms are all screened is
        // not multiplied (its maxima are zero, its g is never read)
        if (uni(C.n_act) * 16 <= K) {
            int any = 0;
            const int per_col = st.kt2 >> 4;                 // 16-byte mask chunks per column j1
            for (int q = threadIdx.x; q < st.kt1 * per_col; q += kBlock) {
                // atoms (cb0 + q / per_col) k2 + a0 + 16 (q % per_col) .. + 15: 16 aligned mask bytes
                const uint4 mv = *(const uint4*)(mask + (size_t)(cb0 + q / per_col) * st.k2 + a0 + 16 * (q % per_col));
                any |= (mv.x | mv.y | mv.z | mv.w) != 0u;
            }
            if (!__syncthreads_or(any)) {
                put_wave_max(P, b, c, mx, false);
                continue;
            }
        }
        if (st.dtype == SL1_F64)
            kron_item_f64(st, a0, cb0, (const double*)smem, (double*)extra, mask, gvec, rz, mx);
        else if (st.dtype == SL1_F32)
            kron_item_f32(st, a0, cb0, (const float*)smem, (float*)extra, mask, gvec, rz, mx);
        else if (st.dtype == SL1_FP8_E4M3)
            kron_item_bf16<uint8_t>(st, a0, cb0, (const float*)smem, (uint16_t*)extra, mask, gvec, rz, mx);
        else
            kron_item_bf16<uint16_t>(st, a0, cb0, (const float*)smem, (uint16_t*)extra, mask, gvec, rz, mx);
        __syncthreads();       // every read of V precedes the next item's phase 1
        put_wave_max(P, b, c, mx, true);
    }
}

// ---------------------------------------------------------------------------
// FAuST correlations g_j = (S_J^T w)_j for every signal on a FAuST stage, w =
// S_{J-1}^T ... S_1^T z formed by the forward launch.  Block (tile, group, stage):
// the tile's kFaustAtoms atoms for up to faust_group(dl) signals on that stage, whose
// w vectors sit in LDS; each wave takes a quarter of the tile, four atoms at a time,
// lane = signal.  The four atoms' entries of S_J^T are loaded once per wave with
// coalesced loads (one per lane per atom, the next four atoms' loads issued before
// this group's products), staged in the wave's LDS slice, and every lane runs the
// four sums against its w, each atom's entries in order (as one signal's chain
// would sum them).  Atoms with more than 64 entries take a plain loop.  Only
// preserved atoms' g are written; each wave leaves its per-signal maxima in slot
// (tile, wave).  The factor entries are read once per tile and group of signals
// instead of once per signal.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void faust_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kBlock) void k_adj_faust(const SolveParams* __restrict__ P, int slot) {
    extern __shared__ __align__(16) char smem[];
    const int stage = blockIdx.z, tile = blockIdx.x, grp = blockIdx.y;
    if (stage >= P->n_stages) return;
    const StageDesc& st = P->st[stage];
    if (st.kind != kFaust || tile >= st.fa_items) return;
    const int K = P->K, batch = P->batch;
    const FaustDesc& F = *st.fa;
    const int dl = F.dim[F.J - 1];
    const int sg = faust_group(dl), ld = dl + 1;
    double* W = (double*)smem;
    int* s_sig = (int*)(smem + (size_t)sg * ld * 8);
    char* after_sig = smem + (size_t)sg * ld * 8 + (((size_t)batch + 1) * 4 + 15) / 16 * 16;
    int* s_par = (int*)after_sig;
    double* s_rz = (double*)(after_sig + 64 * 4 + 256);
    char* stage_base = after_sig + (size_t)64 * 16;
    __shared__ int s_tmp[16];
    // the signals on this stage, in signal order
    int run = 0;
    for (int base = 0; base < batch; base += kBlock) {
        const int b = base + threadIdx.x;
        const int f = (b < batch && P->cnt_adjf[b] == stage + 1) ? 1 : 0;
        int ex;
        const int tot = block_excl_scan(f, ex, s_tmp);
        if (f) s_sig[run + ex] = b;
        run += tot;
    }
    const int g0 = grp * sg, ng = min(sg, run - g0);
    if (ng <= 0) return;                      // block-uniform
    if ((int)threadIdx.x < ng) {
        const int b = s_sig[g0 + threadIdx.x];
        const Control& C = P->ctrl[2 * b + slot];
        double zz = 0.0;
        for (int k = 0; k < P->nrc; ++k) zz += P->res_part[((size_t)b * P->nrc + k) * 3 + 1];
        s_par[threadIdx.x] = C.par;
        s_rz[threadIdx.x] = dual_norm_z(P, st, b, zz);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // the group's w vectors: each wave copies every fourth signal's, eight loads in flight per lane
    for (int q0 = w; q0 < ng; q0 += 8) {
        const double* src0 = P->fw + (size_t)s_sig[g0 + q0] * kFaustMaxDim;
        const double* src1 = q0 + 4 < ng ? P->fw + (size_t)s_sig[g0 + q0 + 4] * kFaustMaxDim : nullptr;
        for (int i0 = 0; i0 < dl; i0 += 256) {
            double v0[4], v1[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + 64 * u + lane;
                v0[u] = i < dl ? src0[i] : 0.0;
                v1[u] = (src1 && i < dl) ? src1[i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i0 + 64 * u + lane;
                if (i < dl) {
                    W[(size_t)q0 * ld + i] = v0[u];
                    if (src1) W[(size_t)(q0 + 4) * ld + i] = v1[u];
                }
            }
        }
    }
    __syncthreads();
    const bool on = lane < ng;
    const int b = on ? s_sig[g0 + lane] : 0;
    const double rz = on ? s_rz[lane] : 0.0;
    double* gvec = gbuf(P, b, on ? s_par[lane] : 0);
    const uint8_t* mask = P->mask + (size_t)b * K;
    const int* tptr = F.tptr + F.tp[F.J - 1];
    const int* tidx = F.tidx + F.tz[F.J - 1];
    const long long vz = F.tz[F.J - 1];
    const double* wl = W + (size_t)(on ? lane : 0) * ld;
    int* sI = (int*)(stage_base + (size_t)w * kFaustStage);          // [4 atoms][64 entries]
    double* sV = (double*)(sI + 4 * 64);
    double mx[3] = {0.0, 0.0, 0.0};
    const int per = kFaustAtoms / 4;
    const int j0 = tile * kFaustAtoms + w * per, j1 = min(K, j0 + per);
    // entries of the first four atoms, one per lane and atom
    int e0[4], n[4];
    int iv[4];
    double vv[4];
    auto fetch = [&](int jb) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = jb + q;
            const bool ok = j < j1;
            e0[q] = ok ? tptr[j] : 0;
            n[q] = ok ? tptr[j + 1] - e0[q] : 0;
            const bool le = lane < n[q];
            iv[q] = le ? tidx[e0[q] + lane] : 0;
            vv[q] = le ? faust_val(F.tval, vz + e0[q] + lane, st.dtype) : 0.0;
        }
    };
    if (j0 < j1) fetch(j0);
    for (int jb = j0; jb < j1; jb += 4) {
        int cn[4], ce[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            cn[q] = n[q];
            ce[q] = e0[q];
            sI[q * 64 + lane] = iv[q];
            sV[q * 64 + lane] = vv[q];
        }
        faust_wave_sync();
        if (jb + 4 < j1) fetch(jb + 4);       // in flight during this group's sums
        const int nmax = max(max(cn[0], cn[1]), max(cn[2], cn[3]));
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (nmax <= 64) {
            for (int k = 0; k < nmax; ++k) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (k < cn[q]) acc[q] = fma(sV[q * 64 + k], wl[sI[q * 64 + k]], acc[q]);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                for (int k = 0; k < cn[q]; ++k)
                    acc[q] = fma(faust_val(F.tval, vz + ce[q] + k, st.dtype), wl[tidx[ce[q] + k]], acc[q]);
        }
        faust_wave_sync();                    // the slice is rewritten by the next group
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = jb + q;
            if (on && j < j1 && mask[j]) {
                gvec[j] = acc[q];
                const double ej = st.eps[j];
                mx[0] = fmax(mx[0], fabs(acc[q]) + ej * rz);
                mx[1] = fmax(mx[1], fabs(acc[q]));
                mx[2] = fmax(mx[2], ej);
            }
        }
    }
    if (on) {
        double* ap = P->adj_part + (((size_t)b * P->nadj_max + tile) * 4 + w) * 3;
        ap[0] = mx[0];
        ap[1] = mx[1];
        ap[2] = mx[2];
    }
}

// FP64 scalar block of iteration t from the per-block partials of the forward
// and correlation launches; computed identically by every block that needs it.
__device__ void scalar_block(const SolveParams* P, int b, const Control& C, Scalars& S, double* s_red) {
    const int nslots = C.nslot;
    double mx[3] = {0.0, 0.0, 0.0};
    // up to 8 slots per thread loaded together (one memory round trip per 8 blockDim slots)
    const double* a0 = P->adj_part + (size_t)b * P->nadj_max * 4 * 3;
    for (int base = 0; base < nslots; base += 8 * (int)blockDim.x) {
        double v[8][3];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = base + u * blockDim.x + threadIdx.x;
            const bool ok = k < nslots;
            const double* ap = a0 + (size_t)(ok ? k : 0) * 3;
            v[u][0] = ok ? ap[0] : 0.0;
            v[u][1] = ok ? ap[1] : 0.0;
            v[u][2] = ok ? ap[2] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            mx[0] = fmax(mx[0], v[u][0]);
            mx[1] = fmax(mx[1], v[u][1]);
            mx[2] = fmax(mx[2], v[u][2]);
        }
    }
    double r2, zz, yz;
    reduce_res_max(P, b, s_red, mx, r2, zz, yz);
    scalars_from(P, C, r2, zz, yz, dual_norm_z(P, P->st[C.stage], b, zz), mx[0], mx[1], mx[2],
                 P->rule ? P->yy[b] : 0.0, S);
}

// ---------------------------------------------------------------------------
// test + FISTA update + compaction (Table I stable GAP Safe row; Algorithm 1
// screening step; Section IV-C look-ahead count).  Item = segment of 256
// entries of the preserved set.
// ---------------------------------------------------------------------------
// NF flags of every thread of the block at once (one exchange of wave counts, two
// barriers): pos[f] = the number of threads before this one (in thread order) with
// flag f set, total[f] = the block's count.  s_w holds (blockDim.x / 64) * NF ints.
template <int NF>
__device__ __forceinline__ void block_scan_flags(const bool (&f)[NF], int* s_w, int (&pos)[NF], int (&total)[NF]) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        const unsigned long long bal = __ballot(f[k]);
        pos[k] = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) s_w[w * NF + k] = __popcll(bal);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NF; ++k) total[k] = 0;
    for (int q = 0; q < nw; ++q) {
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            const int c = s_w[q * NF + k];
            pos[k] += q < w ? c : 0;
            total[k] += c;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ int block_excl_scan_flag(bool f, int* s_w, int& total) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned long long bal = __ballot(f);
    const int pre = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) s_w[w] = __popcll(bal);
    __syncthreads();
    int base = 0;
    for (int k = 0; k < w; ++k) base += s_w[k];
    total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    __syncthreads();
    return base + pre;
}

// one body, two kernels: the dome rule's test lives in its own instantiation, so the
// other rules' update keeps its registers and occupancy
template <bool kDome>
__device__ __forceinline__ void upd_body(const SolveParams* __restrict__ P, int slot) {
    extern __shared__ __align__(16) char smem[];
    const int K = P->K, batch = P->batch;
    int* s_pre = (int*)smem;
    int* s_wpre = s_pre + (P->nseg_max + 1);
    __shared__ double s_red[96];
    __shared__ int s_w[8];           // four waves' counts of two flags
    __shared__ int s_tmp[16];
    const int total = build_work_map(P->cnt_upd, batch, s_wpre, s_tmp);
    const int per = (total + gridDim.x - 1) / gridDim.x;
    const int g0 = blockIdx.x * per, g1 = min(total, g0 + per);
    int cur_b = -1;
    Control C;
    // the scalars the per-atom test and step use, block-uniform (scalar registers)
    struct {
        double c1, c2, Rp, Rd, ny, beta;
        double sp, Rdl, dcut;         // GAP dome (rule 2)
        int conv;
    } U;
    for (int g = g0; g < g1; ++g) {
        const int b = uni(find_signal(s_wpre, batch, g));
        const int c = uni(g - s_wpre[b]);
        if (b != cur_b) {
            cur_b = b;
            C = P->ctrl[2 * b + slot];
            // the list prefixes are fetched before the scalar block, so that both
            // wait on the same memory round trip
            const int* ap = actpre(P, b, C.par);
            const int pv0 = (int)threadIdx.x <= C.nseg_act ? ap[threadIdx.x] : 0;
            Scalars S;
            scalar_block(P, b, C, S, s_red);
            // the block holding the signal's first item stores them (items of a
            // signal are consecutive, so item 0 is the first one a block meets)
            if (c == 0 && threadIdx.x == 0) {
                Scalars T = S;
                if (T.conv == 1) T.tconv = wall_clock64();
                P->sc[b] = T;
                P->cnt_fwd[(size_t)(1 - slot) * batch + b] = P->nrc;
            }
            U.c1 = uni(S.c1);
            U.c2 = uni(S.c2);
            U.Rp = uni(S.Rp);
            U.Rd = uni(S.Rd);
            U.ny = uni(S.ny);
            U.sp = uni(S.sp);
            U.Rdl = uni(S.Rdl);
            U.dcut = uni(S.dcut);
            U.beta = uni(S.beta);
            U.conv = uni(S.conv);
            if ((int)threadIdx.x <= C.nseg_act) s_pre[threadIdx.x] = pv0;
            for (int s = threadIdx.x + kBlock; s <= C.nseg_act; s += kBlock) s_pre[s] = ap[s];
            __syncthreads();
        }
        if (U.conv) continue;
        const int par = C.par, n_act = C.n_act;
        const StageDesc& st = P->st[C.stage];
        const int i = c * kSeg + threadIdx.x;
        const bool valid = i < n_act;
        int j = 0;
        bool keep = false, nzf = false;
        double kt = 0.0, l1 = 0.0, xnv = 0.0;
        if (valid) {
            j = list_get(actbuf(P, b, par), s_pre, C.nseg_act, i);
            double* xc = xbuf(P, b, par);
            double* xo = xbuf(P, b, 1 - par);
            const double gt = gbuf(P, b, par)[j];
            const double gp = gbuf(P, b, 1 - par)[j];
            const double xt = xc[j];
            const double xp = xo[j];
            const double e = st.eps[j];
            const double ag = fabs(gt);
            // sphere test of the rule and the look-ahead flag on the approximate atom
            const int rule = P->rule;
            const double cyj = rule ? P->cy[(size_t)b * K + j] : 0.0;
            const double eI = rule ? P->st[P->n_stages - 1].eps[j] * P->st[P->n_stages - 1].cq : 0.0;
            const double an = P->atom_norm[j], atn = st.at_norm[j];
            if (kDome) {
                // the stable GAP sphere and the GAP dome of theta'; the smaller test decides
                const double il = 1.0 / C.lam;
                const double cyv = cyj * il, sg = U.sp * gt;
                const double u = e * U.c2 + eI * U.ny * il;
                const double mu = fmin(U.c1 * ag + e * U.c2 + U.Rp * an, dome_test(cyv, sg, u, U.Rd, U.Rdl, U.dcut, an));
                const double mc = fmin(U.c1 * ag + U.Rp * atn, dome_test(cyv, sg, 0.0, U.Rd, U.Rdl, U.dcut, atn));
                kt = mc >= 1.0 ? 1.0 : 0.0;
                keep = mu >= 1.0 - P->margin;
            } else {
                keep = atom_test(rule, U, 1.0 / C.lam, U.Rp, ag, e, an, atn, fabs(cyj), eI, 1.0 - P->margin, kt);
            }
            if (C.iter % P->screen_every != 0) keep = true;    // rejections only every screen_every
            // FISTA (or ISTA: beta = 0) step on the preserved coefficients; the gradient at
            // the extrapolated point follows from the two correlation vectors by linearity
            const double beta = U.beta;
            const double zpt = xt + beta * (xt - xp);
            const double h = (1.0 + beta) * gt - beta * gp;
            const double v = zpt + h * st.invL;
            const double thr = C.lam * st.invL;
            double xn = 0.0;
            if (keep) xn = (v > thr) ? v - thr : ((v < -thr) ? v + thr : 0.0);
            xo[j] = xn;
            if (!keep) {
                xc[j] = 0.0;
                P->mask[(size_t)b * K + j] = 0;
                if (xt != 0.0) kt += kRejNz;
            }
            nzf = keep && (xn != 0.0);
            l1 = fabs(xn);
            xnv = xn;
        }
        const bool fl[2] = {keep, nzf};
        int ps[2], ts[2];
        block_scan_flags<2>(fl, s_w, ps, ts);
        const int pk = ps[0], pz = ps[1], tot_keep = ts[0], tot_nz = ts[1];
        if (keep) actbuf(P, b, 1 - par)[c * kSeg + pk] = j;
        if (nzf) {
            nzbuf(P, b, 1 - par)[c * kSeg + pz] = j;
            nzxbuf(P, b, 1 - par)[c * kSeg + pz] = xnv;
        }
        double sums[2] = {kt, l1};
        block_sum<2>(sums, s_red);
        if (threadIdx.x == 0) {
            double* up = P->upd_part + ((size_t)b * P->nseg_max + c) * 4;
            up[0] = (double)tot_keep;
            up[1] = (double)tot_nz;
            up[2] = sums[0];
            up[3] = sums[1];
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_upd(const SolveParams* __restrict__ P, int slot) {
    upd_body<false>(P, slot);
}

// the update of solves with the dome rule (SolveParams::rule == 2)
__global__ __launch_bounds__(kBlock, 5) void k_upd_dome(const SolveParams* __restrict__ P, int slot) {
    upd_body<true>(P, slot);
}

// ---------------------------------------------------------------------------
// Per-signal step on dense stages: the update of iteration t and the forward of
// iteration t + 1 in one block per signal (8 waves), so an iteration is this
// launch and the correlation launches.  The update launch's work (scalar block,
// stable GAP test, look-ahead count, FISTA step) and the switch decision are the
// same per-element expressions as in k_upd and the forward launch; the new lists
// are written contiguously (segment s of a list of n entries starts at
// min(kSeg s, n)), so their prefix counts need no cross-block pass.
//   reads  C_t from control slot 1 - slot (advance = 0: a fresh state, whose
//          forward alone runs), the correlation maxima and residual sums of t;
//   writes C_{t+1} with advance = 1 to slot `slot` (read by the correlation
//          launches of the same slot and by the next step launch), the residual
//          direction z and its sums, the correlation launches' item counts.
// Every stage a signal can reach here is dense (the host's condition for
// choosing this launch); no l_q bounds and no dome rule.
// ---------------------------------------------------------------------------
constexpr int kStepH = 4;            // preserved atoms per thread per pass of the update


__device__ __forceinline__ void step_finish(const SolveParams* P, int b, int slot, const Control& C, const Scalars& S,
                                            int status) {
    Final F;
    F.gap = S.Gt;
    F.gap_cert = S.Gp + S.delta;
    F.iters = C.iter;
    F.stage = C.stage;
    F.status = status;
    F.par = C.par;
    F.t0 = C.t0;
    F.tconv = S.conv == 1 ? wall_clock64() : 0;
    P->fin[b] = F;
    Control D = C;
    D.done = 1;
    D.advance = 0;
    P->ctrl[2 * b + slot] = D;
    P->cnt_adj[b] = 0;
    P->cnt_adjk[b] = 0;
    P->cnt_adjf[b] = 0;
    P->cnt_upd[b] = 0;
    P->cnt_gemm[b] = 0;
    *(int4*)(P->sig_stat + 4 * b) = make_int4(0, 0, 0, 0);
    atomicSub(P->active_signals, 1);
}

__global__ __launch_bounds__(kFwdBlock, 2) void k_step(const SolveParams* __restrict__ P, int slot) {
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.x, tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63;
    const int N = P->N, K = P->K, I = P->n_stages - 1;
    int* s_pre = (int*)smem;                                    // nseg_max + 1 prefix counts
    int* s_j = s_pre + ((P->nseg_max + 1 + 3) & ~3);            // staged nonzeros
    double* s_x = (double*)(((uintptr_t)(s_j + kFwdBlock) + 15) & ~(uintptr_t)15);
    double* s_u = s_x + kFwdBlock;                              // odd waves' row partials
    __shared__ Control s_c;
    __shared__ double s_red[96];
    __shared__ int s_tmp[16];
    __shared__ int s_flags[kFwdWaves * 2 * kStepH];
    if (P->absent[b]) return;     // its iterations run in a whole-solve launch meanwhile
    if (tid == 0) s_c = P->ctrl[2 * b + (1 - slot)];
    __syncthreads();
    Control C = s_c;
    if (C.done) {                 // stopped earlier: the record reaches this slot too
        if (tid == 0) P->ctrl[2 * b + slot] = C;
        return;
    }
    if (P->st[C.stage].kind != kDense) {   // outside this kernel's domain: refused
        if (tid == 0) {
            Scalars S = {};
            step_finish(P, b, slot, C, S, SL1_ELIMIT);
        }
        return;
    }
    const bool stepped = C.advance != 0;
    if (stepped) {
        // ---- scalar block of iteration t (the maxima of the correlation launch) ----
        Scalars S;
        scalar_block(P, b, C, S, s_red);
        if (S.conv) {
            if (tid == 0) step_finish(P, b, slot, C, S, S.conv == 2 ? SL1_MAXITER : SL1_OK);
            return;
        }
        const int par = C.par, n_act = C.n_act, nseg = C.nseg_act;
        const int* ap = actpre(P, b, par);
        for (int q = tid; q <= nseg; q += kFwdBlock) s_pre[q] = ap[q];
        __syncthreads();
        // ---- stable GAP test, look-ahead count, FISTA step, compaction ----
        const StageDesc& st = P->st[C.stage];
        const int* act = actbuf(P, b, par);
        int* nact = actbuf(P, b, 1 - par);
        int* nnz = nzbuf(P, b, 1 - par);
        double* nnx = nzxbuf(P, b, 1 - par);
        double* xc = xbuf(P, b, par);
        double* xo = xbuf(P, b, 1 - par);
        const double* gcur = gbuf(P, b, par);
        const double* gprev = gbuf(P, b, 1 - par);
        uint8_t* mask = P->mask + (size_t)b * K;
        const int rule = P->rule;
        const double invlam = uni(1.0 / C.lam), keep_min = 1.0 - P->margin;
        const double beta = uni(S.beta), invL = st.invL, thr = uni(C.lam * st.invL);
        const bool no_reject = C.iter % P->screen_every != 0;
        const double* eI = P->st[I].eps;
        const double cqI = P->st[I].cq;
        int wpos = 0, zpos = 0;
        double sv[2] = {0.0, 0.0};           // look-ahead count (+ rejected nonzeros), ||x_{t+1}||_1
        // a list of all K atoms is the identity (compactions keep the order); the
        // next pass's list entries are requested before this pass's atom data is used
        int jn[kStepH];
#pragma unroll
        for (int h = 0; h < kStepH; ++h) {
            const int i = h * kFwdBlock + tid;
            jn[h] = i < n_act ? (n_act == K ? i : list_get(act, s_pre, nseg, i)) : 0;
        }
        for (int base = 0; base < n_act; base += kStepH * kFwdBlock) {
            int jj[kStepH];
            bool keep[kStepH], nzf[kStepH];
            double xn[kStepH];
#pragma unroll
            for (int h = 0; h < kStepH; ++h) {
                jj[h] = jn[h];
                keep[h] = nzf[h] = false;
                xn[h] = 0.0;
            }
#pragma unroll
            for (int h = 0; h < kStepH; ++h) {
                const int i = base + kStepH * kFwdBlock + h * kFwdBlock + tid;
                jn[h] = i < n_act ? (n_act == K ? i : list_get(act, s_pre, nseg, i)) : 0;
            }
#pragma unroll
            for (int h = 0; h < kStepH; ++h) {
                const int i = base + h * kFwdBlock + tid;
                if (i < n_act) {
                    const int j = jj[h];
                    const double gt = gcur[j], gp = gprev[j], xt = xc[j], xp = xo[j];
                    const double e = st.eps[j], an = P->atom_norm[j], atn = st.at_norm[j];
                    const double cyj = rule ? P->cy[(size_t)b * K + j] : 0.0;
                    const double eIj = rule ? eI[j] * cqI : 0.0;
                    double kt = 0.0;
                    bool k = atom_test(rule, S, invlam, S.Rp, fabs(gt), e, an, atn, fabs(cyj), eIj, keep_min, kt);
                    if (no_reject) k = true;
                    const double zpt = xt + beta * (xt - xp);
                    const double hh = (1.0 + beta) * gt - beta * gp;
                    const double v = zpt + hh * invL;
                    double x1 = 0.0;
                    if (k) x1 = (v > thr) ? v - thr : ((v < -thr) ? v + thr : 0.0);
                    xo[j] = x1;
                    if (!k) {
                        xc[j] = 0.0;
                        mask[j] = 0;
                        if (xt != 0.0) kt += kRejNz;
                    }
                    sv[0] += kt;
                    sv[1] += fabs(x1);
                    keep[h] = k;
                    nzf[h] = k && x1 != 0.0;
                    xn[h] = x1;
                }
            }
            // positions in list order: the kept and the nonzero atoms of the pass's parts
            bool fl[2 * kStepH];
#pragma unroll
            for (int h = 0; h < kStepH; ++h) {
                fl[2 * h] = keep[h];
                fl[2 * h + 1] = nzf[h];
            }
            int ps[2 * kStepH], ts[2 * kStepH];
            block_scan_flags<2 * kStepH>(fl, s_flags, ps, ts);
#pragma unroll
            for (int h = 0; h < kStepH; ++h) {
                if (keep[h]) nact[wpos + ps[2 * h]] = jj[h];
                if (nzf[h]) {
                    const int q = zpos + ps[2 * h + 1];
                    nnz[q] = jj[h];
                    nnx[q] = xn[h];
                    if (q < kFwdBlock) {      // the forward's first staged chunk, kept in LDS
                        s_j[q] = jj[h];
                        s_x[q] = xn[h];
                    }
                }
                wpos += ts[2 * h];
                zpos += ts[2 * h + 1];
            }
        }
        block_sum<2>(sv, s_red);
        // ---- Algorithm 2 and the momentum sequence ----
        const double rnz = floor(sv[0] / kRejNz);     // rejected nonzero coefficients
        const double kt = sv[0] - rnz * kRejNz;
        const int i_new = switch_dictionary(C.stage, I, S.gamma, P->Gamma, kt, st.rc, (double)K);
        if (tid == 0 && P->trace && C.iter < P->trace_cap) {
            double* tr = P->trace + ((size_t)b * P->trace_cap + C.iter) * SL1_TRACE_FIELDS;
            tr[0] = C.iter; tr[1] = C.stage; tr[2] = C.n_act; tr[3] = wpos;
            tr[4] = kt;
            tr[5] = S.Gp; tr[6] = S.Gt; tr[7] = S.delta; tr[8] = rule ? S.Rd : S.Rp; tr[9] = S.gamma;
            tr[10] = C.l1; tr[11] = S.P; tr[12] = C.n_nz;
        }
        if (i_new != C.stage || rnz > 0.0) {   // a switch, or a rejection that zeroed x_t[j]: restart
            C.stage = i_new;
            C.ksince = 0;
            C.tau = 1.0;
        } else {
            C.ksince += 1;
            C.tau = S.tau_next;
        }
        C.iter += 1;
        C.par = 1 - par;
        C.n_act = wpos;
        C.n_nz = zpos;
        C.l1 = sv[1];
        C.nseg_act = max(1, (wpos + kSeg - 1) / kSeg);
        C.nseg_nz = (zpos + kSeg - 1) / kSeg;
        int* pa = actpre(P, b, C.par);
        int* pz = nzpre(P, b, C.par);
        for (int q = tid; q <= C.nseg_act; q += kFwdBlock) pa[q] = min(q * kSeg, wpos);
        for (int q = tid; q <= C.nseg_nz; q += kFwdBlock) pz[q] = min(q * kSeg, zpos);
        if (P->st[C.stage].kind != kDense) {   // a structured later stage: not this kernel's domain
            if (tid == 0) step_finish(P, b, slot, C, S, SL1_ELIMIT);
            return;
        }
    }
    // ---- forward of the (new) iteration: u = A~ x over the nonzero list, rho = y - u ----
    const StageDesc& st = P->st[C.stage];
    const int par = C.par, nnz = C.n_nz, nseg_nz = C.nseg_nz;
    __syncthreads();                       // s_pre: the update's reads are done
    if (stepped) {                         // the list this block just wrote is contiguous
        for (int q = tid; q <= nseg_nz; q += kFwdBlock) s_pre[q] = min(q * kSeg, nnz);
    } else {
        const int* zp = nzpre(P, b, par);
        for (int q = tid; q <= nseg_nz; q += kFwdBlock) s_pre[q] = zp[q];
    }
    __syncthreads();
    const int* nzi = nzbuf(P, b, par);
    const double* nzx = nzxbuf(P, b, par);
    const int sub = w >> 1, half = w & 1;
    for (int item = 0; item < P->nrc; ++item) {
        const int r0 = item * kFwdRows + sub * 256 + lane * 4;
        const bool rows_ok = r0 < N;
        double yv[4] = {0.0, 0.0, 0.0, 0.0};
        if (half == 0 && rows_ok) {
#pragma unroll
            for (int v = 0; v < 4; ++v) yv[v] = yval(P, b, r0 + v);
        }
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int base = 0; base < nnz; base += kFwdBlock) {
            const int cnt = min(kFwdBlock, nnz - base);
            // after an update a list of one chunk is already staged (and stays so for
            // every item); longer lists are staged chunk by chunk
            if (tid < cnt && !(stepped && nnz <= kFwdBlock)) {
                const int pos = list_pos(s_pre, nseg_nz, base + tid);
                s_j[tid] = nzi[pos];
                s_x[tid] = nzx[pos];
            }
            __syncthreads();
            const int ph = (cnt + 1) >> 1;
            const int k0 = half ? ph : 0, k1 = half ? cnt : ph;
            if (rows_ok && k0 < k1) {
                switch (st.dtype) {
                    case SL1_F64: fwd_dense_gather<SL1_F64, 4>(st, N, r0, s_j, s_x, k0, k1, acc); break;
                    case SL1_F32: fwd_dense_gather<SL1_F32, 8>(st, N, r0, s_j, s_x, k0, k1, acc); break;
                    case SL1_BF16: fwd_dense_gather<SL1_BF16, 8>(st, N, r0, s_j, s_x, k0, k1, acc); break;
                    default: fwd_dense_gather<SL1_FP8_E4M3, 8>(st, N, r0, s_j, s_x, k0, k1, acc); break;
                }
            }
            __syncthreads();
        }
        if (half == 1) {
#pragma unroll
            for (int v = 0; v < 4; ++v) s_u[sub * 256 + lane * 4 + v] = acc[v];
        }
        __syncthreads();
        double sums[3] = {0.0, 0.0, 0.0};
        if (half == 0 && rows_ok) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double rho = yv[v] - (acc[v] + s_u[sub * 256 + lane * 4 + v]);
                P->z[(size_t)b * N + r0 + v] = rho;
                sums[0] += rho * rho;
                sums[1] += rho * rho;
                sums[2] += yv[v] * rho;
            }
        }
        block_sum<3>(sums, s_red);        // its barriers also guard s_u for the next item
        if (tid == 0) {
            double* rp = P->res_part + ((size_t)b * P->nrc + item) * 3;
            rp[0] = sums[0];
            rp[1] = sums[1];
            rp[2] = sums[2];
        }
    }
    // ---- control record and item counts of this slot's correlation launches ----
    if (tid == 0) {
        const int items = adj_items(st, C.n_act, N);
        const bool qual = P->gemm_min > 0 && C.stage == I && C.n_act >= P->gemm_min;
        const bool gemm = qual && P->gemm_on;
        Control D = C;
        D.advance = 1;
        D.nslot = gemm ? 4 * ((K + kGemmAtoms - 1) / kGemmAtoms) : 4 * items;
        P->ctrl[2 * b + slot] = D;
        *(int4*)(P->sig_stat + 4 * b) = make_int4(C.n_act, C.n_act, C.stage < I ? 1 : 0, qual ? 1 : 0);
        P->cnt_adj[b] = gemm ? 0 : items;
        P->cnt_adjk[b] = 0;
        P->cnt_adjf[b] = 0;
        P->cnt_gemm[b] = gemm ? 1 : 0;
        P->cnt_upd[b] = 0;
    }
}

// warm start: x_0 = x_{-1} = x0 (device, batch x K), its nonzeros compacted in atom
// order into the nonzero list of slot 0 (contiguous, so segment s begins at
// min(256 s, n)), ||x_0||_1 into the control record.  One block per signal, after
// k_init; a non-finite entry makes the signal invalid.
__global__ __launch_bounds__(kBlock) void k_init_x0(const SolveParams* __restrict__ P, const double* __restrict__ x0) {
    const int b = blockIdx.x, K = P->K;
    __shared__ int s_w[4];
    __shared__ double s_red[48];
    __shared__ Control s_c;
    if (threadIdx.x == 0) s_c = P->ctrl[2 * b];
    __syncthreads();
    if (s_c.done) return;
    int* nzl = nzbuf(P, b, 0);
    double* nzv = nzxbuf(P, b, 0);
    double* xa = xbuf(P, b, 0);
    double* xb = xbuf(P, b, 1);
    int cnt = 0;
    double l1 = 0.0;
    bool bad = false;
    for (int base = 0; base < K; base += kBlock) {
        const int j = base + threadIdx.x;
        const double v = j < K ? x0[(size_t)b * K + j] : 0.0;
        bad |= !isfinite(v);
        if (j < K) {
            xa[j] = v;
            xb[j] = v;
        }
        const bool nz = v != 0.0;
        int tot;
        const int pos = block_excl_scan_flag(nz, s_w, tot);
        if (nz) {
            nzl[cnt + pos] = j;
            nzv[cnt + pos] = v;
        }
        cnt += tot;
        l1 += fabs(v);
    }
    double sums[2] = {l1, bad ? 1.0 : 0.0};
    block_sum<2>(sums, s_red);
    const int nseg = (cnt + kSeg - 1) / kSeg;
    int* zp = nzpre(P, b, 0);
    for (int s = threadIdx.x; s <= nseg; s += kBlock) zp[s] = min(s * kSeg, cnt);
    if (threadIdx.x == 0) {
        Control C = s_c;
        if (sums[1] != 0.0) {
            C.done = 1;
            C.status = SL1_EINVAL;
            P->fin[b].status = SL1_EINVAL;
            P->cnt_fwd[b] = 0;
            atomicSub(P->active_signals, 1);
        } else {
            C.n_nz = cnt;
            C.nseg_nz = nseg;
            C.l1 = sums[0];
        }
        P->ctrl[2 * b] = C;
        P->ctrl[2 * b + 1] = C;
    }
}

// statistics of the last forward launch, reduced over the batch once per chunk
// (max and sum of |A_t|, signals not on the last stage, signals qualifying for
// the batched correlation product); one block
__global__ __launch_bounds__(kBlock) void k_stat(const SolveParams* __restrict__ P) {
    __shared__ int s_v[4][kBlock / 64];
    int v[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < P->batch; b += kBlock) {
        const int4 q = *(const int4*)(P->sig_stat + 4 * b);
        v[0] = max(v[0], q.x);
        v[1] += q.y;
        v[2] += q.z;
        v[3] += q.w;
    }
    for (int o = 32; o > 0; o >>= 1) {
        v[0] = max(v[0], __shfl_xor(v[0], o));
        v[1] += __shfl_xor(v[1], o);
        v[2] += __shfl_xor(v[2], o);
        v[3] += __shfl_xor(v[3], o);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 4; ++k) s_v[k][w] = v[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        int a = s_v[k][0];
        for (int q = 1; q < kBlock / 64; ++q) a = k == 0 ? max(a, s_v[k][q]) : a + s_v[k][q];
        P->stat[k] = a;
    }
}

// ||y||^2 of every signal in FP64 (the stable Dynamic Safe radius)
__global__ __launch_bounds__(kBlock) void k_ysq(const SolveParams* __restrict__ P, double* yy) {
    __shared__ double s_red[48];
    const int b = blockIdx.x;
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < P->N; i += kBlock) {
        const double t = yval(P, b, i);
        v[0] = fma(t, t, v[0]);
    }
    block_sum<1>(v, s_red);
    if (threadIdx.x == 0) yy[b] = v[0];
}

// ---------------------------------------------------------------------------
// outputs
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_finalize(const SolveParams* __restrict__ P, double* x_out, double* gap,
                                                     double* gap_cert, uint8_t* screened, int32_t* iters,
                                                     int32_t* stage, int32_t* status) {
    const int b = blockIdx.y, c = blockIdx.x, K = P->K;
    const Final F = P->fin[b];
    const int j = c * kSeg + threadIdx.x;
    if (j < K) {
        x_out[(size_t)b * K + j] = xbuf(P, b, F.par)[j];
        if (screened) screened[(size_t)b * K + j] = P->mask[(size_t)b * K + j] ? 0 : 1;
    }
    if (c == 0 && threadIdx.x == 0) {
        gap[b] = F.gap;
        if (gap_cert) gap_cert[b] = F.gap_cert;
        if (iters) iters[b] = F.iters;
        if (stage) stage[b] = F.stage;
        status[b] = F.status;
    }
}

// lambda'_max after one forward/correlation pass from x = 0 (slot 0)
__global__ void k_lambda_out(const SolveParams* __restrict__ P, double* out, int32_t* status) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= P->batch) return;
    const Control& C = P->ctrl[2 * b];
    const StageDesc& st = P->st[0];
    const int nslots = 4 * adj_items(st, C.n_act, P->N);
    double mp = 0.0;
    for (int k = 0; k < nslots; ++k) mp = fmax(mp, P->adj_part[((size_t)b * P->nadj_max * 4 + k) * 3]);
    double r2 = 0.0, zz = 0.0, yz = 0.0;
    for (int k = 0; k < P->nrc; ++k) {
        const double* rp = P->res_part + ((size_t)b * P->nrc + k) * 3;
        r2 += rp[0];
        zz += rp[1];
        yz += rp[2];
    }
    // when z is a rounded copy of y (BF16 Kronecker stages) add the bound
    // ||y - z|| (max ||a~_j|| + max eps_j)
    const bool rounded = st.kind == kKron && (st.dtype == SL1_BF16 || st.dtype == SL1_FP8_E4M3);
    const bool rounded32 = st.kind == kKron && st.dtype == SL1_F32;
    const double d2 = (rounded || rounded32) ? fmax(0.0, r2 - 2.0 * yz + zz) : 0.0;
    out[b] = mp + sqrt(d2) * (st.at_norm_max + st.eps_max * st.cq);     // ||v||_{q*} <= cq ||v||
    status[b] = P->fin[b].status;
}

// correlations a~_j^T z of the lambda pass, all atoms (sl1_dict_adjoint)
__global__ void k_adjoint_out(const SolveParams* __restrict__ P, double* out, double* zout) {
    const int b = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < P->K) out[(size_t)b * P->K + j] = gbuf(P, b, 0)[j];
    if (zout && j < P->N) zout[(size_t)b * P->N + j] = P->z[(size_t)b * P->N + j];
}

__global__ void k_time_out(const SolveParams* __restrict__ P, long long* out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < P->batch) {
        out[2 * b] = P->fin[b].t0;
        out[2 * b + 1] = P->fin[b].tconv;
    }
}

// dense column norms and the rounding-enlarged error bounds (dictionary setup)
template <typename T>
__device__ __forceinline__ double decode_elem(const void* A, size_t idx);
template <> __device__ __forceinline__ double decode_elem<double>(const void* A, size_t idx) {
    return ((const double*)A)[idx];
}
template <> __device__ __forceinline__ double decode_elem<float>(const void* A, size_t idx) {
    return (double)((const float*)A)[idx];
}
template <> __device__ __forceinline__ double decode_elem<uint16_t>(const void* A, size_t idx) {
    return (double)bf16_to_f(((const uint16_t*)A)[idx]);
}
template <> __device__ __forceinline__ double decode_elem<uint8_t>(const void* A, size_t idx) {
    const uint32_t q = ((const uint8_t*)A)[idx];
    auto v = __builtin_amdgcn_cvt_pk_f32_fp8((int)q, false);
    return (double)v[0];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dense_norms(const void* A, const float* scale, int N, int K,
                                                        const double* eps_in, double kappa, double* at_norm,
                                                        double* eps_out, int* bad) {
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= K) return;
    double s = 0.0;
    for (int i = lane; i < N; i += 64) {
        const double v = decode_elem<T>(A, (size_t)j * N + i);
        s += v * v;
    }
    s = wave_sum(s);
    if (lane == 0) {
        const double sc = scale ? (double)scale[j] : 1.0;
        const double nrm = sqrt(s) * fabs(sc);
        at_norm[j] = nrm;
        const double e = eps_in[j];
        if (!(e >= 0.0) || !isfinite(e) || !isfinite(nrm)) atomicOr(bad, 1);
        eps_out[j] = e + kappa * nrm;
    }
}

__global__ void k_eps_fold(const double* eps_in, const double* absnorm, double kappa, int K, double* eps_out,
                           int* bad) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= K) return;
    const double e = eps_in[j];
    if (!(e >= 0.0) || !isfinite(e)) atomicOr(bad, 1);
    eps_out[j] = e + kappa * absnorm[j];
}

// ---------------------------------------------------------------------------
// host-side launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_init(const SolveParams* dP, const LaunchCfg& c, hipStream_t s) {
    hipLaunchKernelGGL(k_init, dim3(c.nseg_max, c.batch), dim3(kBlock), 0, s, dP);
    return hipGetLastError();
}

// kernels of one iteration: 0 forward, 1 dense correlations, 2 Kronecker
// correlations, 3 test/update; a correlation kernel with an empty grid (its
// stage kind is absent) is skipped
// ||z||_{q*} of each signal's stored direction for stages with l_q bounds, q != 2
// (Lemma 2, Lemma 1), right after the forward launch: one block per signal.  The
// largest entry M first, then M (sum_i (|z_i|/M)^{q*})^{1/q*} (q* = 1: the plain sum),
// widened by 2 gamma_n so that it bounds the exact norm (q = 1: M itself, exact).
__global__ __launch_bounds__(kBlock) void k_lq(const SolveParams* __restrict__ P, int slot) {
    const int b = blockIdx.x;
    const StageDesc& st = P->st[P->ctrl[2 * b + slot].stage];
    if (st.qmode == 0) return;
    __shared__ double s_red[16];
    const int N = P->N;
    const double* z = P->z + (size_t)b * N;
    double m[1] = {0.0};
    for (int i = threadIdx.x; i < N; i += kBlock) m[0] = fmax(m[0], fabs(z[i]));
    block_max<1>(m, s_red);
    const double M = m[0];
    double v = M;
    if (st.qmode != 2 && M > 0.0) {
        double t[1] = {0.0};
        for (int i = threadIdx.x; i < N; i += kBlock) {
            const double a = fabs(z[i]);
            t[0] += st.qmode == 3 ? a : pow(a / M, st.qd);
        }
        block_sum<1>(t, s_red);
        v = (st.qmode == 3 ? t[0] : M * pow(t[0], 1.0 / st.qd)) * (1.0 + 2.0 * fp64_slack(N));
    }
    if (threadIdx.x == 0) P->zq[b] = v;
}

hipError_t launch_one(int which, int slot, const SolveParams* dP, const LaunchCfg& c, hipStream_t s) {
    switch (which) {
        case 0:     // the forward, and the dual norms of solves with l_q bounds
            if (c.step) break;
            hipLaunchKernelGGL(k_fwd, dim3(c.g_fwd), dim3(kFwdBlock), c.lds_fwd, s, dP, slot);
            if (c.g_lq > 0) hipLaunchKernelGGL(k_lq, dim3(c.g_lq), dim3(kBlock), 0, s, dP, slot);
            break;
        case 1:
            if (c.g_adj > 0) hipLaunchKernelGGL(k_adj_dense, dim3(c.g_adj), dim3(kBlock), c.lds_adj, s, dP, slot);
            break;
        case 2:
            if (c.g_adjk > 0) hipLaunchKernelGGL(k_adj_kron, dim3(c.g_adjk), dim3(kBlock), c.lds_adjk, s, dP, slot);
            if (c.adjf_x > 0)
                hipLaunchKernelGGL(k_adj_faust, dim3(c.adjf_x, c.adjf_y, c.adjf_z), dim3(kBlock), c.lds_adjf, s, dP,
                                   slot);
            break;
        case 4:
            if (c.g_gemm > 0) hipLaunchKernelGGL(k_adj_gemm, dim3(c.g_gemm), dim3(kBlock), c.lds_gemm, s, dP, slot);
            break;
        case 5:     // finishes the tiles of a row-split product launch (right after it)
            if (c.g_gemm > 0) {
                const int gf = std::max(1, std::min(c.g_gemm / 2, kGemmSplitUnits));
                hipLaunchKernelGGL(k_gemm_fin, dim3(gf), dim3(kBlock), 4 * (2 * (size_t)c.batch + 1), s, dP, slot,
                                   c.g_gemm);
            }
            break;
        case 6:     // the update of the previous iteration and this one's forward, per signal
            if (c.step) hipLaunchKernelGGL(k_step, dim3(c.batch), dim3(kFwdBlock), c.lds_step, s, dP, slot);
            break;
        default:
            if (c.step) break;
            if (c.dome) hipLaunchKernelGGL(k_upd_dome, dim3(c.g_upd), dim3(kBlock), c.lds_upd, s, dP, slot);
            else hipLaunchKernelGGL(k_upd, dim3(c.g_upd), dim3(kBlock), c.lds_upd, s, dP, slot);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_iter(int slot, const SolveParams* dP, const LaunchCfg& c, hipStream_t s) {
    for (int q = 0; q < kGridKernels; ++q) {
        hipError_t e = launch_one(kIterOrder[q], slot, dP, c, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_adj_only(const SolveParams* dP, const LaunchCfg& c, hipStream_t s) {
    hipError_t e = launch_one(1, 0, dP, c, s);
    return e != hipSuccess ? e : launch_one(2, 0, dP, c, s);
}

hipError_t launch_fwd_adj(const SolveParams* dP, const LaunchCfg& c, hipStream_t s) {
    hipError_t e = launch_one(0, 0, dP, c, s);
    return e != hipSuccess ? e : launch_adj_only(dP, c, s);
}

hipError_t launch_finalize(const SolveParams* dP, const LaunchCfg& c, double* x, double* gap, double* gap_cert,
                           uint8_t* screened, int32_t* iters, int32_t* stage, int32_t* status, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(c.nseg_max, c.batch), dim3(kBlock), 0, s, dP, x, gap, gap_cert, screened,
                       iters, stage, status);
    return hipGetLastError();
}

hipError_t launch_lambda_out(const SolveParams* dP, int batch, double* out, int32_t* status, hipStream_t s) {
    hipLaunchKernelGGL(k_lambda_out, dim3((batch + 255) / 256), dim3(256), 0, s, dP, out, status);
    return hipGetLastError();
}

// the batched correlation kernel may use more than the default 64 KB of LDS
hipError_t adjk_lds_attr(size_t lds) {
    return hipFuncSetAttribute((const void*)k_adj_kron, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t adjf_lds_attr(size_t lds) {
    return hipFuncSetAttribute((const void*)k_adj_faust, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t fwd_lds_attr(size_t lds) {
    return hipFuncSetAttribute((const void*)k_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t gemm_lds_attr(size_t lds) {
    if (lds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute((const void*)k_adj_gemm, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// blocks of the update kernel resident at once on the current device (0 on error)
int adj_resident_blocks(size_t lds) {
    int n = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_adj_dense, kBlock, lds) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return n * cus;
}

int upd_resident_blocks(size_t lds) {
    int n = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_upd, kBlock, lds) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return n * cus;
}

// zero fill of n 32-bit words (a kernel rather than hipMemsetAsync, so that a caller
// may capture the calls that clear workspace memory)
__global__ __launch_bounds__(kBlock) void k_zero(uint32_t* __restrict__ p, size_t n) {
    const size_t stride = (size_t)gridDim.x * kBlock;
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    const int grid = (int)std::min<size_t>(2048, (n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_zero, dim3(grid), dim3(kBlock), 0, s, (uint32_t*)p, n);
    return hipGetLastError();
}

hipError_t launch_init_x0(const SolveParams* dP, int batch, const double* x0, hipStream_t s) {
    hipLaunchKernelGGL(k_init_x0, dim3(batch), dim3(kBlock), 0, s, dP, x0);
    return hipGetLastError();
}

hipError_t launch_stat(const SolveParams* dP, hipStream_t s) {
    hipLaunchKernelGGL(k_stat, dim3(1), dim3(kBlock), 0, s, dP);
    return hipGetLastError();
}

hipError_t launch_ysq(const SolveParams* dP, int batch, double* yy, hipStream_t s) {
    hipLaunchKernelGGL(k_ysq, dim3(batch), dim3(kBlock), 0, s, dP, yy);
    return hipGetLastError();
}

hipError_t launch_adjoint_out(const SolveParams* dP, int batch, int K, int N, double* out, double* zout,
                              hipStream_t s) {
    dim3 grid((std::max(K, N) + 255) / 256, batch);
    hipLaunchKernelGGL(k_adjoint_out, grid, dim3(256), 0, s, dP, out, zout);
    return hipGetLastError();
}

hipError_t launch_time_out(const SolveParams* dP, int batch, long long* out, hipStream_t s) {
    hipLaunchKernelGGL(k_time_out, dim3((batch + 255) / 256), dim3(256), 0, s, dP, out);
    return hipGetLastError();
}

hipError_t launch_dense_norms(int dtype, const void* A, const float* scale, int N, int K, const double* eps_in,
                              double kappa, double* at_norm, double* eps_out, int* bad, hipStream_t s) {
    dim3 grid((K + 3) / 4), block(kBlock);
    switch (dtype) {
        case SL1_F64: hipLaunchKernelGGL(k_dense_norms<double>, grid, block, 0, s, A, scale, N, K, eps_in, kappa, at_norm, eps_out, bad); break;
        case SL1_F32: hipLaunchKernelGGL(k_dense_norms<float>, grid, block, 0, s, A, scale, N, K, eps_in, kappa, at_norm, eps_out, bad); break;
        case SL1_BF16: hipLaunchKernelGGL(k_dense_norms<uint16_t>, grid, block, 0, s, A, scale, N, K, eps_in, kappa, at_norm, eps_out, bad); break;
        default: hipLaunchKernelGGL(k_dense_norms<uint8_t>, grid, block, 0, s, A, scale, N, K, eps_in, kappa, at_norm, eps_out, bad); break;
    }
    return hipGetLastError();
}

hipError_t launch_eps_fold(const double* eps_in, const double* absnorm, double kappa, int K, double* eps_out,
                           int* bad, hipStream_t s) {
    hipLaunchKernelGGL(k_eps_fold, dim3((K + 255) / 256), dim3(256), 0, s, eps_in, absnorm, kappa, K, eps_out, bad);
    return hipGetLastError();
}

}  // namespace sl1
