// Per-iteration kernels of the stable-screening FISTA solver (gfx950).
//
// One iteration t of Algorithm 1 (FastL1) for every signal of a batch is three
// launches, each covering all signals (grid.y = signal):
//   k_fwd  forward product u = A~ x_t as a gather over the nonzeros of x_t,
//          residual rho = y - u and its norms (FP64), stored direction z.
//   k_adj  correlations g = A~^T z over the preserved set A_t (dense: one
//          wavefront streams one atom; Kronecker: MFMA tiles of
//          sum_r C_r^T P B_r), the maxima of the stable dual scaling, then the
//          scalar block: dual points, gaps, delta, the stable GAP radius, the
//          gap ratio and the stop decision (FP64).
//   k_upd  per-atom stable GAP test, look-ahead count, FISTA step with soft
//          thresholding, compaction of the preserved set and of the nonzeros
//          (wavefront ballot + prefix), then Algorithm 2 and momentum update.
// Reductions across blocks use the "last block" pattern: every block writes a
// partial, fences, and bumps a per-signal counter; the block that arrives last
// reduces the partials in a fixed order (deterministic) and resets the counter.
// No block ever waits for another, so no launch can hang.
#include <algorithm>

#include "sl1_internal.hpp"

namespace sl1 {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef float f32v4 __attribute__((ext_vector_type(4)));
typedef double f64v2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// workspace accessors
// ---------------------------------------------------------------------------
template <typename W>
__device__ __forceinline__ W* xbuf(const SolveParams* P, int b, int par) {
    return (W*)P->x + ((size_t)b * 2 + par) * P->K;
}
__device__ __forceinline__ double* gbuf(const SolveParams* P, int b, int par) {
    return P->g + ((size_t)b * 2 + par) * P->K;
}
__device__ __forceinline__ int* actbuf(const SolveParams* P, int b, int par) {
    return P->act + ((size_t)b * 2 + par) * P->K;
}
__device__ __forceinline__ int* nzbuf(const SolveParams* P, int b, int par) {
    return P->nz + ((size_t)b * 2 + par) * P->K;
}
__device__ __forceinline__ int* actpre(const SolveParams* P, int b, int par) {
    return P->act_pre + ((size_t)b * 2 + par) * (P->nseg_max + 1);
}
__device__ __forceinline__ int* nzpre(const SolveParams* P, int b, int par) {
    return P->nz_pre + ((size_t)b * 2 + par) * (P->nseg_max + 1);
}
__device__ __forceinline__ unsigned* ctr(const SolveParams* P, int b, int k) {
    return P->counters + (size_t)b * (P->nrc + 3) + k;
}

// Last-block arrival.  Every thread fences its own partial-result stores, the
// block synchronises, thread 0 increments the counter; the block that brings it
// to `expected` is the last one, resets it, and acquires before reading.
__device__ __forceinline__ bool arrive_last(unsigned* c, unsigned expected) {
    __shared__ int s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned prev = atomicAdd(c, 1u);
        s_last = (prev + 1 == expected);
        if (s_last) atomicExch(c, 0u);
    }
    __syncthreads();
    const bool last = s_last != 0;
    if (last) __threadfence();
    return last;
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red /* LDS, NV*4 */) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (l == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[k * 4 + w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = ((red[k * 4 + 0] + red[k * 4 + 1]) + red[k * 4 + 2]) + red[k * 4 + 3];
    __syncthreads();
}

template <int NV>
__device__ __forceinline__ void block_max(double (&v)[NV], double* red) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_max(v[k]);
    __syncthreads();
    if (l == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[k * 4 + w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k)
        v[k] = fmax(fmax(red[k * 4 + 0], red[k * 4 + 1]), fmax(red[k * 4 + 2], red[k * 4 + 3]));
    __syncthreads();
}

__device__ __forceinline__ void load_pre(int* s_pre, const int* pre, int nseg) {
    for (int s = threadIdx.x; s <= nseg; s += kBlock) s_pre[s] = pre[s];
    __syncthreads();
}

__device__ __forceinline__ float bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}
__device__ __forceinline__ uint16_t bf16_bits(float f) {  // f already bf16-exact
    return (uint16_t)(__float_as_uint(f) >> 16);
}

// ---------------------------------------------------------------------------
// initialisation: x_0 = 0, A_0 = {1..K}, stage 0 (Algorithm 1, Initialize)
// ---------------------------------------------------------------------------
template <typename W>
__global__ __launch_bounds__(kBlock) void k_init(const SolveParams* __restrict__ P) {
    const int b = blockIdx.y, c = blockIdx.x, K = P->K;
    const int j = c * kSeg + threadIdx.x;
    if (j < K) {
        xbuf<W>(P, b, 0)[j] = W(0);
        xbuf<W>(P, b, 1)[j] = W(0);
        gbuf(P, b, 0)[j] = 0.0;
        gbuf(P, b, 1)[j] = 0.0;
        P->mask[(size_t)b * K + j] = 1;
        actbuf(P, b, 0)[j] = j;
    }
    if (c != 0) return;
    const int nseg = (K + kSeg - 1) / kSeg;
    int* ap = actpre(P, b, 0);
    for (int s = threadIdx.x; s <= nseg; s += kBlock) ap[s] = min(s * kSeg, K);
    // validate the signal and lambda
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const W* y = (const W*)P->y + (size_t)b * P->N;
    int bad = 0;
    for (int i = threadIdx.x; i < P->N; i += kBlock) bad |= !isfinite((double)y[i]);
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double lam = P->lam ? P->lam[b] : 1.0;
        SigState* S = P->state + b;
        const bool ok = !s_bad && lam > 0.0 && isfinite(lam);
        S->stage = 0;
        S->iter = 0;
        S->done = ok ? 0 : 1;
        S->status = ok ? SL1_OK : SL1_EINVAL;
        S->ksince = 0;
        S->par = 0;
        S->n_act = K;
        S->n_nz = 0;
        S->nseg_act = nseg;
        S->nseg_nz = 0;
        S->conv = 0;
        S->Kt = K;
        S->n_keep = K;
        S->lam = lam;
        S->tau = 1.0;
        S->tau_next = 1.0;
        S->beta = 0.0;
        S->l1 = 0.0;
        S->r2 = S->zz = S->yz = 0.0;
        S->mp = S->mt = S->E = 0.0;
        S->sp = S->st = 0.0;
        S->P = S->Gp = S->Gt = S->delta = S->Rp = 0.0;
        S->gamma = 1.0;
        S->c1 = S->c2 = 0.0;
        S->t0 = wall_clock64();
        S->tconv = 0;
        nzpre(P, b, 0)[0] = 0;
        for (int k = 0; k < P->nrc + 3; ++k) *ctr(P, b, k) = 0u;
        if (ok) atomicAdd(P->active_signals, 1);
    }
}

// ---------------------------------------------------------------------------
// forward product + residual (Section III-C: rho~_t = y - A~ x_t)
// ---------------------------------------------------------------------------
template <typename W>
__device__ __forceinline__ void fwd_accumulate(const StageDesc& st, int N, int j, double xj, int r0,
                                               double (&acc)[4]) {
    if (st.kind == kDense) {
        const size_t off = (size_t)j * N + r0;
        if (st.dtype == SL1_F64) {
            const f64v2* p = (const f64v2*)((const double*)st.A + off);
            f64v2 a = p[0], c = p[1];
            acc[0] += xj * a[0]; acc[1] += xj * a[1]; acc[2] += xj * c[0]; acc[3] += xj * c[1];
        } else if (st.dtype == SL1_F32) {
            f32v4 a = *(const f32v4*)((const float*)st.A + off);
            acc[0] += xj * (double)a[0]; acc[1] += xj * (double)a[1];
            acc[2] += xj * (double)a[2]; acc[3] += xj * (double)a[3];
        } else if (st.dtype == SL1_BF16) {
            u16x4 a = *(const u16x4*)((const uint16_t*)st.A + off);
            const double s = st.scale ? (double)st.scale[j] : 1.0;
            const double xs = xj * s;
            acc[0] += xs * (double)bf16_to_f(a[0]); acc[1] += xs * (double)bf16_to_f(a[1]);
            acc[2] += xs * (double)bf16_to_f(a[2]); acc[3] += xs * (double)bf16_to_f(a[3]);
        } else {
            const uint32_t q = *(const uint32_t*)((const uint8_t*)st.A + off);
            const double s = st.scale ? (double)st.scale[j] : 1.0;
            const double xs = xj * s;
            auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)q, false);
            auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)q, true);
            acc[0] += xs * (double)lo[0]; acc[1] += xs * (double)lo[1];
            acc[2] += xs * (double)hi[0]; acc[3] += xs * (double)hi[1];
        }
    } else {
        // Kronecker atom generated on the fly: a~_j[i] = sum_r B_r[i1,j1] C_r[i2,j2]
        const int n1 = st.n1, k1 = st.k1, n2 = st.n2, k2 = st.k2;
        const int i1 = r0 / n2, i2 = r0 - i1 * n2;
        const int j1 = j / k2, j2 = j - j1 * k2;
        if (st.dtype == SL1_F64) {
            double a[4] = {0, 0, 0, 0};
            for (int r = 0; r < st.R; ++r) {
                const double bv = ((const double*)st.B)[((size_t)r * k1 + j1) * n1 + i1];
                const f64v2* cp = (const f64v2*)((const double*)st.C + ((size_t)r * k2 + j2) * n2 + i2);
                f64v2 c0 = cp[0], c1 = cp[1];
                a[0] += bv * c0[0]; a[1] += bv * c0[1]; a[2] += bv * c1[0]; a[3] += bv * c1[1];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] += xj * a[v];
        } else if (st.dtype == SL1_F32) {
            float a[4] = {0.f, 0.f, 0.f, 0.f};
            for (int r = 0; r < st.R; ++r) {
                const float bv = ((const float*)st.B)[((size_t)r * k1 + j1) * n1 + i1];
                f32v4 c = *(const f32v4*)((const float*)st.C + ((size_t)r * k2 + j2) * n2 + i2);
                a[0] = fmaf(bv, c[0], a[0]); a[1] = fmaf(bv, c[1], a[1]);
                a[2] = fmaf(bv, c[2], a[2]); a[3] = fmaf(bv, c[3], a[3]);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] += xj * (double)a[v];
        } else {
            float a[4] = {0.f, 0.f, 0.f, 0.f};
            for (int r = 0; r < st.R; ++r) {
                const float bv = bf16_to_f(((const uint16_t*)st.B)[((size_t)r * k1 + j1) * n1 + i1]);
                u16x4 c = *(const u16x4*)((const uint16_t*)st.C + ((size_t)r * k2 + j2) * n2 + i2);
                a[0] = fmaf(bv, bf16_to_f(c[0]), a[0]); a[1] = fmaf(bv, bf16_to_f(c[1]), a[1]);
                a[2] = fmaf(bv, bf16_to_f(c[2]), a[2]); a[3] = fmaf(bv, bf16_to_f(c[3]), a[3]);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] += xj * (double)a[v];
        }
    }
}

template <typename W>
__global__ __launch_bounds__(kBlock) void k_fwd(const SolveParams* __restrict__ P) {
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.y;
    SigState* S = P->state + b;
    if (S->done) return;
    const int N = P->N, nrc = P->nrc;
    const int rc = blockIdx.x % nrc, split = blockIdx.x / nrc;
    const int nnz = S->n_nz;
    int nsplit = (nnz + kFwdMinPerSplit - 1) / kFwdMinPerSplit;
    nsplit = max(1, min(kFwdSplits, nsplit));
    if (split >= nsplit) return;
    const int per = (nnz + nsplit - 1) / nsplit;
    const int i0 = min(nnz, split * per), i1 = min(nnz, i0 + per);
    const int par = S->par;
    const StageDesc& st = P->st[S->stage];

    int* s_pre = (int*)smem;
    int* s_j = s_pre + (P->nseg_max + 1);
    double* s_x = (double*)(((uintptr_t)(s_j + kBlock) + 15) & ~(uintptr_t)15);
    __shared__ double s_red[16];
    load_pre(s_pre, nzpre(P, b, par), S->nseg_nz);
    const int* nzi = nzbuf(P, b, par);
    const W* x = xbuf<W>(P, b, par);

    const int r0 = rc * kFwdRows + threadIdx.x * 4;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int base = i0; base < i1; base += kBlock) {
        const int cnt = min(kBlock, i1 - base);
        if ((int)threadIdx.x < cnt) {
            const int j = list_get(nzi, s_pre, S->nseg_nz, base + threadIdx.x);
            s_j[threadIdx.x] = j;
            s_x[threadIdx.x] = (double)x[j];
        }
        __syncthreads();
        if (r0 < N) {
            for (int k = 0; k < cnt; ++k) fwd_accumulate<W>(st, N, s_j[k], s_x[k], r0, acc);
        }
        __syncthreads();
    }
    double* part = P->fwd_part + ((size_t)b * kFwdSplits + split) * N;
    if (r0 < N) {
        f64v2* pp = (f64v2*)(part + r0);
        pp[0] = f64v2{acc[0], acc[1]};
        pp[1] = f64v2{acc[2], acc[3]};
    }
    if (!arrive_last(ctr(P, b, rc), (unsigned)nsplit)) return;

    // last block of this row chunk: rho = y - u, z = stored direction, partial sums
    const bool to_bf16 = (st.kind == kKron && st.dtype == SL1_BF16);
    double sums[3] = {0.0, 0.0, 0.0};
    if (r0 < N) {
        const W* y = (const W*)P->y + (size_t)b * N;
        W* z = (W*)P->z + (size_t)b * N;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double u = 0.0;
            for (int s = 0; s < nsplit; ++s) u += P->fwd_part[((size_t)b * kFwdSplits + s) * N + r0 + v];
            const double yv = (double)y[r0 + v];
            const double rho = yv - u;
            W zw = (W)rho;
            if (to_bf16) zw = (W)bf16_rne((float)rho);
            z[r0 + v] = zw;
            const double zd = (double)zw;
            sums[0] += rho * rho;
            sums[1] += zd * zd;
            sums[2] += yv * zd;
        }
    }
    block_sum<3>(sums, s_red);
    if (threadIdx.x == 0) {
        double* rp = P->res_part + ((size_t)b * nrc + rc) * 3;
        rp[0] = sums[0]; rp[1] = sums[1]; rp[2] = sums[2];
    }
    if (!arrive_last(ctr(P, b, nrc), (unsigned)nrc)) return;
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0, d = 0.0;
        for (int k = 0; k < nrc; ++k) {
            const double* rp = P->res_part + ((size_t)b * nrc + k) * 3;
            a += rp[0]; c += rp[1]; d += rp[2];
        }
        S->r2 = a;
        S->zz = c;
        S->yz = d;
    }
}

// ---------------------------------------------------------------------------
// adjoint: dense streaming correlations over the compacted preserved set
// ---------------------------------------------------------------------------
template <typename W>
__device__ __forceinline__ double dense_dot(const StageDesc& st, int N, int j, const W* zs, int lane) {
    double acc = 0.0;
    const size_t off = (size_t)j * N;
    if (st.dtype == SL1_F64) {
        const double* col = (const double*)st.A + off;
        for (int k = lane * 4; k < N; k += 256) {
            const f64v2* p = (const f64v2*)(col + k);
            f64v2 a = p[0], c = p[1];
            acc += a[0] * (double)zs[k] + a[1] * (double)zs[k + 1] + c[0] * (double)zs[k + 2] + c[1] * (double)zs[k + 3];
        }
    } else if (st.dtype == SL1_F32) {
        const float* col = (const float*)st.A + off;
#pragma unroll 4
        for (int k = lane * 4; k < N; k += 256) {
            f32v4 a = *(const f32v4*)(col + k);
            acc += (double)a[0] * (double)zs[k] + (double)a[1] * (double)zs[k + 1] +
                   (double)a[2] * (double)zs[k + 2] + (double)a[3] * (double)zs[k + 3];
        }
    } else if (st.dtype == SL1_BF16) {
        const uint16_t* col = (const uint16_t*)st.A + off;
        if (st.vec == 8) {
#pragma unroll 2
            for (int k = lane * 8; k < N; k += 512) {
                u16x8 a = *(const u16x8*)(col + k);
#pragma unroll
                for (int v = 0; v < 8; ++v) acc += (double)bf16_to_f(a[v]) * (double)zs[k + v];
            }
        } else {
            for (int k = lane * 4; k < N; k += 256) {
                u16x4 a = *(const u16x4*)(col + k);
#pragma unroll
                for (int v = 0; v < 4; ++v) acc += (double)bf16_to_f(a[v]) * (double)zs[k + v];
            }
        }
    } else {
        const uint8_t* col = (const uint8_t*)st.A + off;
        if (st.vec == 16) {
            for (int k = lane * 16; k < N; k += 1024) {
                u32x4 q = *(const u32x4*)(col + k);
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)q[w], false);
                    auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)q[w], true);
                    const int kk = k + 4 * w;
                    acc += (double)lo[0] * (double)zs[kk] + (double)lo[1] * (double)zs[kk + 1] +
                           (double)hi[0] * (double)zs[kk + 2] + (double)hi[1] * (double)zs[kk + 3];
                }
            }
        } else {
#pragma unroll 2
            for (int k = lane * 4; k < N; k += 256) {
                const uint32_t q = *(const uint32_t*)(col + k);
                auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)q, false);
                auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)q, true);
                acc += (double)lo[0] * (double)zs[k] + (double)lo[1] * (double)zs[k + 1] +
                       (double)hi[0] * (double)zs[k + 2] + (double)hi[1] * (double)zs[k + 3];
            }
        }
    }
    acc = wave_sum(acc);
    if (st.scale) acc *= (double)st.scale[j];
    return acc;
}

// ---------------------------------------------------------------------------
// adjoint: Kronecker tile G[a0:a0+16, cb0:cb0+64] = sum_r C_r^T P B_r with MFMA.
// MFMA 16x16 operand layout (wave64): lane l holds A[l%16][k], B[k][l%16] with
// k = l/16 (x4 shapes) or 4*(l/16)+v (x16 shapes); D[4*(l/16)+v][l%16].
// Wave w handles the terms r = w, w+4, ...; the four partial tiles are summed
// in LDS in a fixed order.
// ---------------------------------------------------------------------------
template <typename AccT>
struct KronLds {
    AccT* V;      // [4 waves][16][n1]
    AccT* red;    // [4 waves][16][64]
};

__device__ __forceinline__ void kron_tile_f32(const StageDesc& st, int a0, int cb0, const float* zs,
                                              float* Vall, f32x4 (&acc)[4]) {
    const int n1 = st.n1, k1 = st.k1, n2 = st.n2, k2 = st.k2, R = st.R;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    float* Vs = Vall + w * 16 * n1;
    const float* Bf = (const float*)st.B;
    const float* Cf = (const float*)st.C;
    const int rounds = (R + 3) >> 2;
    for (int rr = 0; rr < rounds; ++rr) {
        const int r = rr * 4 + w;
        if (r < R) {
            const float* Cr = Cf + (size_t)r * k2 * n2;
            for (int cb = 0; cb < n1; cb += 16) {
                f32x4 d = {0.f, 0.f, 0.f, 0.f};
                for (int k0 = 0; k0 < n2; k0 += 4) {
                    const float av = Cr[(size_t)(a0 + li) * n2 + k0 + lk];
                    const float bv = zs[(cb + li) * n2 + k0 + lk];
                    d = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, d, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) Vs[(4 * lk + v) * n1 + cb + li] = d[v];
            }
        }
        __syncthreads();
        if (r < R) {
            const float* Br = Bf + (size_t)r * k1 * n1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (cb0 + q * 16 < k1) {
                    const int j1 = cb0 + q * 16 + li;
                    for (int k0 = 0; k0 < n1; k0 += 4) {
                        const float av = Vs[li * n1 + k0 + lk];
                        const float bv = Br[(size_t)j1 * n1 + k0 + lk];
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[q], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void kron_tile_f64(const StageDesc& st, int a0, int cb0, const double* zs,
                                              double* Vall, f64x4 (&acc)[4]) {
    const int n1 = st.n1, k1 = st.k1, n2 = st.n2, k2 = st.k2, R = st.R;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    double* Vs = Vall + w * 16 * n1;
    const double* Bf = (const double*)st.B;
    const double* Cf = (const double*)st.C;
    const int rounds = (R + 3) >> 2;
    for (int rr = 0; rr < rounds; ++rr) {
        const int r = rr * 4 + w;
        if (r < R) {
            const double* Cr = Cf + (size_t)r * k2 * n2;
            for (int cb = 0; cb < n1; cb += 16) {
                f64x4 d = {0.0, 0.0, 0.0, 0.0};
                for (int k0 = 0; k0 < n2; k0 += 4) {
                    const double av = Cr[(size_t)(a0 + li) * n2 + k0 + lk];
                    const double bv = zs[(cb + li) * n2 + k0 + lk];
                    d = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, d, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) Vs[(4 * lk + v) * n1 + cb + li] = d[v];
            }
        }
        __syncthreads();
        if (r < R) {
            const double* Br = Bf + (size_t)r * k1 * n1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (cb0 + q * 16 < k1) {
                    const int j1 = cb0 + q * 16 + li;
                    for (int k0 = 0; k0 < n1; k0 += 4) {
                        const double av = Vs[li * n1 + k0 + lk];
                        const double bv = Br[(size_t)j1 * n1 + k0 + lk];
                        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// BF16 factors: P (the stored residual, bf16-exact) and C_r enter the first
// product exactly; the FP32 intermediate V is split into hi + lo BF16 parts so
// the second product loses at most 2^-16 |V| (folded into eps by the library).
__device__ __forceinline__ void kron_tile_bf16(const StageDesc& st, int a0, int cb0, const float* zs,
                                               uint16_t* Vall, f32x4 (&acc)[4]) {
    const int n1 = st.n1, k1 = st.k1, n2 = st.n2, k2 = st.k2, R = st.R;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    uint16_t* Vh = Vall + w * 32 * n1;      // hi part [16][n1]
    uint16_t* Vl = Vh + 16 * n1;            // lo part [16][n1]
    const uint16_t* Bf = (const uint16_t*)st.B;
    const uint16_t* Cf = (const uint16_t*)st.C;
    const int rounds = (R + 3) >> 2;
    for (int rr = 0; rr < rounds; ++rr) {
        const int r = rr * 4 + w;
        if (r < R) {
            const uint16_t* Cr = Cf + (size_t)r * k2 * n2;
            for (int cb = 0; cb < n1; cb += 16) {
                f32x4 d = {0.f, 0.f, 0.f, 0.f};
                for (int k0 = 0; k0 < n2; k0 += 16) {
                    const u16x4 av = *(const u16x4*)(Cr + (size_t)(a0 + li) * n2 + k0 + 4 * lk);
                    const float* zp = zs + (cb + li) * n2 + k0 + 4 * lk;
                    s16x4 a, bb;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        a[v] = (short)av[v];
                        bb[v] = (short)bf16_bits(zp[v]);
                    }
                    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, d, 0, 0, 0);
                }
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float hi = bf16_rne(d[v]);
                    const float lo = bf16_rne(d[v] - hi);
                    Vh[(4 * lk + v) * n1 + cb + li] = bf16_bits(hi);
                    Vl[(4 * lk + v) * n1 + cb + li] = bf16_bits(lo);
                }
            }
        }
        __syncthreads();
        if (r < R) {
            const uint16_t* Br = Bf + (size_t)r * k1 * n1;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (cb0 + q * 16 < k1) {
                    const int j1 = cb0 + q * 16 + li;
                    for (int k0 = 0; k0 < n1; k0 += 16) {
                        const u16x4 hv = *(const u16x4*)(Vh + li * n1 + k0 + 4 * lk);
                        const u16x4 lv = *(const u16x4*)(Vl + li * n1 + k0 + 4 * lk);
                        const u16x4 bv = *(const u16x4*)(Br + (size_t)j1 * n1 + k0 + 4 * lk);
                        s16x4 h, lo, bb;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            h[v] = (short)hv[v];
                            lo[v] = (short)lv[v];
                            bb[v] = (short)bv[v];
                        }
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(h, bb, acc[q], 0, 0, 0);
                        acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lo, bb, acc[q], 0, 0, 0);
                    }
                }
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ double clip_scale(double s0, double m) {
    if (!(m > 0.0)) return s0;
    return fmin(fmax(s0, -1.0 / m), 1.0 / m);
}

template <typename W>
__global__ __launch_bounds__(kBlock) void k_adj(const SolveParams* __restrict__ P) {
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.y;
    SigState* S = P->state + b;
    if (S->done) return;
    const int N = P->N, K = P->K;
    const StageDesc& st = P->st[S->stage];
    const int n_act = S->n_act, par = S->par;
    const int c = blockIdx.x;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double rz = sqrt(S->zz);

    int nitems;
    if (st.kind == kDense) nitems = max(1, (n_act + kAdjAtoms - 1) / kAdjAtoms);
    else nitems = (st.k2 / 16) * ((st.k1 + kKronColTile - 1) / kKronColTile);
    if (c >= nitems) return;

    W* zs = (W*)smem;
    const size_t zbytes = ((size_t)N * sizeof(W) + 15) & ~(size_t)15;
    int* s_pre = (int*)(smem + zbytes);
    char* extra = smem + zbytes + (((size_t)(P->nseg_max + 1) * 4 + 15) & ~(size_t)15);
    __shared__ double s_red[16];

    const W* zg = (const W*)P->z + (size_t)b * N;
    for (int i = threadIdx.x * 4; i < N; i += kBlock * 4) {
#pragma unroll
        for (int v = 0; v < 4; ++v) zs[i + v] = zg[i + v];
    }
    double* g = gbuf(P, b, par);
    double mx[3] = {0.0, 0.0, 0.0};   // max(|g|+eps*|z|), max|g|, max eps over A_t

    if (st.kind == kDense) {
        load_pre(s_pre, actpre(P, b, par), S->nseg_act);   // includes __syncthreads (z ready)
        const int* act = actbuf(P, b, par);
        const int first = c * kAdjAtoms + w * (kAdjAtoms / 4);
        const int last = min(n_act, first + kAdjAtoms / 4);
        for (int i = first; i < last; ++i) {
            const int j = list_get(act, s_pre, S->nseg_act, i);
            const double gj = dense_dot<W>(st, N, j, zs, lane);
            if (lane == 0) {
                g[j] = gj;
                const double e = st.eps[j];
                mx[0] = fmax(mx[0], fabs(gj) + e * rz);
                mx[1] = fmax(mx[1], fabs(gj));
                mx[2] = fmax(mx[2], e);
            }
        }
    } else {
        __syncthreads();
        const int ntc = (st.k1 + kKronColTile - 1) / kKronColTile;
        const int a0 = (c / ntc) * 16, cb0 = (c % ntc) * kKronColTile;
        const int li = lane & 15, lk = lane >> 4;
        const uint8_t* mask = P->mask + (size_t)b * K;
        if (st.dtype == SL1_F64) {
            double* Vall = (double*)extra;
            double* red = Vall + 4 * 16 * P->n1_max;
            f64x4 acc[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = f64x4{0.0, 0.0, 0.0, 0.0};
            kron_tile_f64(st, a0, cb0, (const double*)zs, Vall, acc);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v) red[(w * 16 + 4 * lk + v) * 64 + q * 16 + li] = acc[q][v];
            __syncthreads();
            for (int o = threadIdx.x; o < 16 * 64; o += kBlock) {
                const int i = o >> 6, col = o & 63;
                if (cb0 + col < st.k1) {
                    const double s = ((red[(0 * 16 + i) * 64 + col] + red[(1 * 16 + i) * 64 + col]) +
                                      red[(2 * 16 + i) * 64 + col]) + red[(3 * 16 + i) * 64 + col];
                    const int j = (cb0 + col) * st.k2 + a0 + i;
                    g[j] = s;
                    if (mask[j]) {
                        const double e = st.eps[j];
                        mx[0] = fmax(mx[0], fabs(s) + e * rz);
                        mx[1] = fmax(mx[1], fabs(s));
                        mx[2] = fmax(mx[2], e);
                    }
                }
            }
        } else {
            float* red = (float*)extra;
            char* vspace = extra + 4 * 16 * 64 * sizeof(float);
            f32x4 acc[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (st.dtype == SL1_F32) kron_tile_f32(st, a0, cb0, (const float*)zs, (float*)vspace, acc);
            else kron_tile_bf16(st, a0, cb0, (const float*)zs, (uint16_t*)vspace, acc);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v) red[(w * 16 + 4 * lk + v) * 64 + q * 16 + li] = acc[q][v];
            __syncthreads();
            for (int o = threadIdx.x; o < 16 * 64; o += kBlock) {
                const int i = o >> 6, col = o & 63;
                if (cb0 + col < st.k1) {
                    const double s = (((double)red[(0 * 16 + i) * 64 + col] + (double)red[(1 * 16 + i) * 64 + col]) +
                                      (double)red[(2 * 16 + i) * 64 + col]) + (double)red[(3 * 16 + i) * 64 + col];
                    const int j = (cb0 + col) * st.k2 + a0 + i;
                    g[j] = s;
                    if (mask[j]) {
                        const double e = st.eps[j];
                        mx[0] = fmax(mx[0], fabs(s) + e * rz);
                        mx[1] = fmax(mx[1], fabs(s));
                        mx[2] = fmax(mx[2], e);
                    }
                }
            }
        }
    }
    block_max<3>(mx, s_red);
    if (threadIdx.x == 0) {
        double* ap = P->adj_part + ((size_t)b * P->nadj_max + c) * 3;
        ap[0] = mx[0]; ap[1] = mx[1]; ap[2] = mx[2];
    }
    if (!arrive_last(ctr(P, b, P->nrc + 1), (unsigned)nitems)) return;
    if (threadIdx.x != 0) return;

    // ---- scalar block (FP64): Section III-C, Theorem 1, Section IV-A
    double mp = 0.0, mt = 0.0, E = 0.0;
    for (int k = 0; k < nitems; ++k) {
        const double* ap = P->adj_part + ((size_t)b * P->nadj_max + k) * 3;
        mp = fmax(mp, ap[0]); mt = fmax(mt, ap[1]); E = fmax(E, ap[2]);
    }
    const double lam = S->lam, r2 = S->r2, zz = S->zz, yz = S->yz, l1 = S->l1;
    const double s0 = zz > 0.0 ? yz / (lam * zz) : 0.0;      // projection of y/lam on z
    const double sp = clip_scale(s0, mp);                   // stable dual point theta'
    const double stc = clip_scale(s0, mt);                  // conventional point on A~
    const double Pv = 0.5 * r2 + lam * l1;                  // P(x_t | A~)
    const double Gp = Pv - (lam * sp * yz - 0.5 * lam * lam * sp * sp * zz);
    const double Gt = Pv - (lam * stc * yz - 0.5 * lam * lam * stc * stc * zz);
    const double delta = sqrt(r2) * E * l1 + 0.5 * E * E * l1 * l1;
    const double Rp = sqrt(2.0 * fmax(Gp, 0.0) + 2.0 * delta) / lam;
    S->mp = mp; S->mt = mt; S->E = E;
    S->sp = sp; S->st = stc;
    S->P = Pv; S->Gp = Gp; S->Gt = Gt; S->delta = delta; S->Rp = Rp;
    S->gamma = Gp > 0.0 ? Gt / Gp : 1.0;
    S->c1 = fabs(sp);
    S->c2 = fabs(sp) * sqrt(zz);
    if (S->ksince == 0) {
        S->beta = 0.0;
        S->tau_next = S->tau;
    } else {
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * S->tau * S->tau));
        S->beta = (S->tau - 1.0) / tn;
        S->tau_next = tn;
    }
    const bool on_exact = S->stage == P->n_stages - 1;
    int stop = 0;
    if (on_exact && Gt < P->tol) stop = 1;
    else if (S->iter >= P->max_iter) stop = 2;
    if (P->lambda_only) stop = 3;
    S->conv = stop;
    if (stop == 1) S->tconv = wall_clock64();
}

// ---------------------------------------------------------------------------
// test + FISTA update + compaction (Table I stable GAP Safe row; Algorithm 1
// screening step; Section IV-C look-ahead; Algorithm 2)
// ---------------------------------------------------------------------------
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

template <typename W>
__global__ __launch_bounds__(kBlock) void k_upd(const SolveParams* __restrict__ P) {
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.y;
    SigState* S = P->state + b;
    if (S->done) return;
    const int c = blockIdx.x;
    if (S->conv) {
        if (c == 0 && threadIdx.x == 0) {
            S->done = 1;
            if (S->conv == 2) S->status = SL1_MAXITER;
            atomicSub(P->active_signals, 1);
        }
        return;
    }
    const int K = P->K, n_act = S->n_act, par = S->par;
    const int nblk = max(1, (n_act + kSeg - 1) / kSeg);
    if (c >= nblk) return;
    const StageDesc& st = P->st[S->stage];
    int* s_pre = (int*)smem;
    __shared__ int s_w[4];
    __shared__ double s_red[16];
    load_pre(s_pre, actpre(P, b, par), S->nseg_act);

    const int i = c * kSeg + threadIdx.x;
    const bool valid = i < n_act;
    int j = 0;
    bool keep = false, nzf = false;
    double kt = 0.0, l1 = 0.0;
    if (valid) {
        j = list_get(actbuf(P, b, par), s_pre, S->nseg_act, i);
        W* xc = xbuf<W>(P, b, par);
        W* xo = xbuf<W>(P, b, 1 - par);
        const double gt = gbuf(P, b, par)[j];
        const double gp = gbuf(P, b, 1 - par)[j];
        const double xt = (double)xc[j];
        const double xp = (double)xo[j];
        const double e = st.eps[j];
        const double ag = fabs(gt);
        // stable GAP Safe test: |a~^T theta'| + eps ||theta'|| + R' ||a||
        const double mu = S->c1 * ag + e * S->c2 + S->Rp * P->atom_norm[j];
        keep = mu >= 1.0 - P->margin;
        // look-ahead: conventional test on the approximate atom
        kt = (S->c1 * ag + S->Rp * st.at_norm[j] >= 1.0) ? 1.0 : 0.0;
        // FISTA step on the preserved coefficients
        const double beta = S->beta;
        const double zpt = xt + beta * (xt - xp);
        const double h = (1.0 + beta) * gt - beta * gp;
        const double v = zpt + h * st.invL;
        const double thr = S->lam * st.invL;
        double xn = 0.0;
        if (keep) xn = (v > thr) ? v - thr : ((v < -thr) ? v + thr : 0.0);
        const W xw = (W)xn;
        xo[j] = xw;
        if (!keep) {
            xc[j] = W(0);
            P->mask[(size_t)b * K + j] = 0;
        }
        nzf = keep && (xw != W(0));
        l1 = fabs((double)xw);
    }
    int tot_keep, tot_nz;
    const int pk = block_excl_scan_flag(keep, s_w, tot_keep);
    if (keep) actbuf(P, b, 1 - par)[c * kSeg + pk] = j;
    const int pz = block_excl_scan_flag(nzf, s_w, tot_nz);
    if (nzf) nzbuf(P, b, 1 - par)[c * kSeg + pz] = j;
    double sums[2] = {kt, l1};
    block_sum<2>(sums, s_red);
    if (threadIdx.x == 0) {
        double* up = P->upd_part + ((size_t)b * P->nseg_max + c) * 4;
        up[0] = (double)tot_keep; up[1] = (double)tot_nz; up[2] = sums[0]; up[3] = sums[1];
    }
    if (!arrive_last(ctr(P, b, P->nrc + 2), (unsigned)nblk)) return;

    // ---- last block: prefix counts of the new segments, then Algorithm 2
    int* apn = actpre(P, b, 1 - par);
    int* zpn = nzpre(P, b, 1 - par);
    if (threadIdx.x == 0) {
        int ak = 0, az = 0;
        double kts = 0.0, l1s = 0.0;
        for (int k = 0; k < nblk; ++k) {
            const double* up = P->upd_part + ((size_t)b * P->nseg_max + k) * 4;
            apn[k] = ak; zpn[k] = az;
            ak += (int)up[0]; az += (int)up[1];
            kts += up[2]; l1s += up[3];
        }
        apn[nblk] = ak; zpn[nblk] = az;
        const int t = S->iter;
        if (P->trace && t < P->trace_cap) {
            double* tr = P->trace + ((size_t)b * P->trace_cap + t) * SL1_TRACE_FIELDS;
            tr[0] = t; tr[1] = S->stage; tr[2] = n_act; tr[3] = ak; tr[4] = kts;
            tr[5] = S->Gp; tr[6] = S->Gt; tr[7] = S->delta; tr[8] = S->Rp; tr[9] = S->gamma;
            tr[10] = S->l1; tr[11] = S->P;
        }
        // Algorithm 2 (SwitchDictionary)
        const int I = P->n_stages - 1;
        int i_new = S->stage;
        if (S->stage < I) {
            if (kts <= st.rc * (double)K) i_new = I;            // speed criterion
            else if (S->gamma <= P->Gamma) i_new = S->stage + 1; // convergence criterion
        }
        if (i_new != S->stage) {
            S->stage = i_new;
            S->ksince = 0;
            S->tau = 1.0;
        } else {
            S->ksince += 1;
            S->tau = S->tau_next;
        }
        S->Kt = (int)kts;
        S->n_keep = ak;
        S->n_act = ak;
        S->n_nz = az;
        S->nseg_act = nblk;
        S->nseg_nz = nblk;
        S->l1 = l1s;
        S->iter = t + 1;
        S->par = 1 - par;
    }
}

// ---------------------------------------------------------------------------
// outputs
// ---------------------------------------------------------------------------
template <typename W>
__global__ __launch_bounds__(kBlock) void k_finalize(const SolveParams* __restrict__ P, W* x_out, double* gap,
                                                     double* gap_cert, uint8_t* screened, int32_t* iters,
                                                     int32_t* stage, int32_t* status) {
    const int b = blockIdx.y, c = blockIdx.x, K = P->K;
    const SigState* S = P->state + b;
    const int j = c * kSeg + threadIdx.x;
    if (j < K) {
        x_out[(size_t)b * K + j] = xbuf<W>(P, b, S->par)[j];
        if (screened) screened[(size_t)b * K + j] = P->mask[(size_t)b * K + j] ? 0 : 1;
    }
    if (c == 0 && threadIdx.x == 0) {
        gap[b] = S->Gt;
        if (gap_cert) gap_cert[b] = S->Gp + S->delta;
        if (iters) iters[b] = S->iter;
        if (stage) stage[b] = S->stage;
        status[b] = S->status;
    }
}

__global__ void k_lambda_out(const SolveParams* __restrict__ P, double* out, int32_t* status) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < P->batch) {
        // lambda'_max of the stored direction z; when z is a rounded copy of y
        // (BF16 Kronecker stages), add the bound ||y - z|| (max ||a~_j|| + max eps_j).
        const SigState& S = P->state[b];
        const StageDesc& st = P->st[0];
        const double d2 = fmax(0.0, S.r2 - 2.0 * S.yz + S.zz);
        out[b] = S.mp + sqrt(d2) * (st.at_norm_max + st.eps_max);
        status[b] = S.status;
    }
}

// correlations a~_j^T z of the lambda-mode pass, all atoms (sl1_dict_adjoint)
template <typename W>
__global__ void k_adjoint_out(const SolveParams* __restrict__ P, double* out, W* zout) {
    const int b = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < P->K) out[(size_t)b * P->K + j] = gbuf(P, b, 0)[j];
    if (zout && j < P->N) zout[(size_t)b * P->N + j] = ((const W*)P->z)[(size_t)b * P->N + j];
}

__global__ void k_time_out(const SolveParams* __restrict__ P, long long* out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < P->batch) {
        out[2 * b] = P->state[b].t0;
        out[2 * b + 1] = P->state[b].tconv;
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

template <typename W>
static hipError_t launch_iter_t(const SolveParams* dP, const LaunchCfg& c, hipStream_t s) {
    hipLaunchKernelGGL(k_fwd<W>, dim3(c.nrc * kFwdSplits, c.batch), dim3(kBlock), c.lds_fwd, s, dP);
    hipLaunchKernelGGL(k_adj<W>, dim3(c.nadj_max, c.batch), dim3(kBlock), c.lds_adj, s, dP);
    hipLaunchKernelGGL(k_upd<W>, dim3(c.nseg_max, c.batch), dim3(kBlock), c.lds_upd, s, dP);
    return hipGetLastError();
}

hipError_t launch_init(const SolveParams* dP, const LaunchCfg& c, bool f64, hipStream_t s) {
    if (f64) hipLaunchKernelGGL(k_init<double>, dim3(c.nseg_max, c.batch), dim3(kBlock), 0, s, dP);
    else hipLaunchKernelGGL(k_init<float>, dim3(c.nseg_max, c.batch), dim3(kBlock), 0, s, dP);
    return hipGetLastError();
}

hipError_t launch_iter(const SolveParams* dP, const LaunchCfg& c, bool f64, hipStream_t s) {
    return f64 ? launch_iter_t<double>(dP, c, s) : launch_iter_t<float>(dP, c, s);
}

hipError_t launch_fwd_adj(const SolveParams* dP, const LaunchCfg& c, bool f64, hipStream_t s) {
    if (f64) {
        hipLaunchKernelGGL(k_fwd<double>, dim3(c.nrc * kFwdSplits, c.batch), dim3(kBlock), c.lds_fwd, s, dP);
        hipLaunchKernelGGL(k_adj<double>, dim3(c.nadj_max, c.batch), dim3(kBlock), c.lds_adj, s, dP);
    } else {
        hipLaunchKernelGGL(k_fwd<float>, dim3(c.nrc * kFwdSplits, c.batch), dim3(kBlock), c.lds_fwd, s, dP);
        hipLaunchKernelGGL(k_adj<float>, dim3(c.nadj_max, c.batch), dim3(kBlock), c.lds_adj, s, dP);
    }
    return hipGetLastError();
}

hipError_t launch_adj_only(const SolveParams* dP, const LaunchCfg& c, bool f64, hipStream_t s) {
    if (f64) hipLaunchKernelGGL(k_adj<double>, dim3(c.nadj_max, c.batch), dim3(kBlock), c.lds_adj, s, dP);
    else hipLaunchKernelGGL(k_adj<float>, dim3(c.nadj_max, c.batch), dim3(kBlock), c.lds_adj, s, dP);
    return hipGetLastError();
}

hipError_t launch_finalize(const SolveParams* dP, const LaunchCfg& c, bool f64, void* x, double* gap,
                           double* gap_cert, uint8_t* screened, int32_t* iters, int32_t* stage,
                           int32_t* status, hipStream_t s) {
    if (f64)
        hipLaunchKernelGGL(k_finalize<double>, dim3(c.nseg_max, c.batch), dim3(kBlock), 0, s, dP, (double*)x,
                           gap, gap_cert, screened, iters, stage, status);
    else
        hipLaunchKernelGGL(k_finalize<float>, dim3(c.nseg_max, c.batch), dim3(kBlock), 0, s, dP, (float*)x,
                           gap, gap_cert, screened, iters, stage, status);
    return hipGetLastError();
}

hipError_t launch_lambda_out(const SolveParams* dP, int batch, double* out, int32_t* status, hipStream_t s) {
    hipLaunchKernelGGL(k_lambda_out, dim3((batch + 255) / 256), dim3(256), 0, s, dP, out, status);
    return hipGetLastError();
}

hipError_t launch_adjoint_out(const SolveParams* dP, int batch, int K, int N, bool f64, double* out, void* zout,
                              hipStream_t s) {
    dim3 grid((std::max(K, N) + 255) / 256, batch);
    if (f64) hipLaunchKernelGGL(k_adjoint_out<double>, grid, dim3(256), 0, s, dP, out, (double*)zout);
    else hipLaunchKernelGGL(k_adjoint_out<float>, grid, dim3(256), 0, s, dP, out, (float*)zout);
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
