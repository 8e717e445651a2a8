// Device functions shared by the two solve engines (per-iteration grid kernels
// and the whole-solve workgroup kernel): workspace accessors, block
// reductions, BF16/FP8 decoding, the forward atom generation, the dense
// correlation streams and the FP64 scalar block.  Both engines compute every
// per-element quantity with these same expressions.
#pragma once
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

// block-uniform values (read from LDS or computed identically by every lane)
// moved to scalar registers, so that addresses derived from them are scalar
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename T>
__device__ __forceinline__ T* uni_ptr(T* p) {
    const unsigned long long u = (unsigned long long)p;
    const unsigned int lo = (unsigned int)__builtin_amdgcn_readfirstlane((int)(u & 0xFFFFFFFFull));
    const unsigned int hi = (unsigned int)__builtin_amdgcn_readfirstlane((int)(u >> 32));
    return (T*)(((unsigned long long)hi << 32) | lo);
}
// Full-wave reductions with DPP row operations, for code where all 64 lanes are active:
// prefix operations within each 16-lane row (shifts by 1, 2, 4, 8), then the row
// broadcasts of lanes 15 and 31, which leave the result in lane 63; every lane then
// reads it (uniform).  Lanes without a source contribute 0, so the max form is for
// non-negative values.
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ double dpp_move(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xFFFFFFFFll), CTRL, ROW_MASK, 0xF, BOUND);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, ROW_MASK, 0xF, BOUND);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane63(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xFFFFFFFFll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_sum_full(double v) {
    v += dpp_move<0x111, 0xF, true>(v);     // row_shr:1
    v += dpp_move<0x112, 0xF, true>(v);     // row_shr:2
    v += dpp_move<0x114, 0xF, true>(v);     // row_shr:4
    v += dpp_move<0x118, 0xF, true>(v);     // row_shr:8
    v += dpp_move<0x142, 0xA, false>(v);    // row_bcast:15 into rows 1, 3
    v += dpp_move<0x143, 0xC, false>(v);    // row_bcast:31 into rows 2, 3
    return lane63(v);
}
__device__ __forceinline__ double wave_max_nonneg_full(double v) {
    v = fmax(v, dpp_move<0x111, 0xF, true>(v));
    v = fmax(v, dpp_move<0x112, 0xF, true>(v));
    v = fmax(v, dpp_move<0x114, 0xF, true>(v));
    v = fmax(v, dpp_move<0x118, 0xF, true>(v));
    v = fmax(v, dpp_move<0x142, 0xA, false>(v));
    v = fmax(v, dpp_move<0x143, 0xC, false>(v));
    return lane63(v);
}
__device__ __forceinline__ double uni(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(u & 0xFFFFFFFFll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(u >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// workspace accessors (signal b, buffer parity par)
__device__ __forceinline__ double* xbuf(const SolveParams* P, int b, int par) {
    return P->x + ((size_t)b * 2 + par) * P->K;
}
// signal value y_b[i] (FP32 or FP64 input)
__device__ __forceinline__ double yval(const SolveParams* P, int b, int i) {
    const size_t k = (size_t)b * P->N + i;
    return P->y_f64 ? ((const double*)P->y)[k] : (double)((const float*)P->y)[k];
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
__device__ __forceinline__ double* nzxbuf(const SolveParams* P, int b, int par) {
    return P->nzx + ((size_t)b * 2 + par) * P->K;
}
__device__ __forceinline__ int* actpre(const SolveParams* P, int b, int par) {
    return P->act_pre + ((size_t)b * 2 + par) * (P->nseg_max + 1);
}
__device__ __forceinline__ int* nzpre(const SolveParams* P, int b, int par) {
    return P->nz_pre + ((size_t)b * 2 + par) * (P->nseg_max + 1);
}

// block-wide sums / maxima of NV values, fixed order (red: LDS, NV*16 doubles)
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (l == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[k * 16 + w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double a = 0.0;
        for (int q = 0; q < nw; ++q) a += red[k * 16 + q];
        v[k] = a;
    }
    __syncthreads();
}

template <int NV>
__device__ __forceinline__ void block_max(double (&v)[NV], double* red) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_max(v[k]);
    __syncthreads();
    if (l == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red[k * 16 + w] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double a = red[k * 16];
        for (int q = 1; q < nw; ++q) a = fmax(a, red[k * 16 + q]);
        v[k] = a;
    }
    __syncthreads();
}

// exclusive block-wide prefix of per-thread integer counts; returns the total
__device__ __forceinline__ int block_excl_scan(int v, int& excl, int* s_tmp /* LDS, 16 ints */) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    if (lane == 63) s_tmp[w] = incl;
    __syncthreads();
    int base = 0, total = 0;
    for (int q = 0; q < nw; ++q) {
        if (q < w) base += s_tmp[q];
        total += s_tmp[q];
    }
    excl = base + incl - v;
    __syncthreads();
    return total;
}

__device__ __forceinline__ float bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return __uint_as_float(u & 0xFFFF0000u);
}
__device__ __forceinline__ uint16_t bf16_bits(float f) {  // f already bf16-exact
    return (uint16_t)(__float_as_uint(f) >> 16);
}

// Algorithm 2 (SwitchDictionary): speed criterion first, then gap saturation.
__device__ __forceinline__ int switch_dictionary(int i, int I, double gamma, double Gamma, double K_t, double rc,
                                                 double K) {
    if (i >= I) return I;
    if (K_t <= rc * K) return I;
    if (gamma <= Gamma) return i + 1;
    return i;
}

// dense correlation items: atoms per wave (a wave then has 8 column loads in
// flight per pass at N <= 1024 and N <= 2048)

// a dictionary pointer as a global-memory pointer: its loads are global loads,
// counted by the vector-memory counter alone, so LDS reads issued while they are
// in flight can be waited for without waiting for them
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const void* p) {
    return (const __attribute__((address_space(1))) T*)p;
}

// forward product: adds x_j a~_j[r0..r0+3] (4 rows per lane); a Kronecker atom
// is generated from its factors, sum_r B_r[i1, j1] C_r[i2, j2] in storage precision
__device__ __forceinline__ void fwd_accumulate(const StageDesc& st, int N, int j, double xj, int r0,
                                               double (&acc)[4]) {
    if (st.kind == kDense) {
        const size_t off = (size_t)j * N + r0;
        if (st.dtype == SL1_F64) {
            const auto* p = gmem<f64v2>((const double*)st.A + off);
            f64v2 a = p[0], c = p[1];
            acc[0] += xj * a[0]; acc[1] += xj * a[1]; acc[2] += xj * c[0]; acc[3] += xj * c[1];
        } else if (st.dtype == SL1_F32) {
            f32v4 a = *gmem<f32v4>((const float*)st.A + off);
            acc[0] += xj * (double)a[0]; acc[1] += xj * (double)a[1];
            acc[2] += xj * (double)a[2]; acc[3] += xj * (double)a[3];
        } else if (st.dtype == SL1_BF16) {
            u16x4 a = *gmem<u16x4>((const uint16_t*)st.A + off);
            const double s = st.scale ? (double)st.scale[j] : 1.0;
            const double xs = xj * s;
            acc[0] += xs * (double)bf16_to_f(a[0]); acc[1] += xs * (double)bf16_to_f(a[1]);
            acc[2] += xs * (double)bf16_to_f(a[2]); acc[3] += xs * (double)bf16_to_f(a[3]);
        } else {
            const uint32_t q = *gmem<uint32_t>((const uint8_t*)st.A + off);
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

__device__ __forceinline__ double clip_scale(double s0, double m) {
    if (!(m > 0.0)) return s0;
    const double im = 1.0 / m;
    return fmin(fmax(s0, -im), im);
}

// four consecutive stored elements of a dense column, kept in storage form
// until use so that many loads fit in registers at once
template <int DT> struct Raw4;
template <> struct Raw4<SL1_F64> { f64v2 a, b; };
template <> struct Raw4<SL1_F32> { f32v4 a; };
template <> struct Raw4<SL1_BF16> { u16x4 a; };
template <> struct Raw4<SL1_FP8_E4M3> { uint32_t a; };

template <int DT>
__device__ __forceinline__ Raw4<DT> raw_load(const void* A, size_t idx) {
    Raw4<DT> r;
    if constexpr (DT == SL1_F64) {
        const auto* p = gmem<f64v2>((const double*)A + idx);
        r.a = p[0];
        r.b = p[1];
    } else if constexpr (DT == SL1_F32) {
        r.a = *gmem<f32v4>((const float*)A + idx);
    } else if constexpr (DT == SL1_BF16) {
        r.a = *gmem<u16x4>((const uint16_t*)A + idx);
    } else {
        r.a = *gmem<uint32_t>((const uint8_t*)A + idx);
    }
    return r;
}

// decoded values (exact in FP64)
template <int DT>
__device__ __forceinline__ void raw_get(const Raw4<DT>& r, double (&v)[4]) {
    if constexpr (DT == SL1_F64) {
        v[0] = r.a[0]; v[1] = r.a[1]; v[2] = r.b[0]; v[3] = r.b[1];
    } else if constexpr (DT == SL1_F32) {
        v[0] = r.a[0]; v[1] = r.a[1]; v[2] = r.a[2]; v[3] = r.a[3];
    } else if constexpr (DT == SL1_BF16) {
        v[0] = bf16_to_f(r.a[0]); v[1] = bf16_to_f(r.a[1]); v[2] = bf16_to_f(r.a[2]); v[3] = bf16_to_f(r.a[3]);
    } else {
        const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)r.a, false);
        const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)r.a, true);
        v[0] = lo[0]; v[1] = lo[1]; v[2] = hi[0]; v[3] = hi[1];
    }
}

// NA atoms per wave; each pass issues the loads of NK 256-element steps of all
// NA atoms before the first product (a step that starts past N is skipped; the
// lanes of a step that crosses N load a valid address and discard it).  Per lane
// the products are accumulated in increasing k, so NK changes only how many loads
// are in flight: about 12 KB of stored entries per wave and pass (between 1 and
// 12 steps), whatever the storage type, so that a column of up to 3072 entries
// takes one memory round trip.
template <int DT, int NA>
constexpr int dense_nk() {
    constexpr int es = DT == SL1_F64 ? 8 : (DT == SL1_F32 ? 4 : (DT == SL1_BF16 ? 2 : 1));
    constexpr int nk = 12288 / (NA * 256 * es);
    return nk < 1 ? 1 : (nk > 12 ? 12 : nk);
}

template <int DT, int NA, int NK = dense_nk<DT, NA>()>
__device__ __forceinline__ void dense_dots_t(const StageDesc& st, int N, const int (&js)[NA], const double* zs,
                                             int lane, double (&out)[NA]) {
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;
    for (int kb = 0; kb < N; kb += 256 * NK) {
        Raw4<DT> r[NA][NK];
#pragma unroll
        for (int s = 0; s < NK; ++s) {
            const int k = kb + 256 * s + 4 * lane;
            const int kc = k < N ? k : 0;
            if (kb + 256 * s < N) {
#pragma unroll
                for (int q = 0; q < NA; ++q) r[q][s] = raw_load<DT>(st.A, (size_t)js[q] * N + kc);
            }
        }
#pragma unroll
        for (int s = 0; s < NK; ++s) {
            const int k = kb + 256 * s + 4 * lane;
            if (k < N) {
                const double z0 = zs[k], z1 = zs[k + 1], z2 = zs[k + 2], z3 = zs[k + 3];
#pragma unroll
                for (int q = 0; q < NA; ++q) {
                    double a[4];
                    raw_get<DT>(r[q][s], a);
                    acc[q] += a[0] * z0 + a[1] * z1 + a[2] * z2 + a[3] * z3;
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        out[q] = wave_sum(acc[q]);
        if (st.scale) out[q] *= (double)st.scale[js[q]];
    }
}

template <int NA>
__device__ __forceinline__ void dense_dots(const StageDesc& st, int N, const int (&js)[NA], const double* zs, int lane,
                                           double (&out)[NA]) {
    switch (st.dtype) {
        case SL1_F64: dense_dots_t<SL1_F64, NA>(st, N, js, zs, lane, out); break;
        case SL1_F32: dense_dots_t<SL1_F32, NA>(st, N, js, zs, lane, out); break;
        case SL1_BF16: dense_dots_t<SL1_BF16, NA>(st, N, js, zs, lane, out); break;
        default: dense_dots_t<SL1_FP8_E4M3, NA>(st, N, js, zs, lane, out); break;
    }
}

// FP64 scalar block of iteration t from the residual sums and the maxima over A_t
// Rounding slack of an FP64 quantity formed from N-term sums: gamma_n with
// n = 2 (N + 8) (the dot-product bound n u / (1 - n u), u = 2^-53, doubled).
__device__ __forceinline__ double fp64_slack(int N) {
    const double nu = 2.0 * (double)(N + 8) * 0x1p-53;
    return nu / (1.0 - nu);
}

// ||z||_{q*} of the stored direction, the norm that the stage's l_q bounds pair with
// in the dual scaling and the test (Lemma 2, Lemma 1): sqrt(zz) for l2 bounds,
// otherwise the value the l_q launch stored for the iteration.
__device__ __forceinline__ double dual_norm_z(const SolveParams* P, const StageDesc& st, int b, double zz) {
    return st.qmode == 0 ? sqrt(zz) : P->zq[b];
}

// The parameters the scalar block reads (a loop over many iterations loads them once).
struct ScalarConsts {
    double tol, slack;                // stop tolerance, fp64_slack(N)
    int rule, ista, last_stage, max_iter;
};

__device__ __forceinline__ ScalarConsts scalar_consts(const SolveParams* P) {
    ScalarConsts k;
    k.tol = P->tol;
    k.slack = fp64_slack(P->N);
    k.rule = P->rule;
    k.ista = P->ista;
    k.last_stage = P->n_stages - 1;
    k.max_iter = P->max_iter;
    return k;
}

// zq = ||z||_{q*} for the stage's bound norm (sqrt(zz) for l2 bounds); E, the largest
// eps over A_t, is turned into the l2 column bound of Theorem 1 by the stage's cq.
__device__ __forceinline__ void scalars_core(const ScalarConsts& K, double cq, const Control& C, double r2, double zz,
                                             double yz, double zq, double mp, double mt, double E, double yy,
                                             Scalars& S) {
    const double lam = C.lam, l1 = C.l1;
    const double il = 1.0 / lam;                           // the one division by lambda
    E *= cq;
    const double s0 = zz > 0.0 ? (yz / zz) * il : 0.0;     // projection of y/lam on z
    const double sp = clip_scale(s0, mp);                  // stable dual point theta' (Lemma 2)
    const double stc = clip_scale(s0, mt);                 // conventional point on A~
    const double Pv = 0.5 * r2 + lam * l1;                 // P(x_t | A~)
    const double Gp = Pv - (lam * sp * yz - 0.5 * lam * lam * sp * sp * zz);
    const double Gt = Pv - (lam * stc * yz - 0.5 * lam * lam * stc * stc * zz);
    const double delta = sqrt(r2) * E * l1 + 0.5 * E * E * l1 * l1;     // Theorem 1, r = 1
    S.r2 = r2; S.zz = zz; S.yz = yz;
    S.mp = mp; S.mt = mt; S.E = E;
    S.sp = sp; S.st = stc;
    S.P = Pv; S.Gp = Gp; S.Gt = Gt; S.delta = delta;
    S.Rp = sqrt(2.0 * fmax(Gp, 0.0) + 2.0 * delta) * il;
    S.gamma = Gp > 0.0 ? Gt / Gp : 1.0;
    S.c1 = fabs(sp);
    S.c2 = fabs(sp) * zq;
    // stable Dynamic Safe sphere B(y/lambda, ||theta' - y/lambda||) (Table I): the
    // squared radius s'^2 ||z||^2 - 2 s' y^T z / lambda + ||y||^2 / lambda^2, widened by
    // the FP64 rounding of its sums, gamma (|s'| ||z|| + ||y|| / lambda)^2
    S.ny = sqrt(yy);
    {
        const double q = sp * sp * zz - 2.0 * sp * yz * il + yy * (il * il);
        const double a = fabs(sp) * sqrt(zz) + S.ny * il;
        S.Rd = sqrt(fmax(q, 0.0) + K.slack * a * a);
        S.Rdl = K.rule == 2 ? sqrt(fmax(q - K.slack * a * a, 0.0)) : 0.0;
    }
    // GAP dome of theta' (rule 2): the ball with diameter [theta', y/lambda] keeps theta*
    // (the projection of y/lambda), and weak duality with P(x|A) <= P(x|A~) + delta keeps
    // ||theta* - y/lambda||^2 >= rin2; the cut level 1 - 2 rin2 / Rd^2 grows with Rd and
    // falls with rin2, so the upper bound of Rd and a lower bound of rin2 (sums widened by
    // their FP64 rounding) keep the dome safe
    S.dcut = -1.0;
    if (K.rule == 2) {
        const double g = K.slack;
        const double rin2 = fmax(yy * (1.0 - g) - 2.0 * (Pv + delta) * (1.0 + g), 0.0) * (il * il);
        S.dcut = S.Rd > 0.0 ? fmin(1.0, fmax(-1.0, 1.0 - 2.0 * rin2 / (S.Rd * S.Rd))) : -1.0;
    }
    if (C.ksince == 0 || K.ista) {       // ISTA: no momentum (Section I-B)
        S.beta = 0.0;
        S.tau_next = C.tau;
    } else {
        const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * C.tau * C.tau));
        S.beta = (C.tau - 1.0) / tn;
        S.tau_next = tn;
    }
    const bool on_exact = C.stage == K.last_stage;
    S.conv = (on_exact && Gt < K.tol) ? 1 : (C.iter >= K.max_iter ? 2 : 0);
    S.pad0 = 0;
    S.tconv = 0;
}

__device__ __forceinline__ void scalars_from(const SolveParams* P, const Control& C, double r2, double zz, double yz,
                                             double zq, double mp, double mt, double E, double yy, Scalars& S) {
    scalars_core(scalar_consts(P), P->st[C.stage].cq, C, r2, zz, yz, zq, mp, mt, E, yy, S);
}

// Sphere test of one preserved atom (Table I) and its look-ahead flag (Section IV-C):
//   stable GAP Safe     |a~^T theta'| + eps ||theta'||_{q*} + R' ||a||   (rule 0)
//   stable Dynamic Safe |a^T y| / lambda + ||theta' - y/lambda|| ||a||  (rule 1), with
//                       a^T y formed once on the exact dictionary and widened by its
//                       rounding allowance eI ||y|| (eI: the exact stage's eps times its
//                       cq, since ||y||_{q*} <= cq ||y||)
// ag = |a~^T z|, Rg = the GAP radius to use, acy = |a^T y|, eI the exact stage's eps.
// SC: Scalars, or any record with the fields c1, c2, Rp, Rd, ny
template <typename SC>
__device__ __forceinline__ bool atom_test(int rule, const SC& S, double invlam, double Rg, double ag, double e,
                                          double an, double atn, double acy, double eI, double keep_min,
                                          double& kt) {
    if (rule) {
        const double c = acy * invlam;
        kt = (c + S.Rd * atn >= 1.0) ? 1.0 : 0.0;
        return c + eI * S.ny * invlam + S.Rd * an >= keep_min;
    }
    kt = (S.c1 * ag + S.Rp * atn >= 1.0) ? 1.0 : 0.0;
    return S.c1 * ag + e * S.c2 + Rg * an >= keep_min;
}

// sup {u^T v : ||v|| <= 1, n^T v <= d} for unit u, n with n^T u = t: 1 when the ball's
// maximiser meets the cut (t <= d), else the maximum on the cut circle
__device__ __forceinline__ double dome_cap(double d, double t) {
    t = fmin(1.0, fmax(-1.0, t));
    if (t <= d) return 1.0;
    return d * t + sqrt(fmax(1.0 - d * d, 0.0)) * sqrt(fmax(1.0 - t * t, 0.0));
}

// Upper bound of sup |a^T theta| over the zone's atoms (||a|| = alpha) and the GAP dome:
// cy = a^T y / lambda, sg = s' a~^T z, u = the zone and rounding allowance of both;
// a^T m lies within (cy + sg)/2 +- u/2 and Rd a^T n within (cy - sg) +- u, and the cap
// falls with a^T n, so its lowest value bounds the supremum (dividing a negative lowest
// value by the radius's lower bound, a positive one by its upper bound, errs low).
__device__ __forceinline__ double dome_test(double cy, double sg, double u, double Rd, double Rdl, double dcut,
                                            double alpha) {
    double best = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double sgn = k ? -1.0 : 1.0;
        double v = 0.5 * (sgn * (cy + sg) + u);
        if (Rd > 0.0) {
            const double num = sgn * (cy - sg) - u;
            const double den = (num >= 0.0 ? Rd : Rdl) * alpha;
            const double t = den > 0.0 ? num / den : -1.0;
            v += 0.5 * Rd * alpha * dome_cap(dcut, t);
        }
        best = k ? fmax(best, v) : v;
    }
    return best;
}

}  // namespace sl1
