// Whole-solve engine (gfx950): one workgroup of 8 waves runs Algorithm 1
// (FastL1) for one signal from the first iteration to the stop, with no host
// round trip and no kernel boundary between iterations.  Meant for batches of
// small problems (the per-signal vectors fit in LDS and the Kronecker factors of
// the current stage are copied into LDS once per stage switch).
//
// Iteration t, inside the workgroup (every barrier is block-wide):
//   forward    u = A~ x_t over the nonzeros of x_t (Kronecker atoms generated
//              from the LDS factors; dense columns streamed from HBM), the 8
//              waves split the nonzeros and their row partials are summed in a
//              fixed tree; residual rho = y - u, its norms, stored direction z.
//   correlate  g = A~^T z: dense stages over the preserved list (8 waves x 4
//              atoms in flight); Kronecker stages as two MFMA products
//              V_r = C_r^T Z then G = sum_r V_r B_r with every operand in LDS.
//   scalars    maxima over A_t, then the FP64 scalar block (shared expressions
//              with the per-iteration grid kernels): dual points, gaps, delta,
//              stable radius, gap ratio, stop decision.
//   update     stable GAP Safe test, look-ahead count, FISTA step, in-place
//              compaction of the preserved list and rebuild of the nonzero list.
//   switch     Algorithm 2 and the momentum sequence.
// Per-element arithmetic is the same as in the grid kernels; only the order of
// the FP64 reductions differs.  A launch runs at most a given number of
// iterations and stores its state, so every launch has bounded duration; the
// host relaunches while signals remain.
#include "sl1_device.hpp"

namespace sl1 {

namespace {

__device__ __forceinline__ size_t al16(size_t x) { return (x + 15) & ~(size_t)15; }


// exclusive prefix of a per-thread flag over the 8-wave block; total returned in `total`
// NF flags of every thread at once (one exchange of wave counts, two barriers):
// pos[f] = the number of threads before this one (in thread order) with flag f
// set, total[f] = the block's count of flag f.  s_w holds kWgWaves * NF ints.
template <int NF>
__device__ __forceinline__ void wg_scan_flags(const bool (&f)[NF], int* s_w, int (&pos)[NF], int (&total)[NF]) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        const unsigned long long bal = __ballot(f[k]);
        pos[k] = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) s_w[w * NF + k] = __popcll(bal);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NF; ++k) total[k] = 0;
#pragma unroll
    for (int q = 0; q < kWgWaves; ++q) {
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            const int c = s_w[q * NF + k];
            pos[k] += q < w ? c : 0;
            total[k] += c;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Kronecker forward product: a lane holds the 4 x 4 block of rows i1 = 4 ba + e / 4,
// i2 = 4 bc + e % 4 (block chunk 64 + lane), so that one LDS vector of B_r and
// one of C_r serve 16 products; staged nonzeros carry (j1 << 16) | j2.
// ---------------------------------------------------------------------------
template <int DT>
__device__ __forceinline__ void wg_kron_fwd(const char* fac, const StageDesc& st, int jp, double xj, int ba, int bc,
                                            double (&acc)[16]) {
    const int R = st.R, n1 = st.n1, k1 = st.k1, n2 = st.n2, k2 = st.k2;
    const int j1 = jp >> 16, j2 = jp & 0xFFFF;
    if constexpr (DT == SL1_F64) {
        // two passes of 8 rows keep the FP64 partial products within budget
        const double* Bl = (const double*)fac;
        const double* Cl = Bl + (size_t)R * k1 * n1;
#pragma unroll
        for (int ph = 0; ph < 2; ++ph) {
            double a[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) a[e] = 0.0;
            for (int r = 0; r < R; ++r) {
                const f64v2 b2 = *(const f64v2*)(Bl + ((size_t)r * k1 + j1) * n1 + 4 * ba + 2 * ph);
                const double* cp = Cl + ((size_t)r * k2 + j2) * n2 + 4 * bc;
                const f64v2 c01 = *(const f64v2*)cp, c23 = *(const f64v2*)(cp + 2);
                const double cv[4] = {c01[0], c01[1], c23[0], c23[1]};
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int q = 0; q < 4; ++q) a[p * 4 + q] += b2[p] * cv[q];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[8 * ph + e] += xj * a[e];
        }
    } else {
        float a[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) a[e] = 0.f;
        for (int r = 0; r < R; ++r) {
            float bv[4], cv[4];
            if constexpr (DT == SL1_F32) {
                const float* Bl = (const float*)fac;
                const float* Cl = Bl + (size_t)R * k1 * n1;
                const f32v4 b4 = *(const f32v4*)(Bl + ((size_t)r * k1 + j1) * n1 + 4 * ba);
                const f32v4 c4 = *(const f32v4*)(Cl + ((size_t)r * k2 + j2) * n2 + 4 * bc);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    bv[v] = b4[v];
                    cv[v] = c4[v];
                }
            } else {
                const uint16_t* Bl = (const uint16_t*)fac;
                const uint16_t* Cl = Bl + (size_t)R * k1 * n1;
                const u16x4 b4 = *(const u16x4*)(Bl + ((size_t)r * k1 + j1) * n1 + 4 * ba);
                const u16x4 c4 = *(const u16x4*)(Cl + ((size_t)r * k2 + j2) * n2 + 4 * bc);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    bv[v] = bf16_to_f(b4[v]);
                    cv[v] = bf16_to_f(c4[v]);
                }
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) a[p * 4 + q] = fmaf(bv[p], cv[q], a[p * 4 + q]);
        }
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[e] += xj * (double)a[e];
    }
}

// accumulate this wave's share [k0, k1) of the staged nonzeros of a Kronecker
// stage (entries (j1 << 16) | j2); D64: FP64 factors, else FP32 or BF16
template <bool D64>
__device__ __forceinline__ void wg_kron_range(const StageDesc& st, const char* fac, int ba, int bc, bool kvalid,
                                              const int* s_j, const double* s_x, int k0, int k1, double (&acc)[16]) {
    if (!kvalid) return;
    if constexpr (D64) {
#pragma unroll 1
        for (int k = k0; k < k1; ++k) wg_kron_fwd<SL1_F64>(fac, st, s_j[k], s_x[k], ba, bc, acc);
    } else if (st.dtype == SL1_F32) {
#pragma unroll 1
        for (int k = k0; k < k1; ++k) wg_kron_fwd<SL1_F32>(fac, st, s_j[k], s_x[k], ba, bc, acc);
    } else {
#pragma unroll 1
        for (int k = k0; k < k1; ++k) wg_kron_fwd<SL1_BF16>(fac, st, s_j[k], s_x[k], ba, bc, acc);
    }
}

// sum of the 8 waves' row partials into wave 0, fixed order; scr: 32 KB
__device__ __forceinline__ void wg_reduce_rows(double (&acc)[16], double* scr) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int half = kWgWaves / 2; half >= 1; half >>= 1) {
        if (w >= half && w < 2 * half) {
#pragma unroll
            for (int e = 0; e < 16; ++e) scr[((w - half) * 16 + e) * 64 + lane] = acc[e];
        }
        __syncthreads();
        if (w < half) {
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[e] += scr[(w * 16 + e) * 64 + lane];
        }
        __syncthreads();
    }
}

// signal value y[row] (from LDS when it is held there)
__device__ __forceinline__ double wg_y(const SolveParams* P, int b, const double* yl, int row) {
    return yl ? yl[row] : yval(P, b, row);
}

// Kronecker forward product, residual, stored direction z (LDS) and the FP64
// sums ||rho||^2, ||z||^2, y^T z (into s_sum).  The 8 waves split the staged
// nonzeros; a lane holds a 4 x 4 block of rows (one LDS vector of B_r and one of
// C_r serve 16 products) and the partials meet in a fixed tree.
template <bool D64>
__device__ __forceinline__ void wg_kron_forward(const SolveParams* P, int b, const StageDesc& st, const char* fac,
                                                const double* x, const int* nzl, int n_nz, const int* lj,
                                                const double* lx, bool in_lds, int zround, double* zd,
                                                float* zf, const double* yl, char* scr, double* s_red,
                                                double* s_sum) {
    const int N = P->N, tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int nchunk = (N + kWgRows - 1) / kWgRows;
    const int k2 = st.k2;
    double* s_x = (double*)scr;                                   // staging shares the scratch
    int* s_j = (int*)(scr + kWgStage * 8);
    double sums[3] = {0.0, 0.0, 0.0};
    for (int chunk = 0; chunk < nchunk; ++chunk) {
        const int q = chunk * 64 + lane, nb2 = st.n2 >> 2;
        const bool kvalid = q < (N >> 4);
        const int ba = kvalid ? q / nb2 : 0;
        const int bc = kvalid ? q - ba * nb2 : 0;
        const int rbase = 4 * ba * st.n2 + 4 * bc;
        double acc[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[e] = 0.0;
        for (int base = 0; base < n_nz; base += kWgStage) {
            const int cnt = min(kWgStage, n_nz - base);
            if (tid < cnt) {
                // the LDS copy of the nonzero list (atoms and values) when it holds them
                const int j = in_lds ? lj[base + tid] : nzl[base + tid];
                const int j1 = j / k2;
                s_j[tid] = (j1 << 16) | (j - j1 * k2);
                s_x[tid] = in_lds ? lx[base + tid] : x[j];
            }
            __syncthreads();
            const int pw = (cnt + kWgWaves - 1) / kWgWaves;
            const int k0 = min(cnt, w * pw), k1 = min(cnt, k0 + pw);
            wg_kron_range<D64>(st, fac, ba, bc, kvalid, s_j, s_x, k0, k1, acc);
            __syncthreads();
        }
        wg_reduce_rows(acc, (double*)scr);
        if (w == 0 && kvalid) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = rbase + (e >> 2) * st.n2 + (e & 3);
                const double yv = wg_y(P, b, yl, row);
                const double rho = yv - acc[e];
                double zv = rho;
                if (zround == 1) zv = (double)(float)rho;
                else if (zround == 2) zv = (double)bf16_rne((float)rho);
                zd[row] = zv;
                zf[row] = (float)zv;
                sums[0] += rho * rho;
                sums[1] += zv * zv;
                sums[2] += yv * zv;
            }
        }
    }
    block_sum<3>(sums, s_red);
    if (tid == 0) {
        s_sum[0] = sums[0];
        s_sum[1] = sums[1];
        s_sum[2] = sums[2];
    }
}

// four consecutive elements of a dense column in FP32/BF16/FP8 storage, decoded
// to float (exact); FP64 storage is handled separately
__device__ __forceinline__ f32v4 dense4_f(int dtype, const void* A, size_t idx) {
    f32v4 r;
    if (dtype == SL1_F32) {
        r = *gmem<f32v4>((const float*)A + idx);
    } else if (dtype == SL1_BF16) {
        const u16x4 a = *gmem<u16x4>((const uint16_t*)A + idx);
        r = f32v4{bf16_to_f(a[0]), bf16_to_f(a[1]), bf16_to_f(a[2]), bf16_to_f(a[3])};
    } else {
        const uint32_t q = *gmem<uint32_t>((const uint8_t*)A + idx);
        const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)q, false);
        const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)q, true);
        r = f32v4{lo[0], lo[1], hi[0], hi[1]};
    }
    return r;
}

// u[row0 .. row0 + 3] over the nonzeros [k0, k1) of (lj, lx): G columns per
// step, every load issued before the first product; same per-element arithmetic
// as the grid forward kernel.  D64: FP64 storage; otherwise the storage type is
// decoded per load.
template <bool D64>
__device__ __forceinline__ void wg_dense_quad(const StageDesc& st, int N, int row0, const int* lj, const double* lx,
                                              int k0, int k1, double (&u)[4]) {
    constexpr int G = D64 ? 4 : 8;
    const int dt = st.dtype;
    const float* scale = (!D64 && dt != SL1_F32) ? st.scale : nullptr;
    for (int k = k0; k < k1; k += G) {
        double xs[G];
        if constexpr (D64) {
            Raw4<SL1_F64> r[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int kk = min(k + g, k1 - 1);
                r[g] = raw_load<SL1_F64>(st.A, (size_t)lj[kk] * N + row0);
                xs[g] = k + g < k1 ? lx[kk] : 0.0;
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (k + g < k1) {
                    double a[4];
                    raw_get<SL1_F64>(r[g], a);
#pragma unroll
                    for (int v = 0; v < 4; ++v) u[v] += xs[g] * a[v];
                }
            }
        } else {
            f32v4 r[G];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int kk = min(k + g, k1 - 1);
                const int j = lj[kk];
                r[g] = dense4_f(dt, st.A, (size_t)j * N + row0);
                xs[g] = k + g < k1 ? lx[kk] : 0.0;
                if (scale) xs[g] *= (double)scale[j];
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                if (k + g < k1) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) u[v] += xs[g] * (double)r[g][v];
                }
            }
        }
    }
}

// dense forward product, residual and sums.  Rows go in quads: with N <= 2048
// the Q = N/4 quads are spread over one thread each in S = 512 / 2^ceil(log2 Q)
// groups, the groups split the nonzeros and their partials meet in a fixed tree
// (at most 8 KB of LDS); with larger N one group takes the quads in chunks of
// 512.  Nonzeros come from the LDS list when it holds them, else are staged
// from the global list through the scratch.
template <bool D64>
__device__ __forceinline__ void wg_dense_forward(const SolveParams* P, int b, const StageDesc& st, const double* x,
                                                 const int* nzl, int n_nz, const int* lj, const double* lx,
                                                 bool in_lds, double* zd, float* zf, const double* yl, char* scr,
                                                 double* s_red, double* s_sum) {
    const int N = P->N, tid = threadIdx.x;
    const int Q = N >> 2;
    int qp = 1;
    while (qp < Q) qp <<= 1;
    const int S = Q <= kWgBlock ? kWgBlock / qp : 1;        // groups
    const int T = kWgBlock / S;                             // threads per group
    const int grp = tid / T, q0 = tid - grp * T;
    double* red = (double*)scr;
    double* s_x = (double*)scr;                             // staging (fallback), also in the scratch
    int* s_j = (int*)(scr + kWgStage * 8);
    double sums[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c * T < Q; ++c) {
        const int q = q0 + c * T;
        const bool valid = q < Q;
        const int row0 = 4 * q;
        double u[4] = {0.0, 0.0, 0.0, 0.0};
        if (in_lds) {
            const int per = (n_nz + S - 1) / S;
            const int k0 = min(n_nz, grp * per), k1 = min(n_nz, k0 + per);
            if (valid) wg_dense_quad<D64>(st, N, row0, lj, lx, k0, k1, u);
        } else {
            for (int base = 0; base < n_nz; base += kWgStage) {
                const int cnt = min(kWgStage, n_nz - base);
                if (tid < cnt) {
                    const int j = nzl[base + tid];
                    s_j[tid] = j;
                    s_x[tid] = x[j];
                }
                __syncthreads();
                const int per = (cnt + S - 1) / S;
                const int k0 = min(cnt, grp * per), k1 = min(cnt, k0 + per);
                if (valid) wg_dense_quad<D64>(st, N, row0, s_j, s_x, k0, k1, u);
                __syncthreads();
            }
        }
        // fixed-order tree over the groups
        for (int h = S >> 1; h >= 1; h >>= 1) {
            if (grp >= h && grp < 2 * h && valid) {
#pragma unroll
                for (int v = 0; v < 4; ++v) red[(size_t)(grp - h) * N + row0 + v] = u[v];
            }
            __syncthreads();
            if (grp < h && valid) {
#pragma unroll
                for (int v = 0; v < 4; ++v) u[v] += red[(size_t)grp * N + row0 + v];
            }
            __syncthreads();
        }
        if (grp == 0 && valid) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = row0 + v;
                const double yv = wg_y(P, b, yl, row);
                const double rho = yv - u[v];
                zd[row] = rho;
                if (zf) zf[row] = (float)rho;
                sums[0] += rho * rho;
                sums[1] += rho * rho;
                sums[2] += yv * rho;
            }
        }
    }
    block_sum<3>(sums, s_red);
    if (tid == 0) {
        s_sum[0] = sums[0];
        s_sum[1] = sums[1];
        s_sum[2] = sums[2];
    }
}

// ---------------------------------------------------------------------------
// Kronecker correlations with LDS operands: G[a][j1] = sum_r (C_r^T Z B_r)[a][j1],
// g_j for j = j1 k2 + a.  MFMA 16x16 operand layout (wave64): lane l holds
// A[l%16][k], B[k][l%16] with k = l/16 (x4 shapes) or 4(l/16)+v (x16 shapes);
// D[4(l/16)+v][l%16], except the FP64 16x16x4 form, whose D is D[4v+l/16][l%16]:
// its first product stores V rows in the 4(l/16)+v order and its second reads
// them back as operand rows, so the two within-tile row permutations cancel.
// ---------------------------------------------------------------------------
template <int DT>
__device__ void wg_kron_adj(const StageDesc& st, const char* fac, const double* zd, const float* zf, char* scr,
                            const uint8_t* mask, double rz, double* g, double (&mx)[3]) {
    const int R = st.R, n1 = st.n1, k1 = st.k1, n2 = st.n2, k2 = st.k2;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const int nA = k2 >> 4, nI = n1 >> 4, nJ = k1 >> 4;
    // phase 1: V_r = C_r^T Z (k2 x n1 per term) into scr
    const int t1 = R * nA * nI;
    for (int t = w; t < t1; t += kWgWaves) {
        const int r = t / (nA * nI), rem = t - r * nA * nI;
        const int a0 = (rem / nI) * 16, i0 = (rem % nI) * 16;
        if constexpr (DT == SL1_F64) {
            const double* Cl = (const double*)fac + (size_t)R * k1 * n1;
            const double* cp = Cl + ((size_t)r * k2 + a0 + li) * n2 + lk;
            const double* zp = zd + (size_t)(i0 + li) * n2 + lk;
            f64x4 d = {0.0, 0.0, 0.0, 0.0};
            for (int k0 = 0; k0 < n2; k0 += 4) d = __builtin_amdgcn_mfma_f64_16x16x4f64(cp[k0], zp[k0], d, 0, 0, 0);
            double* V = (double*)scr;
#pragma unroll
            for (int v = 0; v < 4; ++v) V[((size_t)r * k2 + a0 + 4 * lk + v) * n1 + i0 + li] = d[v];
        } else if constexpr (DT == SL1_F32) {
            const float* Cl = (const float*)fac + (size_t)R * k1 * n1;
            const float* cp = Cl + ((size_t)r * k2 + a0 + li) * n2 + lk;
            const float* zp = zf + (size_t)(i0 + li) * n2 + lk;
            f32x4 d = {0.f, 0.f, 0.f, 0.f};
            for (int k0 = 0; k0 < n2; k0 += 4) d = __builtin_amdgcn_mfma_f32_16x16x4f32(cp[k0], zp[k0], d, 0, 0, 0);
            float* V = (float*)scr;
#pragma unroll
            for (int v = 0; v < 4; ++v) V[((size_t)r * k2 + a0 + 4 * lk + v) * n1 + i0 + li] = d[v];
        } else {
            const uint16_t* Cl = (const uint16_t*)fac + (size_t)R * k1 * n1;
            const uint16_t* cp = Cl + ((size_t)r * k2 + a0 + li) * n2 + 4 * lk;
            const float* zp = zf + (size_t)(i0 + li) * n2 + 4 * lk;
            f32x4 d = {0.f, 0.f, 0.f, 0.f};
            for (int k0 = 0; k0 < n2; k0 += 16) {
                const u16x4 av = *(const u16x4*)(cp + k0);
                const f32v4 zv = *(const f32v4*)(zp + k0);
                s16x4 a, bb;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    a[v] = (short)av[v];
                    bb[v] = (short)bf16_bits(zv[v]);
                }
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bb, d, 0, 0, 0);
            }
            uint16_t* Vh = (uint16_t*)scr;
            uint16_t* Vl = Vh + (size_t)R * k2 * n1;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float hi = bf16_rne(d[v]);
                const float lo = bf16_rne(d[v] - hi);
                const size_t o = ((size_t)r * k2 + a0 + 4 * lk + v) * n1 + i0 + li;
                Vh[o] = bf16_bits(hi);
                Vl[o] = bf16_bits(lo);
            }
        }
    }
    __syncthreads();
    // phase 2: G = sum_r V_r B_r, one 16 x 16 output tile per wave at a time
    const int t2 = nA * nJ;
    for (int t = w; t < t2; t += kWgWaves) {
        const int a0 = (t / nJ) * 16, j0 = (t % nJ) * 16;
        double gv[4];
        if constexpr (DT == SL1_F64) {
            const double* Bl = (const double*)fac;
            const double* V = (const double*)scr;
            f64x4 acc = {0.0, 0.0, 0.0, 0.0};
            for (int r = 0; r < R; ++r) {
                const double* vp = V + ((size_t)r * k2 + a0 + li) * n1 + lk;
                const double* bp = Bl + ((size_t)r * k1 + j0 + li) * n1 + lk;
                for (int k0 = 0; k0 < n1; k0 += 4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(vp[k0], bp[k0], acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) gv[v] = acc[v];
        } else if constexpr (DT == SL1_F32) {
            const float* Bl = (const float*)fac;
            const float* V = (const float*)scr;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int r = 0; r < R; ++r) {
                const float* vp = V + ((size_t)r * k2 + a0 + li) * n1 + lk;
                const float* bp = Bl + ((size_t)r * k1 + j0 + li) * n1 + lk;
                for (int k0 = 0; k0 < n1; k0 += 4) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(vp[k0], bp[k0], acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) gv[v] = (double)acc[v];
        } else {
            const uint16_t* Bl = (const uint16_t*)fac;
            const uint16_t* Vh = (const uint16_t*)scr;
            const uint16_t* Vl = Vh + (size_t)R * k2 * n1;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int r = 0; r < R; ++r) {
                const size_t vo = ((size_t)r * k2 + a0 + li) * n1 + 4 * lk;
                const uint16_t* bp = Bl + ((size_t)r * k1 + j0 + li) * n1 + 4 * lk;
                for (int k0 = 0; k0 < n1; k0 += 16) {
                    const u16x4 hv = *(const u16x4*)(Vh + vo + k0);
                    const u16x4 lv = *(const u16x4*)(Vl + vo + k0);
                    const u16x4 bv = *(const u16x4*)(bp + k0);
                    s16x4 h, lo, bb;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        h[v] = (short)hv[v];
                        lo[v] = (short)lv[v];
                        bb[v] = (short)bv[v];
                    }
                    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(h, bb, acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lo, bb, acc, 0, 0, 0);
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) gv[v] = (double)acc[v];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = (j0 + li) * k2 + a0 + 4 * lk + v;
            g[j] = gv[v];
            if (mask[j]) {
                const double e = st.eps[j];
                mx[0] = fmax(mx[0], fabs(gv[v]) + e * rz);
                mx[1] = fmax(mx[1], fabs(gv[v]));
                mx[2] = fmax(mx[2], e);
            }
        }
    }
}

// dense correlations over the preserved list (LDS or global): wave w takes NA
// atoms at a time (N <= 1024: 4 atoms, all 16 column loads in flight); eps_j is
// fetched together with the columns
template <int NA>
__device__ void wg_dense_adj(const StageDesc& st, int N, const int* act, int n_act, const double* zd, double rz,
                             double* g, double (&mx)[3]) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int first = w * NA; first < n_act; first += kWgWaves * NA) {
        int js[NA];
        int cnt = 0;
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const bool ok = first + q < n_act;
            js[q] = ok ? act[first + q] : -1;
            cnt += ok;
        }
#pragma unroll
        for (int q = 0; q < NA; ++q)
            if (js[q] < 0) js[q] = js[0];
        double e[NA];
#pragma unroll
        for (int q = 0; q < NA; ++q) e[q] = st.eps[js[q]];
        double gv[NA];
        switch (st.dtype) {
            case SL1_F64: dense_dots_t<SL1_F64, NA, (NA == 4 ? 2 : 4)>(st, N, js, zd, lane, gv); break;
            case SL1_F32: dense_dots_t<SL1_F32, NA, 4>(st, N, js, zd, lane, gv); break;
            case SL1_BF16: dense_dots_t<SL1_BF16, NA, 4>(st, N, js, zd, lane, gv); break;
            default: dense_dots_t<SL1_FP8_E4M3, NA, 4>(st, N, js, zd, lane, gv); break;
        }
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
}

__device__ __forceinline__ void wg_copy_factors(const StageDesc& st, char* fac) {
    const size_t es = st.dtype == SL1_F64 ? 8 : (st.dtype == SL1_F32 ? 4 : 2);
    const size_t nb = (size_t)st.R * st.k1 * st.n1 * es, nc = (size_t)st.R * st.k2 * st.n2 * es;
    const u32x4* B = (const u32x4*)st.B;
    const u32x4* Cg = (const u32x4*)st.C;
    u32x4* dst = (u32x4*)fac;
    for (size_t i = threadIdx.x; i < nb / 16; i += kWgBlock) dst[i] = B[i];
    u32x4* dc = (u32x4*)(fac + nb);
    for (size_t i = threadIdx.x; i < nc / 16; i += kWgBlock) dc[i] = Cg[i];
}

// phase clock (thread 0, after the phase's closing barrier)
// (an atomic add whose result is unused: the wave does not wait for the memory round
// trip, so profiling barely slows the phases it measures; one block per signal)
__device__ __forceinline__ void wg_stamp_p(long long* prof, int b, int phase, long long& t) {
    if (prof && threadIdx.x == 0) {
        const long long now = wall_clock64();
        atomicAdd((unsigned long long*)(prof + (size_t)b * kWgPhases + phase), (unsigned long long)(now - t));
        t = now;
    }
}
__device__ __forceinline__ void wg_stamp(const SolveParams* P, int b, int phase, long long& t) {
    wg_stamp_p(P->wg_prof, b, phase, t);
}

}  // namespace

// The parameter block re-read through an opaque copy at the start of each phase:
// pointers and sizes then live only within the phase instead of being held in
// registers across the whole iteration loop.
__device__ __forceinline__ const SolveParams* phase_params(const SolveParams* p) {
    asm volatile("" : "+s"(p));
    return p;
}

// ---------------------------------------------------------------------------
// the whole-solve kernel: grid = batch, block = 512; state in P->ctrl[2 b]
// (written by the initialisation kernel and stored back when a launch ends
// before the signal stops); at most max_it iterations per launch.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWgBlock, 4) void k_solve_wg(const SolveParams* __restrict__ P0, int max_it) {
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    // iteration state of the signal, written by thread 0 between barriers
    __shared__ Control sC;
    __shared__ Scalars sS;
    __shared__ double s_red[48];
    __shared__ double s_sum[4];
    __shared__ double s_kt[2];
    __shared__ int s_cnt[2];
    __shared__ int s_w[kWgWaves * 4];
    __shared__ int s_loaded, s_nz_ok, s_act_ok, s_leave;
    __shared__ long long s_clk;

    // a launch beside the grid kernels runs only the signals they leave alone
    if (P0->wg_absent_only && !P0->absent[b]) return;
    if (tid == 0) {
        sC = P0->ctrl[2 * b];
        s_leave = 0;
        s_loaded = -1;
        s_nz_ok = 0;
        s_act_ok = 0;
        s_clk = P0->wg_prof ? wall_clock64() : 0;
    }
    __syncthreads();
    // a signal parked at an earlier launch waits for the engine that takes over
    const int park = P0->wg_park;
    if (sC.done || (park >= 0 && sC.stage >= park)) return;
    const int park_allow = park >= 0 ? P0->wg_park_allow : 0;
    {
        const SolveParams* P = phase_params(P0);
        if (P->wo_y >= 0) {
            double* yl = (double*)(smem + P->wo_y);
            for (int i = tid; i < P->N; i += kWgBlock) yl[i] = yval(P, b, i);
        }
    }

    for (int it = 0; it < max_it; ++it) {
        const int stage = uni(sC.stage), par = uni(sC.par);
        const int n_nz = uni(sC.n_nz), n_act = uni(sC.n_act);
        if (park >= 0 && stage >= park) break;    // state stored below, lists in slot 0
        if (uni(s_leave)) break;                  // one of the last few short of the park stage
        // the live and parked counts, requested now and compared at the end of the iteration
        int n_live = 0, n_parked = 0;
        if (park_allow > 0 && tid == 0) {
            n_live = __hip_atomic_load(P0->active_signals, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            n_parked = __hip_atomic_load(P0->active_signals + 8, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // ---- factors of a new Kronecker stage, and the two lists, into LDS ----
        {
            const SolveParams* P = phase_params(P0);
            const StageDesc& st = P->st[stage];
            // a layout without factor space serves dense stages only (the host
            // chooses it when every live signal is on the last, dense, stage)
            const bool bad = P->wo_scr < 0 || (st.kind == kKron && P->wo_fac < 0);
            if (bad) {
                if (tid == 0) {
                    Final F;
                    F.gap = 0.0;
                    F.gap_cert = 0.0;
                    F.iters = sC.iter;
                    F.stage = sC.stage;
                    F.status = SL1_ELIMIT;
                    F.par = sC.par;
                    F.t0 = sC.t0;
                    F.tconv = 0;
                    P->fin[b] = F;
                    sC.done = 1;
                    P->ctrl[2 * b] = sC;
                    atomicSub(P->active_signals, 1);
                }
                return;
            }
            if (st.kind == kKron && uni(s_loaded) != stage) {
                wg_copy_factors(st, smem + P->wo_fac);
                if (tid == 0) s_loaded = stage;
            }
            const bool fill_nz = !uni(s_nz_ok) && n_nz <= P->wg_cap_nz;
            const bool fill_act = !uni(s_act_ok) && n_act <= P->wg_cap_act;
            if (fill_nz) {
                const int* nzl = nzbuf(P, b, 0);
                const double* x = xbuf(P, b, par);
                int* lj = (int*)(smem + P->wo_lnj);
                double* lx = (double*)(smem + P->wo_lnx);
                for (int i = tid; i < n_nz; i += kWgBlock) {
                    const int j = nzl[i];
                    lj[i] = j;
                    lx[i] = x[j];
                }
            }
            if (fill_act) {
                const int* act = actbuf(P, b, 0);
                int* la = (int*)(smem + P->wo_lact);
                for (int i = tid; i < n_act; i += kWgBlock) la[i] = act[i];
            }
            __syncthreads();
            if (tid == 0) {
                if (fill_nz) s_nz_ok = 1;
                if (fill_act) s_act_ok = 1;
            }
            __syncthreads();
        }
        // ---- forward product and residual ----
        {
            const SolveParams* P = phase_params(P0);
            const StageDesc& st = P->st[stage];
            double* zd = (double*)(smem + P->wo_zd);
            float* zf = P->wo_zf >= 0 ? (float*)(smem + P->wo_zf) : nullptr;
            const double* yl = P->wo_y >= 0 ? (const double*)(smem + P->wo_y) : nullptr;
            char* scr = P->wo_scr >= 0 ? smem + P->wo_scr : nullptr;
            const double* x = xbuf(P, b, par);
            const int* nzl = nzbuf(P, b, 0);
            if (st.kind == kKron) {
                const char* fac = smem + P->wo_fac;
                const int zround = st.dtype == SL1_BF16 ? 2 : (st.dtype == SL1_F32 ? 1 : 0);
                const bool in_lds = uni(s_nz_ok) != 0;
                const int* lj = (const int*)(smem + P->wo_lnj);
                const double* lx = (const double*)(smem + P->wo_lnx);
                if (st.dtype == SL1_F64)
                    wg_kron_forward<true>(P, b, st, fac, x, nzl, n_nz, lj, lx, in_lds, zround, zd, zf, yl, scr, s_red, s_sum);
                else
                    wg_kron_forward<false>(P, b, st, fac, x, nzl, n_nz, lj, lx, in_lds, zround, zd, zf, yl, scr, s_red, s_sum);
            } else {
                const bool in_lds = uni(s_nz_ok) != 0;
                const int* lj = (const int*)(smem + P->wo_lnj);
                const double* lx = (const double*)(smem + P->wo_lnx);
                if (st.dtype == SL1_F64) wg_dense_forward<true>(P, b, st, x, nzl, n_nz, lj, lx, in_lds, zd, zf, yl, scr, s_red, s_sum);
                else wg_dense_forward<false>(P, b, st, x, nzl, n_nz, lj, lx, in_lds, zd, zf, yl, scr, s_red, s_sum);
            }
            __syncthreads();
            wg_stamp(P, b, 0, s_clk);
        }
        // ---- correlations over A_t, maxima of the stable dual scaling, scalars ----
        {
            const SolveParams* P = phase_params(P0);
            const int N = P->N, K = P->K;
            const StageDesc& st = P->st[stage];
            const double* zd = (const double*)(smem + P->wo_zd);
            const double rz = uni(sqrt(s_sum[1]));
            double* gvec = gbuf(P, b, par);
            double mx[3] = {0.0, 0.0, 0.0};
            if (st.kind == kDense) {
                const int* act = uni(s_act_ok) ? (const int*)(smem + P->wo_lact) : actbuf(P, b, 0);
                if (N <= 1024) wg_dense_adj<4>(st, N, act, n_act, zd, rz, gvec, mx);
                else wg_dense_adj<1>(st, N, act, n_act, zd, rz, gvec, mx);
            } else {
                const char* fac = smem + P->wo_fac;
                char* scr = smem + P->wo_scr;
                const float* zf = (const float*)(smem + P->wo_zf);
                const uint8_t* mask = P->mask + (size_t)b * K;
                if (st.dtype == SL1_F64) wg_kron_adj<SL1_F64>(st, fac, zd, zf, scr, mask, rz, gvec, mx);
                else if (st.dtype == SL1_F32) wg_kron_adj<SL1_F32>(st, fac, zd, zf, scr, mask, rz, gvec, mx);
                else wg_kron_adj<SL1_BF16>(st, fac, zd, zf, scr, mask, rz, gvec, mx);
            }
            block_max<3>(mx, s_red);
            if (tid == 0) {
                Scalars S;
                scalars_from(P, sC, s_sum[0], s_sum[1], s_sum[2], sqrt(s_sum[1]), mx[0], mx[1], mx[2],
                             P->rule ? P->yy[b] : 0.0, S);
                if (S.conv == 1) S.tconv = wall_clock64();
                sS = S;
            }
            __syncthreads();
            wg_stamp(P, b, st.kind == kDense ? 1 : 2, s_clk);
        }
        if (uni(sS.conv)) {
            if (tid == 0) {
                const SolveParams* P = phase_params(P0);
                Final F;
                F.gap = sS.Gt;
                F.gap_cert = sS.Gp + sS.delta;
                F.iters = sC.iter;
                F.stage = sC.stage;
                F.status = sS.conv == 2 ? SL1_MAXITER : SL1_OK;
                F.par = sC.par;
                F.t0 = sC.t0;
                F.tconv = sS.tconv;
                P->fin[b] = F;
                sC.done = 1;
                P->ctrl[2 * b] = sC;
                atomicSub(P->active_signals, 1);
            }
            return;
        }
        // ---- stable GAP test, look-ahead count, FISTA step, compaction ----
        {
            const SolveParams* P = phase_params(P0);
            const int K = P->K;
            const StageDesc& st = P->st[stage];
            const int cap_nz = P->wg_cap_nz, cap_act = P->wg_cap_act;
            int* act = actbuf(P, b, 0);
            int* nzl = nzbuf(P, b, 0);
            int* la = (int*)(smem + P->wo_lact);
            int* lj = (int*)(smem + P->wo_lnj);
            double* lx = (double*)(smem + P->wo_lnx);
            const bool act_lds = uni(s_act_ok) != 0;
            uint8_t* mask = P->mask + (size_t)b * K;
            double* xc = xbuf(P, b, par);
            double* xo = xbuf(P, b, 1 - par);
            const double* gcur = gbuf(P, b, par);
            const double* gprev = gbuf(P, b, 1 - par);
            const double* eps = st.eps;
            const double* atn = st.at_norm;
            const double* an = P->atom_norm;
            const double c1 = uni(sS.c1), c2 = uni(sS.c2), Rp = uni(sS.Rp), beta = uni(sS.beta);
            const double invL = st.invL, thr = uni(sC.lam) * st.invL, keep_min = 1.0 - P->margin;
            const int rule = P->rule;
            const double Rd = uni(sS.Rd), invlam = uni(1.0 / sC.lam), eyl = uni(sS.ny / sC.lam);
            const double* cyb = rule ? P->cy + (size_t)b * K : nullptr;
            const double* eI = P->st[P->n_stages - 1].eps;
            const bool no_reject = uni(sC.iter) % P->screen_every != 0;
            int wpos = 0, zpos = 0;
            double sv[2] = {0.0, 0.0};   // look-ahead count K_t, ||x_{t+1}||_1
            // a list of all K atoms is the identity (compactions keep the order)
            const bool ident = n_act == K;
            for (int base = 0; base < n_act; base += 2 * kWgBlock) {
                int jj[2];
                bool keep[2], nzf[2];
                double xnv[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i = base + h * kWgBlock + tid;
                    keep[h] = nzf[h] = false;
                    jj[h] = 0;
                    xnv[h] = 0.0;
                    if (i < n_act) {
                        const int j = ident ? i : (act_lds ? la[i] : act[i]);
                        jj[h] = j;
                        const double gt = gcur[j];
                        const double gp = gprev[j];
                        const double xt = xc[j];
                        const double xp = xo[j];
                        const double e = eps[j];
                        const double ag = fabs(gt);
                        if (rule) {
                            // stable Dynamic Safe: |a^T y| / lambda + ||theta' - y/lambda|| ||a||
                            const double c = fabs(cyb[j]) * invlam;
                            keep[h] = c + eI[j] * eyl + Rd * an[j] >= keep_min;
                            sv[0] += (c + Rd * atn[j] >= 1.0) ? 1.0 : 0.0;
                        } else {
                            // stable GAP Safe: |a~^T theta'| + eps ||theta'|| + R' ||a||
                            keep[h] = c1 * ag + e * c2 + Rp * an[j] >= keep_min;
                            // look-ahead: conventional test on the approximate atom
                            sv[0] += (c1 * ag + Rp * atn[j] >= 1.0) ? 1.0 : 0.0;
                        }
                        if (no_reject) keep[h] = true;
                        // FISTA (ISTA: beta = 0) step from the two correlation vectors
                        const double zpt = xt + beta * (xt - xp);
                        const double hh = (1.0 + beta) * gt - beta * gp;
                        const double v = zpt + hh * invL;
                        double xn = 0.0;
                        if (keep[h]) xn = (v > thr) ? v - thr : ((v < -thr) ? v + thr : 0.0);
                        xo[j] = xn;
                        if (!keep[h]) {
                            xc[j] = 0.0;
                            mask[j] = 0;
                            if (xt != 0.0) sv[0] += kRejNz;
                        }
                        nzf[h] = keep[h] && (xn != 0.0);
                        xnv[h] = xn;
                        sv[1] += fabs(xn);
                    }
                }
                // every read of this part of the list precedes the in-place writes
                __syncthreads();
                // positions in list order: the kept and the nonzero atoms of both halves
                const bool fl[4] = {keep[0], nzf[0], keep[1], nzf[1]};
                int ps[4], ts[4];
                wg_scan_flags<4>(fl, s_w, ps, ts);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int pk = ps[2 * h], pz = ps[2 * h + 1];
                    if (keep[h]) {
                        act[wpos + pk] = jj[h];
                        if (wpos + pk < cap_act) la[wpos + pk] = jj[h];
                    }
                    if (nzf[h]) {
                        nzl[zpos + pz] = jj[h];
                        if (zpos + pz < cap_nz) {
                            lj[zpos + pz] = jj[h];
                            lx[zpos + pz] = xnv[h];
                        }
                    }
                    wpos += ts[2 * h];
                    zpos += ts[2 * h + 1];
                }
            }
            block_sum<2>(sv, s_red);
            if (tid == 0) {
                s_kt[0] = sv[0];
                s_kt[1] = sv[1];
                s_cnt[0] = wpos;
                s_cnt[1] = zpos;
                s_act_ok = wpos <= cap_act;
                s_nz_ok = zpos <= cap_nz;
            }
            __syncthreads();
            wg_stamp(P, b, 3, s_clk);
        }
        // ---- trace row, Algorithm 2, momentum (thread 0) ----
        if (tid == 0) {
            const SolveParams* P = phase_params(P0);
            const StageDesc& st = P->st[stage];
            Control C = sC;
            // rejected nonzero coefficients travel above the look-ahead count
            const double rnz = floor(s_kt[0] / kRejNz);
            const double kt = s_kt[0] - rnz * kRejNz;
            if (P->trace && C.iter < P->trace_cap) {
                double* tr = P->trace + ((size_t)b * P->trace_cap + C.iter) * SL1_TRACE_FIELDS;
                tr[0] = C.iter; tr[1] = C.stage; tr[2] = C.n_act; tr[3] = s_cnt[0];
                tr[4] = kt;
                tr[5] = sS.Gp; tr[6] = sS.Gt; tr[7] = sS.delta; tr[8] = P->rule ? sS.Rd : sS.Rp; tr[9] = sS.gamma;
                tr[10] = C.l1; tr[11] = sS.P; tr[12] = C.n_nz;
            }
            const int i_new = switch_dictionary(C.stage, P->n_stages - 1, sS.gamma, P->Gamma, kt, st.rc, (double)P->K);
            if (i_new != C.stage || rnz > 0.0) {   // a switch, or a rejection that zeroed x_t[j]: restart
                C.stage = i_new;
                C.ksince = 0;
                C.tau = 1.0;
            } else {
                C.ksince += 1;
                C.tau = sS.tau_next;
            }
            C.iter += 1;
            C.par = 1 - C.par;
            C.n_act = s_cnt[0];
            C.n_nz = s_cnt[1];
            C.l1 = s_kt[1];
            if (park >= 0 && C.stage >= park && stage < park) atomicAdd(P->active_signals + 8, 1);
            // when at most park_allow live signals (counts of this iteration's start) are short
            // of the park stage, the ones still short of it stop here as well
            if (park_allow > 0 && C.stage < park && n_live - n_parked <= park_allow) s_leave = 1;
            sC = C;
        }
        __syncthreads();
    }
    if (tid == 0) P0->ctrl[2 * b] = sC;
}

// ---------------------------------------------------------------------------
// Tail kernel of the hybrid solve: every live signal is on the last, dense,
// stage with a small preserved set.  The whole per-atom state of the preserved
// set lives in LDS by list position (index, x_t, x_{t-1}, g_t, g_{t-1}, eps_j,
// ||a_j||, ||a~_j||) and moves with the compaction.  Two modes per signal:
//   columns  an iteration forms the residual from the gathered columns and
//            correlates it with the preserved columns (all 8 waves); global
//            memory is touched only for those columns, for atoms being screened
//            (their x and mask entries) and at exit;
//   Gram     once |A_t| fits the Gram capacity, G = A_t^T A_t and c = A_t^T y are
//            formed once (FP64 MFMA over the stored columns), after which an
//            iteration has no N-length work: g = c - G x_t, y^T rho =
//            ||y||^2 - c^T x_t and ||rho||^2 = y^T rho - x_t^T g (rho = y - A x_t).
//            A_t only shrinks, so G stays valid; positions keep their row of G.
//            Wave 0 runs these iterations alone, without workgroup barriers.
// The FP64 rounding of the Gram forms is bounded a priori (standard dot-product
// bound gamma_n = n u / (1 - n u), u = 2^-53, n doubled for slack): every |g_j|
// is off by at most eta ||a_j||, eta = gamma_n (||y|| + X) with X = sum_k ||a_k||
// |x_k|, so eta ||a_j|| joins the dual-scaling maximum (Lemma 2 stays exact) and
// the sphere test; ||rho||^2 and y^T rho are off by at most 4 gamma_n (||y|| + X)^2
// and gamma_n (||y|| + X)^2, whose effect on P(x_t) - D(theta') is added to delta
// (Theorem 1), hence to the radius R' and to the certified gap.
// ---------------------------------------------------------------------------
namespace {

struct TailState {
    int* la;                 // atom index
    int* lg;                 // Gram mode: a compaction's new position of each position
    double *xt, *xp, *gt, *gm, *e, *an, *atn;   // x_t, x_{t-1}, g_t, g_{t-1}, eps, norms
    double* cy;              // a^T y on the exact dictionary (stable Dynamic Safe)
};

__device__ __forceinline__ TailState tail_state(char* smem, const SolveParams* P) {
    const int cap = P->wg_cap_act;
    TailState T;
    T.la = (int*)(smem + P->wo_lact);
    double* base = (double*)(smem + P->wo_tail);
    T.xt = base;
    T.xp = base + cap;
    T.gt = base + 2 * (size_t)cap;
    T.gm = base + 3 * (size_t)cap;
    T.e = base + 4 * (size_t)cap;
    T.an = base + 5 * (size_t)cap;
    T.atn = base + 6 * (size_t)cap;
    T.cy = base + 7 * (size_t)cap;
    T.lg = (int*)(base + 8 * (size_t)cap);
    return T;
}

// LDS ordering among the lanes of one wave (no other wave takes part)
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// correlations of the preserved positions (wave w takes NA positions at a time)
template <int NA>
__device__ void tail_adj(const StageDesc& st, int N, const TailState& T, int n_act, const double* zd, double rz,
                         double (&mx)[3]) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int first = w * NA; first < n_act; first += kWgWaves * NA) {
        int js[NA];
        int cnt = 0;
#pragma unroll
        for (int q = 0; q < NA; ++q) {
            const bool ok = first + q < n_act;
            js[q] = T.la[ok ? first + q : first];
            cnt += ok;
        }
        double gv[NA];
        switch (st.dtype) {
            case SL1_F64: dense_dots_t<SL1_F64, NA, (NA == 4 ? 2 : 4)>(st, N, js, zd, lane, gv); break;
            case SL1_F32: dense_dots_t<SL1_F32, NA, 4>(st, N, js, zd, lane, gv); break;
            case SL1_BF16: dense_dots_t<SL1_BF16, NA, 4>(st, N, js, zd, lane, gv); break;
            default: dense_dots_t<SL1_FP8_E4M3, NA, 4>(st, N, js, zd, lane, gv); break;
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < NA; ++q) {
                if (q < cnt) {
                    const int i = first + q;
                    const double e = T.e[i];
                    T.gt[i] = gv[q];
                    mx[0] = fmax(mx[0], fabs(gv[q]) + e * rz);
                    mx[1] = fmax(mx[1], fabs(gv[q]));
                    mx[2] = fmax(mx[2], e);
                }
            }
        }
    }
}

// c_i = a_{la[i]}^T y for positions i < m (one wave per position, FP64 sums)
template <int DT>
__device__ void tail_gram_c(const StageDesc& st, int N, const int* la, int m, const double* yl, double* c) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int i = w; i < m; i += kWgWaves) {
        const int j = la[i];
        const size_t cj = (size_t)j * N;
        double acc = 0.0;
        for (int r = 4 * l; r < N; r += 256) {
            double a[4];
            raw_get<DT>(raw_load<DT>(st.A, cj + r), a);
#pragma unroll
            for (int v = 0; v < 4; ++v) acc = fma(a[v], yl[r + v], acc);
        }
        acc = wave_sum(acc);
        if (l == 0) c[i] = st.scale ? acc * (double)st.scale[j] : acc;
    }
}

// Gram matrix of positions 0..m-1 (column-major, leading dimension ld) with FP64
// MFMA 16x16x4: one wave per 16 x 16 tile (I, J), I <= J.  Lane l reads rows
// k0 + 4 (l / 16) .. + 3 of the columns at positions 16 I + l % 16 and
// 16 J + l % 16 and feeds row k0 + 4 (l / 16) + v to the v-th MFMA of a step,
// so the four MFMAs of a step cover 16 rows; column scales apply at the end.
// FP64 accumulator layout: lane l holds D[4 v + l / 16][l % 16].
template <int DT>
__device__ void tail_gram_g(const StageDesc& st, int N, const int* la, int m, double* G, int ld) {
    constexpr int U = DT == SL1_F64 ? 4 : 8;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
    const int nt = (m + 15) >> 4;
    const int ntiles = nt * (nt + 1) / 2;
    for (int t = w; t < ntiles; t += kWgWaves) {
        int I = 0, rem = t;
        while (rem >= nt - I) {
            rem -= nt - I;
            ++I;
        }
        const int J = I + rem;
        const int pa = min(16 * I + li, m - 1), pb = min(16 * J + li, m - 1);
        const size_t ca = (size_t)la[pa] * N, cb = (size_t)la[pb] * N;
        f64x4 d = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < N; k0 += 16 * U) {
            Raw4<DT> ra[U], rb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int r = k0 + 16 * u + 4 * lk;
                const int rr = r < N ? r : 0;          // rows past N read row 0 and are zeroed
                ra[u] = raw_load<DT>(st.A, ca + rr);
                rb[u] = raw_load<DT>(st.A, cb + rr);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool ok = k0 + 16 * u + 4 * lk < N;
                double a[4], bv[4];
                raw_get<DT>(ra[u], a);
                raw_get<DT>(rb[u], bv);
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    d = __builtin_amdgcn_mfma_f64_16x16x4f64(ok ? a[v] : 0.0, bv[v], d, 0, 0, 0);
            }
        }
        const double sb = st.scale ? (double)st.scale[la[pb]] : 1.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = 16 * I + 4 * v + lk, c = 16 * J + li;
            if (r < m && c < m) {
                const double sa = st.scale ? (double)st.scale[la[r]] : 1.0;
                const double val = d[v] * sa * sb;
                G[(size_t)c * ld + r] = val;
                if (I != J) G[(size_t)r * ld + c] = val;
            }
        }
    }
}

// Gram mode set-up for positions 0..m-1 (all threads): c into T.gt, ||y||^2,
// then (y no longer needed; the Gram region overlays z, the scratch and y) G and
// c, row i of G and c_i belonging to position i (the Gram loop keeps it so).
__device__ __attribute__((noinline)) void tail_gram_build(const SolveParams* P, int b, const StageDesc& st,
                                                          char* smem, int m, double* s_red, double* s_yy) {
    const int N = P->N, gcap = P->wg_cap_gram, tid = threadIdx.x;
    const TailState T = tail_state(smem, P);
    const double* yl = (const double*)(smem + P->wo_y);
    switch (st.dtype) {
        case SL1_F64: tail_gram_c<SL1_F64>(st, N, T.la, m, yl, T.gt); break;
        case SL1_F32: tail_gram_c<SL1_F32>(st, N, T.la, m, yl, T.gt); break;
        case SL1_BF16: tail_gram_c<SL1_BF16>(st, N, T.la, m, yl, T.gt); break;
        default: tail_gram_c<SL1_FP8_E4M3>(st, N, T.la, m, yl, T.gt); break;
    }
    double yy[1] = {0.0};
    for (int i = tid; i < N; i += kWgBlock) yy[0] = fma(yl[i], yl[i], yy[0]);
    block_sum<1>(yy, s_red);              // its barriers also order every read of y before G
    if (tid == 0) *s_yy = yy[0];
    double* G = (double*)(smem + P->wo_gram);
    double* cv = G + (size_t)gcap * gcap;
    switch (st.dtype) {
        case SL1_F64: tail_gram_g<SL1_F64>(st, N, T.la, m, G, gcap); break;
        case SL1_F32: tail_gram_g<SL1_F32>(st, N, T.la, m, G, gcap); break;
        case SL1_BF16: tail_gram_g<SL1_BF16>(st, N, T.la, m, G, gcap); break;
        default: tail_gram_g<SL1_FP8_E4M3>(st, N, T.la, m, G, gcap); break;
    }
    for (int i = tid; i < m; i += kWgBlock) cv[i] = T.gt[i];
    __syncthreads();
}

// Gram-mode iterations of one signal, wave 0 only; lane l holds list positions
// l + 64 h, h < H (Gram capacity <= 64 H).  Row and column i of G and c_i belong
// to position i: a rejection compacts them with the positions.  Leaves the control
// state in *sCp; sets *s_done when the signal stopped.
template <int H>
__device__ __forceinline__ void tail_gram_loop(const SolveParams* P0, int b, int it, int max_it, char* smem,
                                               Control* sCp, int* s_done, long long* s_clk, double yy) {
    const int l = threadIdx.x & 63;
    const SolveParams* P = phase_params(P0);
    Control C = *sCp;
    const StageDesc& st = P->st[uni(C.stage)];
    const int N = P->N, K = P->K, gcap = P->wg_cap_gram;
    const TailState T = tail_state(smem, P);
    double* G = (double*)(smem + P->wo_gram);
    double* cv = G + (size_t)gcap * gcap;
    int* nidx = T.lg;                          // scratch of a compaction: new position or -1
    const double invL = uni(st.invL), lam = uni(C.lam), thr = uni(lam * st.invL), keep_min = uni(1.0 - P->margin);
    const double invlam = uni(1.0 / lam);
    const double ny = uni(sqrt(yy));
    // what the iterations read of the parameter block, loaded once (block-uniform)
    ScalarConsts SK = scalar_consts(P);
    SK.tol = uni(SK.tol);
    SK.slack = uni(SK.slack);
    SK.rule = uni(SK.rule);
    SK.ista = uni(SK.ista);
    SK.last_stage = uni(SK.last_stage);
    SK.max_iter = uni(SK.max_iter);
    const double cq = uni(st.cq);
    const int rule = SK.rule, screen_every = uni(P->screen_every);
    const int trace_cap = P->trace ? uni(P->trace_cap) : 0;
    double* const trace = uni_ptr(P->trace);
    double* const xb0 = uni_ptr(xbuf(P, b, 0));
    double* const xb1 = uni_ptr(xbuf(P, b, 1));
    uint8_t* const maskb = uni_ptr(P->mask + (size_t)b * K);
    long long* const prof = uni_ptr(P->wg_prof);
    const double yyb = rule ? uni(P->yy[b]) : 0.0;
    const unsigned long long below = (1ull << l) - 1ull;
    int n_act = uni(C.n_act), n_nz = 0;
    double X;
    {
        double xs = 0.0;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const int i = l + 64 * h;
            const bool in = i < n_act;
            const double xv = in ? T.xt[i] : 0.0;
            if (in) xs += T.an[i] * fabs(xv);
            n_nz += __popcll(__ballot(xv != 0.0));
        }
        X = uni(wave_sum(xs));
    }
    // max eps over the preserved positions: it changes only when atoms are screened
    double me_pos = 0.0;
#pragma unroll
    for (int h = 0; h < H; ++h) {
        const int i = l + 64 * h;
        if (i < n_act) me_pos = fmax(me_pos, T.e[i]);
    }
    double me_c = uni(wave_max_nonneg_full(me_pos));
    wave_sync_lds();
    for (; it < max_it; ++it) {
        // per-iteration copies of the parameter block and of the lane's positions
        // keep addresses out of the loop-carried registers
        const SolveParams* Pi = phase_params(P0);
        int lo = l;
        asm volatile("" : "+v"(lo));
        const int par = uni(C.par);
        const double nu = 2.0 * (double)(N + n_nz + 2) * 0x1p-53;
        const double gam = uni(nu / (1.0 - nu));
        const double YX = uni(ny + X);
        const double eta = uni(gam * YX);
        // ---- g = c - G x_t over the preserved positions ----
        // g_i = c_i - sum_k G[k][i] x_k in position order (G is symmetric; lanes read
        // consecutive entries of a row, and a zero x_k adds an exact zero), four
        // independent chains (any order is within the bound)
        double xt[H], g[H];
        double cx = 0.0, xg = 0.0, m1 = 0.0, m0 = 0.0;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            const int i = lo + 64 * h;
            xt[h] = g[h] = 0.0;
            if (i < n_act) {
                xt[h] = T.xt[i];
                const double* Gc = G + i;
                double g0 = cv[i], g1 = 0.0, g2 = 0.0, g3 = 0.0;
                int k = 0;
#pragma unroll 1
                for (; k + 8 <= n_act; k += 8) {
                    // the step's reads are issued before its products
                    const double* Gk = Gc + (size_t)k * gcap;
                    double a[8], x[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) a[u] = Gk[(size_t)u * gcap];
#pragma unroll
                    for (int u = 0; u < 8; ++u) x[u] = T.xt[k + u];
                    asm volatile("" ::: "memory");
                    g0 = fma(-a[0], x[0], g0);
                    g1 = fma(-a[1], x[1], g1);
                    g2 = fma(-a[2], x[2], g2);
                    g3 = fma(-a[3], x[3], g3);
                    g0 = fma(-a[4], x[4], g0);
                    g1 = fma(-a[5], x[5], g1);
                    g2 = fma(-a[6], x[6], g2);
                    g3 = fma(-a[7], x[7], g3);
                }
                for (; k + 4 <= n_act; k += 4) {
                    g0 = fma(-Gc[(size_t)k * gcap], T.xt[k], g0);
                    g1 = fma(-Gc[(size_t)(k + 1) * gcap], T.xt[k + 1], g1);
                    g2 = fma(-Gc[(size_t)(k + 2) * gcap], T.xt[k + 2], g2);
                    g3 = fma(-Gc[(size_t)(k + 3) * gcap], T.xt[k + 3], g3);
                }
                for (; k < n_act; ++k) g0 = fma(-Gc[(size_t)k * gcap], T.xt[k], g0);
                const double gi = (g0 + g1) + (g2 + g3);
                g[h] = gi;
                cx = fma(cv[i], xt[h], cx);
                xg = fma(xt[h], gi, xg);
                m1 = fmax(m1, fabs(gi) + eta * T.an[i]);
                m0 = fmax(m0, fabs(gi));
            }
        }
        // the five wave reductions (all 64 lanes of wave 0 take part; m1, m0, me >= 0)
        cx = uni(wave_sum_full(cx));
        xg = uni(wave_sum_full(xg));
        m1 = uni(wave_max_nonneg_full(m1));
        m0 = uni(wave_max_nonneg_full(m0));
        const double me = me_c;
        // ---- scalars (uniform) ----
        const double yr = yy - cx;
        const double r2 = fmax(yr - xg, 0.0);
        const double e_yr = gam * YX * YX, e_r2 = 4.0 * gam * YX * YX;
        const double rz = uni(sqrt(r2 + e_r2));
        double c1, c2, Rp, Rd, ny, beta, tau_next, Gp, Gt, delta, gam_t, Pv;
        int conv;
        {
            Scalars S;
            // the stable point scales by the bound max(|g_j| + eta ||a_j||) (Lemma 2 holds for the
            // exact products); the conventional gap of the stop test by max |g_j|, as the grid
            // engine does
            scalars_core(SK, cq, C, r2, r2, yr, sqrt(r2), m1 + me * rz, m0, me, yyb, S);
            c1 = uni(S.c1);
            beta = uni(S.beta);
            tau_next = uni(S.tau_next);
            Gp = uni(S.Gp);
            Gt = uni(S.Gt);
            gam_t = uni(S.gamma);
            Pv = uni(S.P);
            conv = uni(S.conv);
            delta = uni(S.delta + 0.5 * e_r2 + lam * c1 * e_yr + 0.5 * lam * lam * c1 * c1 * e_r2 + lam * gam * C.l1);
            Rp = uni(sqrt(2.0 * fmax(Gp, 0.0) + 2.0 * delta) * invlam);
            c2 = uni(c1 * rz);
            // the Dynamic Safe radius also carries the Gram errors of ||rho||^2 and y^T rho
            Rd = uni(sqrt(S.Rd * S.Rd + c1 * c1 * e_r2 + 2.0 * c1 * e_yr * invlam));
            ny = uni(S.ny);
        }
        wg_stamp_p(prof, b, 2, *s_clk);
        if (conv) {
            double* xc = xbuf(Pi, b, par);
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int i = lo + 64 * h;
                if (i < n_act) xc[T.la[i]] = xt[h];
            }
            if (l == 0) {
                Final F;
                F.gap = Gt;
                F.gap_cert = Gp + delta;
                F.iters = C.iter;
                F.stage = C.stage;
                F.status = conv == 2 ? SL1_MAXITER : SL1_OK;
                F.par = C.par;
                F.t0 = C.t0;
                F.tconv = conv == 1 ? wall_clock64() : 0;
                Pi->fin[b] = F;
                C.done = 1;
                Pi->ctrl[2 * b] = C;
                *sCp = C;
                *s_done = 1;
                atomicSub(Pi->active_signals, 1);
            }
            return;
        }
        // ---- stable GAP test (|g_j| + eta ||a_j||), look-ahead count, FISTA step ----
        const double Rq = uni(Rp + c1 * eta);
        bool keep[H], nzf[H];
        double xn[H];
        double kt = 0.0, l1 = 0.0, Xn = 0.0;
        const bool screen_now = C.iter % screen_every == 0;   // rejections only every screen_every
        {
            double* xc = par ? xb1 : xb0;
            double* xo = par ? xb0 : xb1;
            uint8_t* mask = maskb;
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int i = lo + 64 * h;
                keep[h] = nzf[h] = false;
                xn[h] = 0.0;
                if (i < n_act) {
                    const double an = T.an[i], ag = fabs(g[h]);
                    if (rule) {          // stable Dynamic Safe with a^T y given
                        const double c = fabs(T.cy[i]) * invlam;
                        keep[h] = c + T.e[i] * ny * invlam + Rd * an >= keep_min;
                        kt += (c + Rd * T.atn[i] >= 1.0) ? 1.0 : 0.0;
                    } else {
                        keep[h] = c1 * ag + T.e[i] * c2 + Rq * an >= keep_min;
                        kt += (c1 * ag + Rp * T.atn[i] >= 1.0) ? 1.0 : 0.0;
                    }
                    if (!screen_now) keep[h] = true;
                    const double xp = T.xp[i], gm = T.gm[i];
                    const double zpt = xt[h] + beta * (xt[h] - xp);
                    const double hh = (1.0 + beta) * g[h] - beta * gm;
                    const double v = zpt + hh * invL;
                    if (keep[h]) xn[h] = (v > thr) ? v - thr : ((v < -thr) ? v + thr : 0.0);
                    if (!keep[h]) {      // screened: its coefficient is zero in both iterates
                        const int j = T.la[i];
                        xc[j] = 0.0;
                        xo[j] = 0.0;
                        mask[j] = 0;
                        if (xt[h] != 0.0) kt += kRejNz;
                    }
                    nzf[h] = keep[h] && (xn[h] != 0.0);
                    l1 += fabs(xn[h]);
                    Xn += an * fabs(xn[h]);
                }
            }
        }
        // ---- compaction (positions keep their order); without a rejection every position
        // stays and only the iterates and the correlations change ----
        int nkeep = 0;
#pragma unroll
        for (int h = 0; h < H; ++h) nkeep += __popcll(__ballot(keep[h]));
        int wpos = 0, zpos = 0;
#pragma unroll
        for (int h = 0; h < H; ++h) zpos += __popcll(__ballot(nzf[h]));
        wave_sync_lds();                  // every lane's reads of x_t precede the writes
        if (uni(nkeep) == n_act) {
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int i = lo + 64 * h;
                if (keep[h]) {
                    T.xt[i] = xn[h];
                    T.xp[i] = xt[h];
                    T.gm[i] = g[h];
                }
            }
            wpos = n_act;
        } else {
            // new position of each kept position (-1: rejected)
            int np[H];
#pragma unroll
            for (int h = 0; h < H; ++h) {
                const int i = lo + 64 * h;
                const unsigned long long bk = __ballot(keep[h]);
                np[h] = keep[h] ? wpos + __popcll(bk & below) : -1;
                wpos += __popcll(bk);
                if (i < n_act) nidx[i] = np[h];
            }
            // the per-position state: every lane reads its kept entries, then writes them
            double mep = 0.0;
            {
                int jj[H];
                double ev[H], anv[H], atv[H], cyv[H], cvv[H];
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    const int i = lo + 64 * h;
                    jj[h] = 0;
                    ev[h] = anv[h] = atv[h] = cyv[h] = cvv[h] = 0.0;
                    if (keep[h]) {
                        jj[h] = T.la[i];
                        ev[h] = T.e[i];
                        anv[h] = T.an[i];
                        atv[h] = T.atn[i];
                        cyv[h] = T.cy[i];
                        cvv[h] = cv[i];
                    }
                }
                wave_sync_lds();
#pragma unroll
                for (int h = 0; h < H; ++h) {
                    if (keep[h]) {
                        const int q = np[h];
                        T.la[q] = jj[h];
                        T.xt[q] = xn[h];
                        T.xp[q] = xt[h];
                        T.gm[q] = g[h];
                        T.e[q] = ev[h];
                        T.an[q] = anv[h];
                        T.atn[q] = atv[h];
                        T.cy[q] = cyv[h];
                        cv[q] = cvv[h];
                        mep = fmax(mep, ev[h]);
                    }
                }
            }
            wave_sync_lds();
            // rows and columns of G follow their positions: four rows are read before any of
            // them is written; a kept row r goes to row nidx[r] <= r, whose old content was read
            // in this batch or an earlier one, so nothing is overwritten before it is read
            const int n_old = n_act;
            for (int r0 = 0; r0 < n_old; r0 += 4) {
                double v[4][H];
                int nr[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int r = r0 + u;
                    nr[u] = r < n_old ? nidx[r] : -1;
#pragma unroll
                    for (int h = 0; h < H; ++h) {
                        const int k = lo + 64 * h;
                        v[u][h] = (r < n_old && k < n_old) ? G[(size_t)r * gcap + k] : 0.0;
                    }
                }
                wave_sync_lds();
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int rn = uni(nr[u]);
                    if (rn >= 0) {
#pragma unroll
                        for (int h = 0; h < H; ++h)
                            if (np[h] >= 0) G[(size_t)rn * gcap + np[h]] = v[u][h];
                    }
                }
                wave_sync_lds();
            }
            me_c = uni(wave_max_nonneg_full(mep));
        }
        wave_sync_lds();
        kt = uni(wave_sum_full(kt));
        l1 = uni(wave_sum_full(l1));
        Xn = uni(wave_sum_full(Xn));
        // rejected nonzero coefficients travel above the look-ahead count
        const double rnz = uni(floor(kt / kRejNz));
        kt -= rnz * kRejNz;
        wg_stamp_p(prof, b, 3, *s_clk);
        // ---- trace row and momentum (the last stage stays) ----
        if (l == 0 && trace && C.iter < trace_cap) {
            double* tr = trace + ((size_t)b * trace_cap + C.iter) * SL1_TRACE_FIELDS;
            tr[0] = C.iter; tr[1] = C.stage; tr[2] = C.n_act; tr[3] = wpos;
            tr[4] = kt;
            tr[5] = Gp; tr[6] = Gt; tr[7] = delta; tr[8] = rule ? Rd : Rp; tr[9] = gam_t;
            tr[10] = C.l1; tr[11] = Pv; tr[12] = C.n_nz;
        }
        if (rnz > 0.0) {                  // a rejection that zeroed x_t[j]: momentum restarts
            C.ksince = 0;
            C.tau = 1.0;
        } else {
            C.ksince += 1;
            C.tau = tau_next;
        }
        C.iter += 1;
        C.par = 1 - par;
        C.n_act = wpos;
        C.n_nz = zpos;
        C.l1 = l1;
        n_act = wpos;
        n_nz = zpos;
        X = Xn;
    }
    if (l == 0) *sCp = C;
}

}  // namespace

__global__ __launch_bounds__(kWgBlock, 4) void k_solve_tail(const SolveParams* __restrict__ P0, int max_it) {
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    __shared__ Control sC;
    __shared__ Scalars sS;
    __shared__ double s_red[48];
    __shared__ double s_sum[4];
    __shared__ double s_kt[2];
    __shared__ double s_yy;
    __shared__ int s_cnt[2];
    __shared__ int s_w[kWgWaves * 4];
    __shared__ int s_done;
    __shared__ long long s_clk;

    if (tid == 0) {
        sC = P0->ctrl[2 * b];
        s_done = 0;
        s_clk = P0->wg_prof ? wall_clock64() : 0;
    }
    __syncthreads();
    if (sC.done) return;
    // state of the preserved set into LDS
    {
        const SolveParams* P = phase_params(P0);
        const int N = P->N, par = uni(sC.par), n_act = uni(sC.n_act), n_nz = uni(sC.n_nz);
        const StageDesc& st = P->st[uni(sC.stage)];
        const bool bad = st.kind != kDense || uni(sC.stage) != P->n_stages - 1 || P->wo_tail < 0 ||
                         P->wg_cap_nz < P->wg_cap_act || n_act > P->wg_cap_act || n_nz > P->wg_cap_nz ||
                         P->wg_cap_gram > 64 * 2 || (P->wg_cap_gram > 0 && P->wo_gram < 0);
        if (bad) {   // the host hands over only dense, small sets; anything else is refused
            if (tid == 0) {
                Final F;
                F.gap = 0.0;
                F.gap_cert = 0.0;
                F.iters = sC.iter;
                F.stage = sC.stage;
                F.status = SL1_ELIMIT;
                F.par = sC.par;
                F.t0 = sC.t0;
                F.tconv = 0;
                P->fin[b] = F;
                sC.done = 1;
                P->ctrl[2 * b] = sC;
                atomicSub(P->active_signals, 1);
            }
            return;
        }
        double* yl = (double*)(smem + P->wo_y);
        for (int i = tid; i < N; i += kWgBlock) yl[i] = yval(P, b, i);
        const TailState T = tail_state(smem, P);
        const int* act = actbuf(P, b, 0);
        const double* xc = xbuf(P, b, par);
        const double* xo = xbuf(P, b, 1 - par);
        const double* gprev = gbuf(P, b, 1 - par);
        for (int i = tid; i < n_act; i += kWgBlock) {
            const int j = act[i];
            T.la[i] = j;
            T.xt[i] = xc[j];
            T.xp[i] = xo[j];
            T.gm[i] = gprev[j];
            T.e[i] = st.eps[j];
            T.an[i] = P->atom_norm[j];
            T.atn[i] = st.at_norm[j];
            T.cy[i] = P->rule ? P->cy[(size_t)b * P->K + j] : 0.0;
        }
        const int* nzl = nzbuf(P, b, 0);
        int* lj = (int*)(smem + P->wo_lnj);
        double* lx = (double*)(smem + P->wo_lnx);
        for (int i = tid; i < n_nz; i += kWgBlock) {
            const int j = nzl[i];
            lj[i] = j;
            lx[i] = xc[j];
        }
        __syncthreads();
    }

    int it = 0;
    bool gram = false;
    for (; it < max_it; ++it) {
        const int par = uni(sC.par), n_nz = uni(sC.n_nz), n_act = uni(sC.n_act);
        if (P0->wg_cap_gram > 0 && n_act <= P0->wg_cap_gram) {
            gram = true;
            break;
        }
        // ---- forward product and residual ----
        {
            const SolveParams* P = phase_params(P0);
            const StageDesc& st = P->st[uni(sC.stage)];
            double* zd = (double*)(smem + P->wo_zd);
            const double* yl = (const double*)(smem + P->wo_y);
            char* scr = smem + P->wo_scr;
            const int* lj = (const int*)(smem + P->wo_lnj);
            const double* lx = (const double*)(smem + P->wo_lnx);
            if (st.dtype == SL1_F64) wg_dense_forward<true>(P, b, st, nullptr, nullptr, n_nz, lj, lx, true, zd, nullptr, yl, scr, s_red, s_sum);
            else wg_dense_forward<false>(P, b, st, nullptr, nullptr, n_nz, lj, lx, true, zd, nullptr, yl, scr, s_red, s_sum);
            __syncthreads();
            wg_stamp(P, b, 0, s_clk);
        }
        // ---- correlations, maxima of the stable dual scaling, scalars ----
        {
            const SolveParams* P = phase_params(P0);
            const int N = P->N;
            const StageDesc& st = P->st[uni(sC.stage)];
            const double* zd = (const double*)(smem + P->wo_zd);
            const double rz = uni(sqrt(s_sum[1]));
            const TailState T = tail_state(smem, P);
            double mx[3] = {0.0, 0.0, 0.0};
            if (N <= 1024) tail_adj<4>(st, N, T, n_act, zd, rz, mx);
            else tail_adj<1>(st, N, T, n_act, zd, rz, mx);
            block_max<3>(mx, s_red);
            if (tid == 0) {
                Scalars S;
                scalars_from(P, sC, s_sum[0], s_sum[1], s_sum[2], sqrt(s_sum[1]), mx[0], mx[1], mx[2],
                             P->rule ? P->yy[b] : 0.0, S);
                if (S.conv == 1) S.tconv = wall_clock64();
                sS = S;
            }
            __syncthreads();
            wg_stamp(P, b, 1, s_clk);
        }
        if (uni(sS.conv)) {
            // the final iterate x_t of the preserved atoms to global memory
            const SolveParams* P = phase_params(P0);
            const TailState T = tail_state(smem, P);
            double* xc = xbuf(P, b, par);
            for (int i = tid; i < n_act; i += kWgBlock) xc[T.la[i]] = T.xt[i];
            if (tid == 0) {
                Final F;
                F.gap = sS.Gt;
                F.gap_cert = sS.Gp + sS.delta;
                F.iters = sC.iter;
                F.stage = sC.stage;
                F.status = sS.conv == 2 ? SL1_MAXITER : SL1_OK;
                F.par = sC.par;
                F.t0 = sC.t0;
                F.tconv = sS.tconv;
                P->fin[b] = F;
                sC.done = 1;
                P->ctrl[2 * b] = sC;
                atomicSub(P->active_signals, 1);
            }
            return;
        }
        // ---- stable GAP test, look-ahead count, FISTA step, compaction (LDS) ----
        {
            const SolveParams* P = phase_params(P0);
            const int K = P->K;
            const StageDesc& st = P->st[uni(sC.stage)];
            const TailState T = tail_state(smem, P);
            int* lj = (int*)(smem + P->wo_lnj);
            double* lx = (double*)(smem + P->wo_lnx);
            uint8_t* mask = P->mask + (size_t)b * K;
            double* xc = xbuf(P, b, par);
            double* xo = xbuf(P, b, 1 - par);
            const double c1 = uni(sS.c1), c2 = uni(sS.c2), Rp = uni(sS.Rp), beta = uni(sS.beta);
            const double invL = st.invL, thr = uni(sC.lam) * st.invL, keep_min = 1.0 - P->margin;
            const int rule = P->rule;
            const double Rd = uni(sS.Rd), invlam = uni(1.0 / sC.lam), eyl = uni(sS.ny / sC.lam);
            const bool no_reject = uni(sC.iter) % P->screen_every != 0;
            int wpos = 0, zpos = 0;
            double sv[2] = {0.0, 0.0};   // look-ahead count K_t, ||x_{t+1}||_1
            for (int base = 0; base < n_act; base += kWgBlock) {
                const int i = base + tid;
                const bool valid = i < n_act;
                bool keep = false, nzf = false;
                int j = 0;
                double xn = 0.0, xt = 0.0, gt = 0.0, e = 0.0, an = 0.0, atn = 0.0, cy = 0.0;
                if (valid) {
                    j = T.la[i];
                    xt = T.xt[i];
                    gt = T.gt[i];
                    e = T.e[i];
                    an = T.an[i];
                    atn = T.atn[i];
                    cy = T.cy[i];
                    const double xp = T.xp[i];
                    const double gp = T.gm[i];
                    const double ag = fabs(gt);
                    if (rule) {
                        // stable Dynamic Safe: |a^T y| / lambda + ||theta' - y/lambda|| ||a||
                        const double c = fabs(cy) * invlam;
                        keep = c + e * eyl + Rd * an >= keep_min;
                        sv[0] += (c + Rd * atn >= 1.0) ? 1.0 : 0.0;
                    } else {
                        // stable GAP Safe: |a~^T theta'| + eps ||theta'|| + R' ||a||
                        keep = c1 * ag + e * c2 + Rp * an >= keep_min;
                        // look-ahead: conventional test on the approximate atom
                        sv[0] += (c1 * ag + Rp * atn >= 1.0) ? 1.0 : 0.0;
                    }
                    if (no_reject) keep = true;
                    // FISTA step from the two correlation vectors (gradient by linearity)
                    const double zpt = xt + beta * (xt - xp);
                    const double hh = (1.0 + beta) * gt - beta * gp;
                    const double v = zpt + hh * invL;
                    if (keep) xn = (v > thr) ? v - thr : ((v < -thr) ? v + thr : 0.0);
                    if (!keep) {         // screened: its coefficient is zero in both iterates
                        xc[j] = 0.0;
                        xo[j] = 0.0;
                        mask[j] = 0;
                        if (xt != 0.0) sv[0] += kRejNz;
                    }
                    nzf = keep && (xn != 0.0);
                    sv[1] += fabs(xn);
                }
                // every read of this part of the state precedes the in-place writes
                __syncthreads();
                const bool fl[2] = {keep, nzf};
                int ps[2], ts[2];
                wg_scan_flags<2>(fl, s_w, ps, ts);
                const int pk = ps[0], pz = ps[1], tk = ts[0], tz = ts[1];
                if (keep) {
                    const int q = wpos + pk;
                    T.la[q] = j;
                    T.xt[q] = xn;        // x_{t+1}
                    T.xp[q] = xt;        // x_t
                    T.gm[q] = gt;        // g_t
                    T.e[q] = e;
                    T.an[q] = an;
                    T.atn[q] = atn;
                    T.cy[q] = cy;
                }
                if (nzf) {
                    lj[zpos + pz] = j;
                    lx[zpos + pz] = xn;
                }
                wpos += tk;
                zpos += tz;
            }
            block_sum<2>(sv, s_red);
            if (tid == 0) {
                s_kt[0] = sv[0];
                s_kt[1] = sv[1];
                s_cnt[0] = wpos;
                s_cnt[1] = zpos;
            }
            __syncthreads();
            wg_stamp(P, b, 3, s_clk);
        }
        // ---- trace row and momentum (thread 0; the last stage stays) ----
        if (tid == 0) {
            const SolveParams* P = phase_params(P0);
            Control C = sC;
            // rejected nonzero coefficients travel above the look-ahead count
            const double rnz = floor(s_kt[0] / kRejNz);
            if (P->trace && C.iter < P->trace_cap) {
                double* tr = P->trace + ((size_t)b * P->trace_cap + C.iter) * SL1_TRACE_FIELDS;
                tr[0] = C.iter; tr[1] = C.stage; tr[2] = C.n_act; tr[3] = s_cnt[0];
                tr[4] = s_kt[0] - rnz * kRejNz;
                tr[5] = sS.Gp; tr[6] = sS.Gt; tr[7] = sS.delta; tr[8] = P->rule ? sS.Rd : sS.Rp; tr[9] = sS.gamma;
                tr[10] = C.l1; tr[11] = sS.P; tr[12] = C.n_nz;
            }
            if (rnz > 0.0) {               // a rejection that zeroed x_t[j]: momentum restarts
                C.ksince = 0;
                C.tau = 1.0;
            } else {
                C.ksince += 1;
                C.tau = sS.tau_next;
            }
            C.iter += 1;
            C.par = 1 - C.par;
            C.n_act = s_cnt[0];
            C.n_nz = s_cnt[1];
            C.l1 = s_kt[1];
            sC = C;
        }
        __syncthreads();
    }
    if (gram) {
        {
            const SolveParams* P = phase_params(P0);
            tail_gram_build(P, b, P->st[uni(sC.stage)], smem, uni(sC.n_act), s_red, &s_yy);
        }
        if (tid < 64) tail_gram_loop<2>(P0, b, it, max_it, smem, &sC, &s_done, &s_clk, s_yy);
        __syncthreads();
        if (s_done) return;
    }
    // the launch ends before the signal stops: state back to global memory
    {
        const SolveParams* P = phase_params(P0);
        const int par = uni(sC.par), n_act = uni(sC.n_act), n_nz = uni(sC.n_nz);
        const TailState T = tail_state(smem, P);
        const int* lj = (const int*)(smem + P->wo_lnj);
        int* act = actbuf(P, b, 0);
        int* nzl = nzbuf(P, b, 0);
        double* xc = xbuf(P, b, par);
        double* xo = xbuf(P, b, 1 - par);
        double* gprev = gbuf(P, b, 1 - par);
        for (int i = tid; i < n_act; i += kWgBlock) {
            const int j = T.la[i];
            act[i] = j;
            xc[j] = T.xt[i];
            xo[j] = T.xp[i];
            gprev[j] = T.gm[i];
        }
        if (gram) {
            // the Gram loop keeps no nonzero list: the positions with x_t != 0, in order
            int base_nz = 0;
            for (int base = 0; base < n_act; base += kWgBlock) {
                const int i = base + tid;
                const bool f[1] = {i < n_act && T.xt[i] != 0.0};
                int pos[1], tot[1];
                wg_scan_flags<1>(f, s_w, pos, tot);
                if (f[0]) nzl[base_nz + pos[0]] = T.la[i];
                base_nz += tot[0];
            }
        } else {
            for (int i = tid; i < n_nz; i += kWgBlock) nzl[i] = lj[i];
        }
        if (tid == 0) P->ctrl[2 * b] = sC;
    }
}

// ---------------------------------------------------------------------------
// hand-over from the per-iteration grid kernels: the state C_t of control slot
// `slot` (slot 0 after a forward launch has formed it with the segment prefixes
// of its two lists; slot 1 after a chunk of step launches, whose state of
// iteration t waits for its update, which the tail redoes from the top of the
// iteration) goes to slot 0, where the tail kernel reads it, and the segmented
// lists of buffer C.par are copied into contiguous lists in buffer 0,
// the layout of the whole-solve kernel.  Segments go in increasing order, each
// read completely before it is written, so the in-place case (par = 0) is safe:
// a segment's destination never reaches a later segment's source.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSeg) void k_to_wg(const SolveParams* __restrict__ P, int slot) {
    const int b = blockIdx.x;
    const Control C = P->ctrl[2 * b + slot];
    if (slot != 0 && threadIdx.x == 0) P->ctrl[2 * b] = C;     // the tail reads slot 0
    if (C.done) return;
    const int par = uni(C.par);
    for (int which = 0; which < 2; ++which) {
        const int nseg = uni(which ? C.nseg_nz : C.nseg_act);
        const int* pre = which ? nzpre(P, b, par) : actpre(P, b, par);
        const int* src = which ? nzbuf(P, b, par) : actbuf(P, b, par);
        int* dst = which ? nzbuf(P, b, 0) : actbuf(P, b, 0);
        for (int sg = 0; sg < nseg; ++sg) {
            const int p0 = pre[sg], cnt = pre[sg + 1] - p0;
            int v = 0;
            if ((int)threadIdx.x < cnt) v = src[(size_t)sg * kSeg + threadIdx.x];
            __syncthreads();
            if ((int)threadIdx.x < cnt) dst[p0 + threadIdx.x] = v;
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// After a whole-solve phase that parked signals at the last stage: the
// statistics the host's hand-over decisions read (the same four as the grid
// kernels' per-chunk reduction: max and sum of |A_t|, signals not yet on the
// park stage, signals that qualify for the batched correlation product).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_wg_stat(const SolveParams* __restrict__ P) {
    __shared__ int s_v[4][kBlock / 64];
    const int park = P->wg_park;
    int v[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < P->batch; b += kBlock) {
        const Control& C = P->ctrl[2 * b];
        if (C.done) continue;
        const bool on_last = C.stage == P->n_stages - 1;
        v[0] = max(v[0], C.n_act);
        v[1] += C.n_act;
        v[2] += C.stage < park ? 1 : 0;
        v[3] += (P->gemm_min > 0 && on_last && P->st[C.stage].kind == kDense && C.n_act >= P->gemm_min) ? 1 : 0;
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

// ---------------------------------------------------------------------------
// Whole-solve state -> grid state, one block per signal.  The whole-solve kernel
// keeps contiguous lists in slot 0 and reads x from its buffers; the grid kernels
// read segmented lists of the iterate's parity with prefix counts and the
// nonzero values beside the nonzero list.  A contiguous list is a segmented one
// whose segment s starts at min(kSeg s, n), so the lists only move when the
// parity is 1.  The state enters both control slots with advance = 0: the next
// forward launch (slot 0, reading slot 1) takes it as is, like the state of the
// initialisation kernel.  Each block reads only its own signal's slot-0 lists
// before writing its slot-1 lists (disjoint buffers).
// ---------------------------------------------------------------------------
// mode 0: every signal; mode 1: a live signal short of stage `park` is marked absent
// instead (the grid kernels leave it alone while a whole-solve launch beside them
// goes on with it); mode 2: the absent signals only, which join the grid kernels.
__global__ __launch_bounds__(kSeg) void k_wg_to_grid(const SolveParams* __restrict__ P, int mode, int park) {
    const int b = blockIdx.x, batch = P->batch;
    if (mode == 2 && !P->absent[b]) return;
    __shared__ Control s_c;
    if (threadIdx.x == 0) s_c = P->ctrl[2 * b];
    __syncthreads();
    Control C = s_c;
    if (mode == 1 && !C.done && C.stage < park) {
        if (threadIdx.x == 0) {
            P->absent[b] = 1;
            P->cnt_fwd[b] = 0;
            P->cnt_fwd[(size_t)batch + b] = 0;
            P->cnt_adj[b] = 0;
            P->cnt_adjk[b] = 0;
            P->cnt_adjf[b] = 0;
            P->cnt_upd[b] = 0;
            P->cnt_gemm[b] = 0;
            *(int4*)(P->sig_stat + 4 * b) = make_int4(0, 0, 0, 0);
        }
        return;
    }
    if (threadIdx.x == 0) P->absent[b] = 0;
    if (C.done) {
        if (threadIdx.x == 0) {
            P->ctrl[2 * b + 1] = C;
            P->cnt_fwd[b] = 0;
            P->cnt_fwd[(size_t)batch + b] = 0;
            *(int4*)(P->sig_stat + 4 * b) = make_int4(0, 0, 0, 0);
        }
        return;
    }
    const int par = uni(C.par), n_act = uni(C.n_act), n_nz = uni(C.n_nz);
    const int nseg_act = max(1, (n_act + kSeg - 1) / kSeg);
    const int nseg_nz = (n_nz + kSeg - 1) / kSeg;
    const int* a0 = actbuf(P, b, 0);
    const int* z0 = nzbuf(P, b, 0);
    int* a1 = actbuf(P, b, par);
    int* z1 = nzbuf(P, b, par);
    double* zx = nzxbuf(P, b, par);
    const double* x = xbuf(P, b, par);
    for (int i = threadIdx.x; i < n_act; i += kSeg) {
        const int j = a0[i];
        if (par) a1[i] = j;
    }
    for (int i = threadIdx.x; i < n_nz; i += kSeg) {
        const int j = z0[i];
        if (par) z1[i] = j;
        zx[i] = x[j];
    }
    int* ap = actpre(P, b, par);
    int* zp = nzpre(P, b, par);
    for (int q = threadIdx.x; q <= nseg_act; q += kSeg) ap[q] = min(q * kSeg, n_act);
    for (int q = threadIdx.x; q <= nseg_nz; q += kSeg) zp[q] = min(q * kSeg, n_nz);
    if (threadIdx.x == 0) {
        C.advance = 0;
        C.nslot = 0;
        C.nseg_act = nseg_act;
        C.nseg_nz = nseg_nz;
        P->ctrl[2 * b + 0] = C;
        P->ctrl[2 * b + 1] = C;
        P->cnt_fwd[b] = P->nrc;                       // slot 0
        P->cnt_fwd[(size_t)batch + b] = 0;            // slot 1
        P->cnt_adj[b] = 0;
        P->cnt_adjk[b] = 0;
        P->cnt_adjf[b] = 0;
        P->cnt_upd[b] = 0;
        P->cnt_gemm[b] = 0;
        *(int4*)(P->sig_stat + 4 * b) = make_int4(n_act, n_act, C.stage < P->n_stages - 1 ? 1 : 0, 0);
    }
}

hipError_t launch_wg_stat(const SolveParams* dP, hipStream_t s) {
    hipLaunchKernelGGL(k_wg_stat, dim3(1), dim3(kBlock), 0, s, dP);
    return hipGetLastError();
}

hipError_t launch_wg_to_grid(const SolveParams* dP, int batch, hipStream_t s, int mode, int park) {
    hipLaunchKernelGGL(k_wg_to_grid, dim3(batch), dim3(kSeg), 0, s, dP, mode, park);
    return hipGetLastError();
}

hipError_t launch_to_wg(const SolveParams* dP, int batch, int slot, hipStream_t s) {
    hipLaunchKernelGGL(k_to_wg, dim3(batch), dim3(kSeg), 0, s, dP, slot);
    return hipGetLastError();
}

hipError_t launch_solve_tail(const SolveParams* dP, int batch, size_t lds, int max_it, hipStream_t s) {
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_solve_tail, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_solve_tail, dim3(batch), dim3(kWgBlock), lds, s, dP, max_it);
    return hipGetLastError();
}

hipError_t launch_solve_wg(const SolveParams* dP, int batch, size_t lds, int max_it, hipStream_t s) {
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute((const void*)k_solve_wg, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_solve_wg, dim3(batch), dim3(kWgBlock), lds, s, dP, max_it);
    return hipGetLastError();
}

}  // namespace sl1
