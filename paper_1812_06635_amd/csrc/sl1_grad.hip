// Implicit adjoint of the Lasso solution map on the final support.
//
// On the support S of x* with signs s, the optimality conditions of Section II
// read A_S^T (y - A_S x_S) = lambda s, hence x_S = G^{-1} (A_S^T y - lambda s) with
// G = A_S^T A_S, and for an incoming gradient v = dL/dx:
//   dL/dy = A_S G^{-1} v_S,   dL/dlambda = -s^T G^{-1} v_S.
// Steps (FP64): compact S per signal, build G (one block per row), Cholesky
// factorisation and two triangular solves (one block per signal, every thread
// taking part), then A_S w.
#include <algorithm>
#include <mutex>
#include <vector>

#include "sl1_device.hpp"

namespace sl1 {

constexpr int kGradMaxSupport = 1024;

struct GradDict {
    int dtype, N, K;
    const void* A;
    const float* scale;
};

__device__ __forceinline__ double atom_elem(const GradDict& d, int j, int i) {
    const size_t idx = (size_t)j * d.N + i;
    double v;
    switch (d.dtype) {
        case SL1_F64: v = ((const double*)d.A)[idx]; break;
        case SL1_F32: v = (double)((const float*)d.A)[idx]; break;
        case SL1_BF16: v = (double)bf16_to_f(((const uint16_t*)d.A)[idx]); break;
        default: {
            const uint32_t q = ((const uint8_t*)d.A)[idx];
            auto f = __builtin_amdgcn_cvt_pk_f32_fp8((int)q, false);
            v = (double)f[0];
        }
    }
    return d.scale ? v * (double)d.scale[j] : v;
}

__global__ __launch_bounds__(kBlock) void k_grad_support(const double* x, int K, int* sidx, int* cnt, double* sgn) {
    const int b = blockIdx.x;
    const double* xb = x + (size_t)b * K;
    __shared__ int s_w[4];
    __shared__ int s_base;
    if (threadIdx.x == 0) s_base = 0;
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int j0 = 0; j0 < K; j0 += kBlock) {
        const int j = j0 + threadIdx.x;
        const double v = j < K ? xb[j] : 0.0;
        const bool f = v != 0.0;
        const unsigned long long bal = __ballot(f);
        const int pre = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) s_w[w] = __popcll(bal);
        __syncthreads();
        int base = s_base;
        for (int k = 0; k < w; ++k) base += s_w[k];
        const int pos = base + pre;
        if (f && pos < kGradMaxSupport) {
            sidx[(size_t)b * kGradMaxSupport + pos] = j;
            sgn[(size_t)b * kGradMaxSupport + pos] = v > 0 ? 1.0 : -1.0;
        }
        __syncthreads();
        if (threadIdx.x == 0) s_base += s_w[0] + s_w[1] + s_w[2] + s_w[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) cnt[b] = s_base;
}

// Row p of G = A_S^T A_S for signal b (grid: (kGradMaxSupport, batch)).
__global__ __launch_bounds__(kBlock) void k_grad_gram(GradDict d, const int* sidx, const int* cnt, double* G, int ld) {
    extern __shared__ __align__(16) char smem[];
    const int b = blockIdx.y, p = blockIdx.x;
    const int s = cnt[b];
    if (s > kGradMaxSupport || p >= s) return;
    double* ap = (double*)smem;
    const int jp = sidx[(size_t)b * kGradMaxSupport + p];
    for (int i = threadIdx.x; i < d.N; i += kBlock) ap[i] = atom_elem(d, jp, i);
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = w; q <= p; q += 4) {
        const int jq = sidx[(size_t)b * kGradMaxSupport + q];
        double acc = 0.0;
        for (int i = lane; i < d.N; i += 64) acc += ap[i] * atom_elem(d, jq, i);
        acc = wave_sum(acc);
        if (lane == 0) {
            G[((size_t)b * ld + p) * ld + q] = acc;
            G[((size_t)b * ld + q) * ld + p] = acc;
        }
    }
}

// In-place Cholesky G = L L^T (lower), then L L^T w = v; one block per signal.
// Right-looking factorisation: per column k the pivot, the column scaled, then the
// trailing lower triangle (pairs j <= i, spread over the block); the substitutions
// are column-oriented (per k: w_k /= L_kk, then every thread updates its w_i), the
// right-hand side and the solution in LDS.
__global__ __launch_bounds__(kBlock) void k_grad_solve(const int* sidx, const int* cnt, const double* sgn, double* G,
                                                      const double* dx, int K, double* wout, double* dlam, int* flag,
                                                      int ld) {
    const int b = blockIdx.x;
    const int s = cnt[b];
    if (s > kGradMaxSupport) {
        if (threadIdx.x == 0) atomicOr(flag, 2);
        return;
    }
    double* Gb = G + (size_t)b * ld * ld;
    __shared__ double s_w[kGradMaxSupport];
    __shared__ double s_piv, s_red[48];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    for (int i = threadIdx.x; i < s; i += kBlock) s_w[i] = dx[(size_t)b * K + sidx[(size_t)b * kGradMaxSupport + i]];
    double gm = 0.0;
    for (int k = threadIdx.x; k < s; k += kBlock) gm = fmax(gm, fabs(Gb[(size_t)k * ld + k]));
    double gmv[1] = {gm};
    block_max<1>(gmv, s_red);
    const double gmax = gmv[0];
    for (int k = 0; k < s; ++k) {
        if (threadIdx.x == 0) {
            const double d = Gb[(size_t)k * ld + k];
            if (!(d > 1e-13 * gmax)) s_bad = 1;
            s_piv = sqrt(fmax(d, 1e-300));
            Gb[(size_t)k * ld + k] = s_piv;
        }
        __syncthreads();
        const double piv = s_piv;
        for (int i = k + 1 + threadIdx.x; i < s; i += kBlock) Gb[(size_t)i * ld + k] /= piv;
        __syncthreads();
        // trailing update G[i][j] -= L[i][k] L[j][k] over k < j <= i < s: pair t = i' (i' + 1) / 2 + j'
        const int m = s - k - 1;
        const long long pairs = (long long)m * (m + 1) / 2;
        for (long long t = threadIdx.x; t < pairs; t += kBlock) {
            int ii = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
            while ((long long)ii * (ii + 1) / 2 > t) --ii;
            while ((long long)(ii + 1) * (ii + 2) / 2 <= t) ++ii;
            const int jj = (int)(t - (long long)ii * (ii + 1) / 2);
            const int i = k + 1 + ii, j = k + 1 + jj;
            Gb[(size_t)i * ld + j] -= Gb[(size_t)i * ld + k] * Gb[(size_t)j * ld + k];
        }
        __syncthreads();
    }
    // forward: L u = v_S
    for (int k = 0; k < s; ++k) {
        if (threadIdx.x == 0) s_w[k] /= Gb[(size_t)k * ld + k];
        __syncthreads();
        const double wk = s_w[k];
        for (int i = k + 1 + threadIdx.x; i < s; i += kBlock) s_w[i] -= Gb[(size_t)i * ld + k] * wk;
        __syncthreads();
    }
    // backward: L^T w = u
    for (int k = s - 1; k >= 0; --k) {
        if (threadIdx.x == 0) s_w[k] /= Gb[(size_t)k * ld + k];
        __syncthreads();
        const double wk = s_w[k];
        for (int i = threadIdx.x; i < k; i += kBlock) s_w[i] -= Gb[(size_t)k * ld + i] * wk;
        __syncthreads();
    }
    double* w = wout + (size_t)b * ld;
    double dl[1] = {0.0};
    for (int i = threadIdx.x; i < s; i += kBlock) {
        w[i] = s_w[i];
        dl[0] -= sgn[(size_t)b * kGradMaxSupport + i] * s_w[i];
    }
    block_sum<1>(dl, s_red);
    if (threadIdx.x == 0) {
        if (s_bad) atomicOr(flag, 1);
        dlam[b] = dl[0];
    }
}

template <typename W>
__global__ __launch_bounds__(kBlock) void k_grad_dy(GradDict d, const int* sidx, const int* cnt, const double* wv,
                                                   W* dy, int ld) {
    const int b = blockIdx.y;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int s = min(cnt[b], kGradMaxSupport);
    if (i >= d.N) return;
    double acc = 0.0;
    for (int p = 0; p < s; ++p)
        acc += wv[(size_t)b * ld + p] * atom_elem(d, sidx[(size_t)b * kGradMaxSupport + p], i);
    dy[(size_t)b * d.N + i] = (W)acc;
}

}  // namespace sl1

struct sl1_dict_s;
extern "C" int sl1_grad_impl_dense_info(sl1_dict_s* d, int* kind, int* dtype, int64_t* N, int64_t* K,
                                        const void** A, const float** scale);

using namespace sl1;

// Device memory of the gradient, per device: grown to the largest call and kept
// until the process ends (calls on one device are serialised by its mutex).
namespace {
constexpr int kGradDevices = 64;
struct GradWs {
    std::mutex mu;
    char* mem1 = nullptr;
    size_t cap1 = 0;
    char* mem2 = nullptr;
    size_t cap2 = 0;
};
GradWs g_grad_ws[kGradDevices];

int grad_reserve(char*& mem, size_t& cap, size_t bytes) {
    if (bytes <= cap) return SL1_OK;
    if (mem) (void)hipFree(mem);
    mem = nullptr;
    cap = 0;
    if (hipMalloc(&mem, bytes) != hipSuccess) {
        mem = nullptr;
        return SL1_ENOMEM;
    }
    cap = bytes;
    return SL1_OK;
}
}  // namespace

extern "C" int sl1_grad(sl1_dict A, int64_t batch, const double* x, const void* y, const double* lambda,
                        const double* dx, void* dy, double* dlambda, int y_dtype, void* stream) {
    (void)y;
    (void)lambda;
    if (!A || !x || !dx || !dy || !dlambda || batch < 1) return SL1_EINVAL;
    if (y_dtype != SL1_F64 && y_dtype != SL1_F32) return SL1_EDTYPE;
    int kind = 0, dtype = 0;
    int64_t N = 0, K = 0;
    const void* Ap = nullptr;
    const float* sc = nullptr;
    int st = sl1_grad_impl_dense_info(A, &kind, &dtype, &N, &K, &Ap, &sc);
    if (st != SL1_OK) return st;
    if (kind != 0) return SL1_EDTYPE;
    if (N * 8 > 64 * 1024) return SL1_ELIMIT;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kGradDevices) return SL1_EHIP;
    GradWs& ws = g_grad_ws[dev];
    std::lock_guard<std::mutex> lock(ws.mu);
    const size_t B = batch, M = kGradMaxSupport;
    const size_t bytes1 = B * M * 4 + B * 4 + 16 + B * M * 8 + 64;
    if (grad_reserve(ws.mem1, ws.cap1, bytes1) != SL1_OK) return SL1_ENOMEM;
    char* mem = ws.mem1;
    int* sidx = (int*)mem;
    int* cnt = (int*)(mem + B * M * 4);
    double* sgn = (double*)(((uintptr_t)(cnt + B) + 15) & ~(uintptr_t)15);
    int* flag = (int*)(sgn + B * M);
    GradDict gd{dtype, (int)N, (int)K, Ap, sc};
    const bool f64 = y_dtype == SL1_F64;
    if (hipMemsetAsync(flag, 0, 4, s) != hipSuccess) return SL1_EHIP;
    hipLaunchKernelGGL(k_grad_support, dim3(B), dim3(kBlock), 0, s, x, (int)K, sidx, cnt, sgn);
    std::vector<int> hc(B);
    if (hipMemcpyAsync(hc.data(), cnt, B * 4, hipMemcpyDeviceToHost, s) != hipSuccess) return SL1_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return SL1_EHIP;
    int smax = 1;
    for (int c : hc) {
        if (c > kGradMaxSupport || c > N) return SL1_ELIMIT;
        smax = std::max(smax, c);
    }
    const int ld = smax;
    if (grad_reserve(ws.mem2, ws.cap2, B * (size_t)ld * ld * 8 + B * (size_t)ld * 8) != SL1_OK) return SL1_ENOMEM;
    double* G = (double*)ws.mem2;
    double* wv = G + B * (size_t)ld * ld;
    hipLaunchKernelGGL(k_grad_gram, dim3(smax, B), dim3(kBlock), N * 8, s, gd, sidx, cnt, G, ld);
    hipLaunchKernelGGL(k_grad_solve, dim3(B), dim3(kBlock), 0, s, sidx, cnt, sgn, G, dx, (int)K, wv, dlambda, flag, ld);
    if (f64) hipLaunchKernelGGL(k_grad_dy<double>, dim3((N + kBlock - 1) / kBlock, B), dim3(kBlock), 0, s, gd, sidx, cnt, wv, (double*)dy, ld);
    else hipLaunchKernelGGL(k_grad_dy<float>, dim3((N + kBlock - 1) / kBlock, B), dim3(kBlock), 0, s, gd, sidx, cnt, wv, (float*)dy, ld);
    if (hipGetLastError() != hipSuccess) return SL1_EHIP;
    int hflag = 0;
    if (hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return SL1_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return SL1_EHIP;
    if (hflag & 2) return SL1_ELIMIT;
    if (hflag & 1) return SL1_ESINGULAR;
    return SL1_OK;
}
