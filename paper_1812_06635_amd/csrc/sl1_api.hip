// C ABI of the stablel1 library: dictionary handles, workspaces, the solve
// driver (iteration chunks replayed from a captured hipGraph, convergence polled
// between chunks), lambda'_max and relative-complexity measurement.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "sl1_internal.hpp"

namespace sl1 {
hipError_t launch_init(const SolveParams*, const LaunchCfg&, hipStream_t);
hipError_t launch_iter(int, const SolveParams*, const LaunchCfg&, hipStream_t);
hipError_t launch_fwd_adj(const SolveParams*, const LaunchCfg&, hipStream_t);
hipError_t launch_one(int, int, const SolveParams*, const LaunchCfg&, hipStream_t);
hipError_t launch_adj_only(const SolveParams*, const LaunchCfg&, hipStream_t);
hipError_t launch_finalize(const SolveParams*, const LaunchCfg&, double*, double*, double*, uint8_t*, int32_t*,
                           int32_t*, int32_t*, hipStream_t);
hipError_t launch_lambda_out(const SolveParams*, int, double*, int32_t*, hipStream_t);
hipError_t launch_time_out(const SolveParams*, int, long long*, hipStream_t);
hipError_t launch_adjoint_out(const SolveParams*, int, int, int, double*, double*, hipStream_t);
hipError_t launch_ysq(const SolveParams*, int, double*, hipStream_t);
hipError_t launch_stat(const SolveParams*, hipStream_t);
hipError_t launch_init_x0(const SolveParams*, int, const double*, hipStream_t);
int upd_resident_blocks(size_t);
int adj_resident_blocks(size_t);
hipError_t gemm_lds_attr(size_t);
hipError_t fwd_lds_attr(size_t);
hipError_t adjk_lds_attr(size_t);
hipError_t adjf_lds_attr(size_t);
hipError_t launch_dense_norms(int, const void*, const float*, int, int, const double*, double, double*, double*,
                              int*, hipStream_t);
hipError_t launch_eps_fold(const double*, const double*, double, int, double*, int*, hipStream_t);
hipError_t launch_solve_wg(const SolveParams*, int, size_t, int, hipStream_t);
hipError_t launch_solve_tail(const SolveParams*, int, size_t, int, hipStream_t);
hipError_t launch_to_wg(const SolveParams*, int, int, hipStream_t);
hipError_t launch_wg_stat(const SolveParams*, hipStream_t);
hipError_t launch_wg_to_grid(const SolveParams*, int, hipStream_t, int, int);
hipError_t launch_zero(void*, size_t, hipStream_t);
}  // namespace sl1

using namespace sl1;

struct sl1_dict_s {
    int kind = 0, dtype = 0, device = 0;
    int64_t N = 0, K = 0;
    int R = 0, n1 = 0, k1 = 0, n2 = 0, k2 = 0, vec = 4;
    int kt2 = 16, kt1 = 16;    // Kronecker correlation tile shape (sl1_tune_kron may change it)
    const void* A = nullptr;   // borrowed (dense)
    float* scale = nullptr;    // owned
    void* B = nullptr;         // owned (kron)
    void* C = nullptr;         // owned (kron)
    double* eps_eff = nullptr; // owned
    double* at_norm = nullptr; // owned
    // FAuST (owned): device descriptor and the concatenated CSR arrays of the
    // factors and of their transposes
    FaustDesc* fa = nullptr;
    int* fa_ptr = nullptr;
    int* fa_idx = nullptr;
    void* fa_val = nullptr;
    int* fa_tptr = nullptr;
    int* fa_tidx = nullptr;
    void* fa_tval = nullptr;
    int fa_maxd = 0, fa_q = 0, fa_dlast = 0;
    double eps_max_in = 0.0, eps_max_eff = 0.0, at_norm_max = 0.0, rc_model = 1.0;
    double q = 2.0;            // norm of the error bounds (1 <= q <= inf)
};

// The allocation-free solve's workspace: one fixed array per device, kept until the
// process ends.  Host code never passes `scratch` itself to a kernel or a copy (in
// host code it names a host-side stand-in); it uses the device address that
// hipGetSymbolAddress returns, taken once per device with that device current.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

#define HIP_TRY(x)                                   \
    do {                                             \
        hipError_t e_ = (x);                         \
        if (e_ != hipSuccess) return SL1_EHIP;       \
    } while (0)

namespace {

constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53
constexpr double kU32 = 5.9604644775390625e-08;  // 2^-24

size_t dtype_size(int dt) {
    switch (dt) {
        case SL1_F64: return 8;
        case SL1_F32: return 4;
        case SL1_BF16: return 2;
        case SL1_FP8_E4M3: return 1;
    }
    return 0;
}

double bf16_host(uint16_t b) {
    uint32_t u = ((uint32_t)b) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}

// OCP FP8 E4M3FN code -> value (bias 7, subnormals m 2^-9, 0x7F / 0xFF are NaN)
double fp8_host(uint8_t b) {
    const int e = (b >> 3) & 15, m = b & 7;
    double v;
    if (e == 15 && m == 7) v = std::nan("");
    else if (e == 0) v = std::ldexp((double)m, -9);
    else v = std::ldexp(1.0 + m / 8.0, e - 7);
    return (b & 0x80) ? -v : v;
}

// Bound on |computed - exact| of both products with a stage, per unit
// ||abs-atom||_2 ||vector||_2 (standard gamma_n = n u accumulation bounds, doubled
// to cover any order or internal precision of the matrix-core accumulation).
// The allowances bound a correlation's rounding by kappa (|a~_j|^T |z|) <= kappa ||a~_j||_2 ||z||_2;
// against l_q bounds, which pair with ||z||_{q*}, ||z||_2 <= N^((1/q - 1/2)_+) ||z||_{q*}.
double bound_norm_factor(const sl1_dict_s& d) {
    const double e = std::isinf(d.q) ? -0.5 : 1.0 / d.q - 0.5;
    return e > 0.0 ? std::pow((double)d.N, e) : 1.0;
}

// q of an l_q bound: 1 <= q <= inf (NaN rejected)
bool valid_bound_norm(double q) { return q >= 1.0; }

double rounding_allowance(const sl1_dict_s& d) {
    const double N = (double)d.N, K = (double)d.K;
    if (d.kind == kDense) return 2.0 * (N + K + 32.0) * kU64;
    const double n1 = d.n1, n2 = d.n2, R = d.R;
    if (d.dtype == SL1_F64) return 2.0 * (n2 + R * n1 + R + K + 32.0) * kU64;
    if (d.dtype == SL1_F32) return 2.0 * (n2 + R * n1 + R + 10.0) * kU32 + 2.0 * (K + 24.0) * kU64;
    // BF16 (and FP8 factors, decoded exactly to BF16 for the same products): exact first
    // product inputs, FP32 accumulation, hi/lo split of the intermediate (residual
    // <= 2^-18, counted as 2^-16)
    return 2.0 * (n2 + 2.0 * R * n1 + R + 10.0) * kU32 + 1.52587890625e-05 + 2.0 * (K + 24.0) * kU64;
}

struct Workspace {
    int device = 0, batch = 0, N = 0, K = 0;
    int nseg_max = 0, nrc = 0, nadj_max = 0;
    void* mem = nullptr;
    SolveParams* dP = nullptr;
    SolveParams* hP = nullptr;   // pinned
    int* d_active = nullptr;
    int* h_active = nullptr;     // pinned
    int32_t* d_status = nullptr;
    long long* d_times = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_a = nullptr, ev_b = nullptr;
    // a second stream for a whole-solve launch beside the grid kernels (its params
    // in dP2), with the events that order the two and time it
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_j = nullptr, ev_k = nullptr, ev_c = nullptr, ev_d = nullptr;
    SolveParams* dP2 = nullptr;
    // captured chunks of grid iterations, one per launch set: bit 0 with the
    // Kronecker correlation launch, bit 1 with the batched correlation product
    hipGraphExec_t graph[8] = {};           // chunk graphs by launch set (Kronecker, product, step)
    int graph_chunk[8] = {};
    LaunchCfg graph_cfg[8] = {};
    int last_gram_cap = 0;    // Gram capacity of the last hybrid tail (0: none)
    double* d_cy = nullptr;   // stable Dynamic Safe: [batch][K] a^T y on the exact dictionary (lazy)
    double* d_yy = nullptr;   // [batch] ||y||^2
    double prof_ms[kGridKernels] = {};      // grid kernels: forward, dense / Kronecker correlations, update,
    long long prof_n[kGridKernels] = {};    // batched correlations and their finishing pass
    int last_gemm_min = 0;                  // |A_t| threshold of the batched correlations (0: off)
    long long* d_wgprof = nullptr;          // [batch][kWgPhases] phase clocks of the whole-solve engine
    double phase_ms[kWgPhases] = {0, 0, 0, 0};
    double wg_ms = 0.0;                     // whole-solve launches of the last profiled solve
    long long wg_n = 0;
    double park_phase_ms[kWgPhases] = {0, 0, 0, 0};   // the part of those of the Kronecker phase
    double park_ms = 0.0;
    long long park_n = 0;                   // and their number (with a launch beside the grid kernels)
    int last_engine = 0;
    std::vector<hipEvent_t> prof_ev;
    std::mutex mu;
    // a view over memory this object does not own (device memory, host blocks and the
    // stream belong to the caller); it records no graphs or events
    bool borrowed = false;
    ~Workspace() {
        if (borrowed) return;
        for (auto& g : graph)
            if (g) (void)hipGraphExecDestroy(g);
        if (mem) (void)hipFree(mem);
        if (d_cy) (void)hipFree(d_cy);
        if (d_yy) (void)hipFree(d_yy);
        if (hP) (void)hipHostFree(hP);
        if (h_active) (void)hipHostFree(h_active);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (ev_a) (void)hipEventDestroy(ev_a);
        if (ev_b) (void)hipEventDestroy(ev_b);
        for (hipEvent_t e : {ev_j, ev_k, ev_c, ev_d})
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : prof_ev) (void)hipEventDestroy(e);
        if (stream2) (void)hipStreamDestroy(stream2);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

std::mutex g_ws_mu;
// Workspaces are shared: every call holds its own reference for its whole duration,
// so dropping a cached entry never frees memory, a stream or a mutex still in use.
std::map<std::tuple<int, int, int, int>, std::shared_ptr<Workspace>> g_ws;

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// Byte layout of a workspace for (w.batch, w.N, w.K) in one device allocation; with
// m != nullptr the solver's pointers into it are set in p and w.  Returns its size.
size_t workspace_layout(Workspace& w, char* m, SolveParams* pp) {
    const size_t ws = 8;
    const size_t B = w.batch, K = w.K, N = w.N;
    w.nseg_max = (w.K + kSeg - 1) / kSeg;
    w.nrc = (w.N + kFwdRows - 1) / kFwdRows;
    w.nadj_max = std::max(1, (w.K + 3) / 4);   // dense correlation items hold >= 4 atoms
    const size_t np = w.nseg_max + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += al(bytes); return o; };
    const size_t o_ctrl = take(B * 2 * sizeof(Control));
    const size_t o_sc = take(B * sizeof(Scalars));
    const size_t o_fin = take(B * sizeof(Final));
    const size_t o_x = take(B * 2 * K * ws);
    const size_t o_g = take(B * 2 * K * 8);
    const size_t o_mask = take(B * K);
    const size_t o_act = take(B * 2 * K * 4);
    const size_t o_nz = take(B * 2 * K * 4);
    const size_t o_nzx = take(B * 2 * K * 8);
    const size_t o_ap = take(B * 2 * np * 4);
    const size_t o_zp = take(B * 2 * np * 4);
    const size_t o_z = take(B * N * ws);
    const size_t o_rp = take(B * w.nrc * 3 * 8);
    const size_t o_zq = take(B * 8);
    const size_t o_adp = take(B * w.nadj_max * 4 * 3 * 8);
    const size_t o_up = take(B * w.nseg_max * 4 * 8);
    const size_t o_cnt = take(B * 12 * 4);
    const size_t o_fw = take(B * kFaustMaxDim * 8);
    const size_t o_gpart = take((size_t)kGemmSplitUnits * kGemmAtoms * kGemmSig * 8);
    const size_t o_act_sig = take(64);
    const size_t o_status = take(B * 4);
    const size_t o_times = take(B * 16);
    const size_t o_wgprof = take(B * kWgPhases * 8);
    const size_t o_params = take(sizeof(SolveParams));
    const size_t o_params2 = take(sizeof(SolveParams));
    if (!m) return off;
    SolveParams& p = *pp;
    p.ctrl = (Control*)(m + o_ctrl);
    p.sc = (Scalars*)(m + o_sc);
    p.fin = (Final*)(m + o_fin);
    p.x = (double*)(m + o_x);
    p.g = (double*)(m + o_g);
    p.mask = (uint8_t*)(m + o_mask);
    p.act = (int*)(m + o_act);
    p.nz = (int*)(m + o_nz);
    p.nzx = (double*)(m + o_nzx);
    p.act_pre = (int*)(m + o_ap);
    p.nz_pre = (int*)(m + o_zp);
    p.z = (double*)(m + o_z);
    p.res_part = (double*)(m + o_rp);
    p.zq = (double*)(m + o_zq);
    p.adj_part = (double*)(m + o_adp);
    p.upd_part = (double*)(m + o_up);
    p.cnt_fwd = (int*)(m + o_cnt);
    p.cnt_adj = p.cnt_fwd + 2 * B;
    p.cnt_adjk = p.cnt_adj + B;
    p.cnt_upd = p.cnt_adjk + B;
    p.cnt_gemm = p.cnt_upd + B;
    p.sig_stat = p.cnt_gemm + B;
    p.cnt_adjf = p.sig_stat + 4 * B;
    p.absent = p.cnt_adjf + B;
    p.fw = (double*)(m + o_fw);
    p.gemm_part = (double*)(m + o_gpart);
    p.active_signals = (int*)(m + o_act_sig);
    p.stat = p.active_signals + 4;
    p.nseg_max = w.nseg_max;
    p.nrc = w.nrc;
    p.nadj_max = w.nadj_max;
    w.d_active = p.active_signals;
    w.d_status = (int32_t*)(m + o_status);
    w.d_times = (long long*)(m + o_times);
    w.d_wgprof = (long long*)(m + o_wgprof);
    w.dP = (SolveParams*)(m + o_params);
    w.dP2 = (SolveParams*)(m + o_params2);
    return off;
}

int make_workspace(Workspace& w) {
    const size_t bytes = workspace_layout(w, nullptr, nullptr);
    if (hipMalloc(&w.mem, bytes) != hipSuccess) return SL1_ENOMEM;
    if (hipHostMalloc((void**)&w.hP, sizeof(SolveParams), hipHostMallocDefault) != hipSuccess) return SL1_ENOMEM;
    if (hipHostMalloc((void**)&w.h_active, 64, hipHostMallocDefault) != hipSuccess) return SL1_ENOMEM;
    std::memset(w.hP, 0, sizeof(SolveParams));
    workspace_layout(w, (char*)w.mem, w.hP);
    if (hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) != hipSuccess) return SL1_EHIP;
    if (hipEventCreateWithFlags(&w.ev_in, hipEventDisableTiming) != hipSuccess) return SL1_EHIP;
    if (hipEventCreateWithFlags(&w.ev_out, hipEventDisableTiming) != hipSuccess) return SL1_EHIP;
    if (hipEventCreate(&w.ev_a) != hipSuccess) return SL1_EHIP;
    if (hipEventCreate(&w.ev_b) != hipSuccess) return SL1_EHIP;
    if (hipStreamCreateWithFlags(&w.stream2, hipStreamNonBlocking) != hipSuccess) return SL1_EHIP;
    if (hipEventCreateWithFlags(&w.ev_j, hipEventDisableTiming) != hipSuccess) return SL1_EHIP;
    if (hipEventCreateWithFlags(&w.ev_k, hipEventDisableTiming) != hipSuccess) return SL1_EHIP;
    if (hipEventCreate(&w.ev_c) != hipSuccess) return SL1_EHIP;
    if (hipEventCreate(&w.ev_d) != hipSuccess) return SL1_EHIP;
    if (hipMemsetAsync(w.mem, 0, bytes, w.stream) != hipSuccess) return SL1_EHIP;
    if (hipStreamSynchronize(w.stream) != hipSuccess) return SL1_EHIP;
    return SL1_OK;
}

// Orders the library stream after the caller's stream (a workspace on the
// caller's own stream needs nothing), and back.
int order_after(Workspace* w, hipStream_t us) {
    if (w->ev_in) {
        HIP_TRY(hipEventRecord(w->ev_in, us));
        HIP_TRY(hipStreamWaitEvent(w->stream, w->ev_in, 0));
    }
    return SL1_OK;
}
int order_before(Workspace* w, hipStream_t us) {
    if (w->ev_out) {
        HIP_TRY(hipEventRecord(w->ev_out, w->stream));
        HIP_TRY(hipStreamWaitEvent(us, w->ev_out, 0));
    }
    return SL1_OK;
}

// Clears n bytes of workspace memory: hipMemsetAsync on the library's own stream,
// a fill kernel on a borrowed workspace (which runs on the caller's stream).
hipError_t clear_ws(Workspace* w, void* p, size_t n) {
    return w->borrowed ? launch_zero(p, n, w->stream) : hipMemsetAsync(p, 0, n, w->stream);
}

// Every per-signal status of the last finalisation or lambda pass, read in fixed-size
// pieces: the most negative one (an error) or SL1_MAXITER if any signal stopped at the cap.
int read_statuses(Workspace* w, int64_t batch) {
    int32_t hs[256];
    int result = SL1_OK;
    for (int64_t b0 = 0; b0 < batch; b0 += 256) {
        const int64_t n = std::min<int64_t>(256, batch - b0);
        HIP_TRY(hipMemcpyAsync(hs, w->d_status + b0, n * 4, hipMemcpyDeviceToHost, w->stream));
        HIP_TRY(hipStreamSynchronize(w->stream));
        for (int64_t i = 0; i < n; ++i) {
            if (hs[i] < 0) return hs[i];
            if (hs[i] == SL1_MAXITER) result = SL1_MAXITER;
        }
    }
    return result;
}

int get_workspace(int device, int batch, int N, int K, std::shared_ptr<Workspace>* out) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto key = std::make_tuple(device, batch, N, K);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) {
        *out = it->second;
        return SL1_OK;
    }
    // keep the cache small: drop idle workspaces of other shapes on this device.  An
    // entry is idle when the cache holds its only reference (new references are made
    // only here, under g_ws_mu); one in use by a concurrent call stays.
    for (auto i = g_ws.begin(); i != g_ws.end();) {
        if (std::get<0>(i->first) == device && g_ws.size() >= 4 && i->second.use_count() == 1) i = g_ws.erase(i);
        else ++i;
    }
    auto w = std::make_shared<Workspace>();
    w->device = device;
    w->batch = batch;
    w->N = N;
    w->K = K;
    int st = make_workspace(*w);
    if (st != SL1_OK) return st;
    *out = w;
    g_ws[key] = std::move(w);
    return SL1_OK;
}

void fill_stage(StageDesc& s, const sl1_dict_s& d, double L, double rc) {
    std::memset(&s, 0, sizeof(s));
    s.kind = d.kind;
    s.dtype = d.dtype;
    s.R = d.R;
    s.n1 = d.n1;
    s.k1 = d.k1;
    s.n2 = d.n2;
    s.k2 = d.k2;
    s.kt2 = d.kt2;
    s.kt1 = d.kt1;
    s.vec = d.vec;
    s.A = d.A;
    s.scale = d.scale;
    s.B = d.B;
    s.C = d.C;
    s.eps = d.eps_eff;
    s.at_norm = d.at_norm;
    s.fa = d.fa;
    s.fa_items = d.kind == kFaust ? (int)((d.K + kFaustAtoms - 1) / kFaustAtoms) : 0;
    s.fa_maxd = d.fa_maxd;
    s.fa_dlast = d.fa_dlast;
    s.L = L;
    s.invL = 1.0 / L;
    s.rc = rc;
    s.at_norm_max = d.at_norm_max;
    s.eps_max = d.eps_max_eff;
    // l_q bounds: the dual exponent q* and the l2 constant N^((1/2 - 1/q)_+)
    s.qmode = d.q == 2.0 ? 0 : (d.q == 1.0 ? 2 : (std::isinf(d.q) ? 3 : 1));
    s.qd = d.q == 1.0 ? INFINITY : (std::isinf(d.q) ? 1.0 : d.q / (d.q - 1.0));
    s.cq = d.q > 2.0 ? std::pow((double)d.N, std::isinf(d.q) ? 0.5 : 0.5 - 1.0 / d.q) : 1.0;
}

// Bytes of the V region of a Kronecker correlation item: R terms x kt2 rows x n1
// (FP64 for FP64 factors; FP32, or a BF16 hi + lo pair, otherwise).
size_t kron_v_bytes(int dtype, int R, int kt2, int n1) {
    return (size_t)R * kt2 * n1 * (dtype == SL1_F64 ? 8 : 4);
}

// A tile shape (kt2 x kt1 atoms per item) is usable when it divides the atom grid and
// its V region fits.
bool kron_shape_ok(const sl1_dict_s& d, int kt2, int kt1) {
    return kt2 >= 16 && kt1 >= 16 && kt2 % 16 == 0 && kt1 % 16 == 0 && d.k2 % kt2 == 0 && d.k1 % kt1 == 0 &&
           kron_v_bytes(d.dtype, d.R, kt2, d.n1) <= (size_t)kKronVLds;
}

// Shape before any tuning: items of at least 4 output tiles (one per wave) where the
// grid allows, 64 columns j1 at most.
void kron_default_shape(sl1_dict_s& d) {
    int kt1 = 16;
    for (int c : {64, 32, 16})
        if (d.k1 % c == 0) { kt1 = c; break; }
    int kt2 = 16;
    for (int r = 16; r <= d.k2; r += 16)
        if (d.k2 % r == 0 && kron_shape_ok(d, r, kt1)) {
            kt2 = r;
            if (r * kt1 >= 1024) break;
        }
    d.kt2 = kt2;
    d.kt1 = kt1;
}

LaunchCfg launch_cfg(const Workspace& w, const SolveParams& p) {
    LaunchCfg c{};
    c.batch = w.batch;
    c.nseg_max = w.nseg_max;
    c.nrc = w.nrc;
    c.nadj_max = w.nadj_max;
    const size_t ws = 8;
    const size_t nseg1 = (size_t)w.nseg_max + 1, nb1 = (size_t)w.batch + 1;
    c.lds_fwd = 4 * (2 * nseg1 + kFwdBlock + nb1) + 16 + kFwdBlock * 8 + 4 * 256 * 8 + (size_t)p.fwd_fac_lds;
    c.lds_upd = 4 * (nseg1 + nb1);
    c.lds_step = 4 * ((nseg1 + 3) & ~(size_t)3) + 4 * kFwdBlock + 16 + 8 * kFwdBlock + 8 * 4 * 256;
    // persistent grids: enough blocks to fill the chip, never more than the work;
    // a correlation kernel whose stage kind is absent is not launched
    bool dense = false;
    int kron_items = 0, faust_tiles = 0, faust_groups = 0;
    size_t extra = 0, faust_lds = 0;
    for (int i = 0; i < p.n_stages; ++i) {
        const StageDesc& s = p.st[i];
        if (s.kind == kDense) {
            dense = true;
            continue;
        }
        if (s.kind == kFaust) {      // FAuST correlations: their own launch, all signals of a tile at once
            faust_tiles = std::max(faust_tiles, s.fa_items);
            const int dl = s.fa_dlast;
            const int sg = faust_group(dl);
            faust_groups = std::max(faust_groups, (w.batch + sg - 1) / sg);
            faust_lds = std::max(faust_lds, faust_lds_bytes(dl, sg, w.batch));
            continue;
        }
        kron_items = std::max(kron_items, (s.k2 / s.kt2) * (s.k1 / s.kt1));
        extra = std::max(extra, kron_v_bytes(s.dtype, s.R, s.kt2, s.n1));
    }
    c.g_fwd = (int)std::min<long long>((long long)w.batch * w.nrc, 512);
    c.dome = p.rule == 2 ? 1 : 0;
    c.g_lq = 0;
    for (int i = 0; i < p.n_stages; ++i)
        if (p.st[i].qmode != 0) c.g_lq = w.batch;
    c.g_adjk = kron_items ? (int)std::min<long long>((long long)w.batch * kron_items, 1024) : 0;
    c.adjf_x = faust_tiles;
    c.adjf_y = faust_tiles ? faust_groups : 0;
    c.adjf_z = faust_tiles ? p.n_stages : 0;
    c.lds_adjf = faust_lds;
    // update: one resident round of blocks (each block takes a contiguous range of items)
#ifdef SL1_UPD_GRID
    const int upd_cap = SL1_UPD_GRID;
#else
    const int upd_res = upd_resident_blocks(c.lds_upd);
    const int upd_cap = upd_res > 0 ? std::min(upd_res, 4096) : 1024;
#endif
    c.g_upd = (int)std::min<long long>((long long)w.batch * w.nseg_max, upd_cap);
    const size_t zb = ((size_t)w.N * ws + 15) & ~(size_t)15;
    c.lds_adj = zb + 4 * (nseg1 + nb1);
    // streaming correlations: one resident round of blocks (each block pays its
    // signal's set-up once and then takes a contiguous range of items; a second
    // round would pay it again: 1024 blocks against 2048 took the launch on the
    // 512-signal Kronecker workload from 29 to 27 us)
    const int adj_res = adj_resident_blocks(c.lds_adj);
    c.g_adj = dense ? (int)std::min<long long>((long long)w.batch * w.nadj_max, adj_res > 0 ? adj_res : 1024) : 0;
    c.lds_adjk = zb + ((4 * nb1 + 15) & ~(size_t)15) + extra;
    // batched correlations on a dense exact stage: one block per (64-signal, 64-atom)
    // tile, or per row split of a tile while the tiles are few (up to kGemmMaxSplit
    // splits, kGemmSplitUnits partial tiles); two LDS buffers of a 32-row chunk of
    // A (room for FP64) and z, + the flag prefix and signal list
    c.lds_gemm = 2 * ((size_t)kGemmAtoms * 33 * 2 * 4 + (size_t)kGemmSig * 33 * 8) + 4 * (2 * (size_t)w.batch + 1);
    const bool last_dense = p.n_stages > 0 && p.st[p.n_stages - 1].kind == kDense;
    const long long tiles_max = (long long)((w.batch + kGemmSig - 1) / kGemmSig) * ((w.K + kGemmAtoms - 1) / kGemmAtoms);
    const long long g_split = std::min<long long>(tiles_max * kGemmMaxSplit, kGemmSplitUnits);
    c.g_gemm = (last_dense && c.lds_gemm <= 159 * 1024) ? (int)std::min<long long>(std::max(tiles_max, g_split), 1024) : 0;
    return c;
}

// |A_t| from which a signal on the exact dense stage joins the batched correlation
// product, which forms all K correlations: at least K/8 preserved atoms and 4a per
// 64-atom tile (a = atoms per wave of the streaming kernel).
int gemm_min_atoms(const SolveParams& p) {
    const int per = 4 * (p.N <= 1024 ? 2 : 1);     // the documented gate, independent of the stream kernel's width
    return std::max(per * ((p.K + kGemmAtoms - 1) / kGemmAtoms), std::max(1, p.K / 8));
}

bool cfg_equal(const LaunchCfg& a, const LaunchCfg& b) {
    if (a.adjf_x != b.adjf_x || a.adjf_y != b.adjf_y || a.adjf_z != b.adjf_z || a.lds_adjf != b.lds_adjf) return false;
    return a.batch == b.batch && a.nseg_max == b.nseg_max && a.nrc == b.nrc && a.nadj_max == b.nadj_max &&
           a.g_fwd == b.g_fwd && a.g_adj == b.g_adj && a.g_adjk == b.g_adjk && a.g_upd == b.g_upd &&
           a.g_gemm == b.g_gemm && a.g_lq == b.g_lq && a.dome == b.dome && a.lds_fwd == b.lds_fwd && a.lds_adj == b.lds_adj &&
           a.lds_adjk == b.lds_adjk && a.lds_upd == b.lds_upd && a.lds_gemm == b.lds_gemm && a.step == b.step &&
           a.lds_step == b.lds_step;
}

int check_lds(const LaunchCfg& c) {
    const size_t lim = 160 * 1024;
    if (c.lds_adj > lim || c.lds_adjk > lim || c.lds_fwd > lim) return SL1_ELIMIT;
    return SL1_OK;
}

// LDS layout of the whole-solve kernel; sets the region offsets in p and
// returns the dynamic LDS bytes (0: does not fit).
//   full: z (FP64 and FP32), the largest Kronecker stage's factors, a scratch
//         (forward staging; with Kronecker stages also the cross-wave sums and
//         the intermediate V), then y and the two lists when two workgroups per
//         CU can still share the LDS;
//   tail: every live signal on the last, dense, stage with at most max_act
//         preserved atoms: z (FP64), an 8 KB scratch, y, both lists of max_act
//         entries and the per-position state of the preserved set; with gram,
//         the Gram region (G, c, row atoms) overlays z, the scratch and y, its
//         capacity the largest multiple of 16 up to 128 that keeps two
//         workgroups per CU when the batch needs them.
size_t wg_layout(SolveParams& p, bool tail, int max_act, bool gram) {
    auto a16 = [](size_t x) { return (x + 15) & ~(size_t)15; };
    const size_t lim = 160 * 1024 - 1024;       // static LDS of the kernel stays below 1 KB
    const size_t two_per_cu = 79 * 1024;
    size_t off = 0;
    auto put = [&](size_t bytes) {
        const size_t o = off;
        off += a16(bytes);
        return (int)std::min<size_t>(o, (size_t)INT32_MAX);
    };
    const size_t N = (size_t)p.N;
    p.wo_gram = -1;
    p.wg_cap_gram = 0;
    p.wo_zd = put(N * 8);
    if (tail) {
        const int cap = std::max(64, (max_act + 63) & ~63);
        p.wo_zf = p.wo_fac = -1;
        p.wo_scr = put(8192);                    // the dense forward's cross-group sums
        p.wo_y = put(N * 8);
        const size_t colbuf = off;
        const size_t lists = a16((size_t)cap * 4) + a16((size_t)cap * 8) + a16((size_t)cap * 4) +
                             a16((size_t)cap * (8 * 8 + 4));
        auto gbytes = [&](size_t g) { return a16(g * g * 8) + a16(g * 8) + a16(g * 4); };
        if (gram) {
            const size_t target = (p.batch > 256 && colbuf + lists <= two_per_cu) ? two_per_cu : lim;
            for (int g = 128; g >= 16; g -= 16) {
                if (std::max(colbuf, gbytes((size_t)g)) + lists <= target) {
                    p.wg_cap_gram = g;
                    p.wo_gram = 0;
                    off = std::max(colbuf, gbytes((size_t)g));
                    break;
                }
            }
        }
        p.wg_cap_nz = p.wg_cap_act = cap;
        p.wo_lnj = put((size_t)cap * 4);
        p.wo_lnx = put((size_t)cap * 8);
        p.wo_lact = put((size_t)cap * 4);
        p.wo_tail = put((size_t)cap * (8 * 8 + 4));
        return off <= lim ? off : 0;
    }
    p.wo_tail = -1;
    size_t fac = 0, scr = 8192;                 // forward staging (6 KB) or cross-group sums (8 KB)
    for (int i = 0; i < p.n_stages; ++i) {
        const StageDesc& s = p.st[i];
        if (s.kind == kFaust) return 0;         // FAuST stages run in the grid kernels only
        if (s.qmode != 0) return 0;             // so do stages with l_q bounds, q != 2
        if (s.kind != kKron) continue;
        if (s.dtype == SL1_FP8_E4M3) return 0;  // and Kronecker stages with FP8 factors
        const size_t es = s.dtype == SL1_F64 ? 8 : (s.dtype == SL1_F32 ? 4 : 2);
        fac = std::max(fac, a16(((size_t)s.R * s.k1 * s.n1 + (size_t)s.R * s.k2 * s.n2) * es));
        const size_t v = (size_t)s.R * s.k2 * s.n1 * (s.dtype == SL1_F64 ? 8 : 4);   // BF16: hi + lo
        scr = std::max(scr, std::max(a16(v), (size_t)(kWgWaves / 2) * 16 * 64 * 8));
    }
    p.wo_zf = put(N * 4);
    p.wo_fac = fac ? put(fac) : -1;
    p.wo_scr = put(scr);
    const int cap_nz = 256, cap_act = 512;
    const size_t extra = a16(N * 8) + a16((size_t)cap_nz * 12) + a16((size_t)cap_act * 4);
    if (off + extra <= two_per_cu) {
        p.wo_y = put(N * 8);
        p.wg_cap_nz = cap_nz;
        p.wg_cap_act = cap_act;
        p.wo_lnj = put((size_t)cap_nz * 4);
        p.wo_lnx = put((size_t)cap_nz * 8);
        p.wo_lact = put((size_t)cap_act * 4);
    } else {
        p.wo_y = -1;
        p.wg_cap_nz = p.wg_cap_act = 0;
        p.wo_lnj = p.wo_lnx = p.wo_lact = 0;     // never dereferenced with capacity 0
    }
    return off <= lim ? off : 0;
}

// Iterations per whole-solve launch: bounded so that one launch streams at most
// ~8 GB of dense dictionary per workgroup; the host relaunches while signals remain.
int wg_iters_per_launch(const SolveParams& p) {
    size_t es = 0;
    for (int i = 0; i < p.n_stages; ++i)
        if (p.st[i].kind == kDense) es = std::max(es, p.st[i].dtype == SL1_F64 ? (size_t)8 : (size_t)4);
    if (es == 0) return 4096;
    const double per = (double)p.N * (double)p.K * (double)es;
    return (int)std::max(1.0, std::min(4096.0, 8.0e9 / per));
}

int current_device(int* dev) {
    return hipGetDevice(dev) == hipSuccess ? SL1_OK : SL1_EHIP;
}

// Common validation of a stage sequence; fills the host params.
int prepare(const sl1_dict* seq, int n_stages, const double* L, const double* rc, int y_dtype, SolveParams& p) {
    if (!seq || n_stages < 1) return SL1_EINVAL;
    if (n_stages > SL1_MAX_STAGES) return SL1_ELIMIT;
    if (y_dtype != SL1_F64 && y_dtype != SL1_F32) return SL1_EDTYPE;
    const sl1_dict_s* d0 = seq[0];
    if (!d0) return SL1_EINVAL;
    int n1_max = 0;
    size_t fac = 0;
    for (int i = 0; i < n_stages; ++i) {
        const sl1_dict_s* d = seq[i];
        if (!d) return SL1_EINVAL;
        if (d->N != d0->N || d->K != d0->K || d->device != d0->device) return SL1_ESHAPE;
        const double Li = L ? L[i] : 0.0;
        if (!(Li > 0.0) || !std::isfinite(Li)) return SL1_EINVAL;
        const double rci = rc ? rc[i] : d->rc_model;
        if (!std::isfinite(rci)) return SL1_EINVAL;
        fill_stage(p.st[i], *d, Li, rci);
        if (d->kind == kKron) {
            n1_max = std::max(n1_max, d->n1);
            // the forward kernel stages a Kronecker stage's factors in LDS when they fit
            const size_t es = dtype_size(d->dtype);
            const size_t fb = (size_t)d->R * ((size_t)d->n1 * d->k1 + (size_t)d->n2 * d->k2) * es;
            if (fb <= (size_t)kFwdFacLds) fac = std::max(fac, fb);
        }
        if (d->kind == kFaust) {    // the forward chain's vectors, scatter block and column bounds; then
                                    // z and the two vectors of the adjoint's chain
            fac = std::max(fac, (2 * (size_t)d->fa_maxd + (size_t)d->fa_dlast * d->fa_q) * 8 + 2 * (size_t)kFwdBlock * 4);
            fac = std::max(fac, 3 * (size_t)d->fa_maxd * 8);
        }
    }
    p.fwd_fac_lds = (int)fac;
    p.n_stages = n_stages;
    p.N = (int)d0->N;
    p.K = (int)d0->K;
    p.y_f64 = y_dtype == SL1_F64;
    p.n1_max = n1_max;
    return SL1_OK;
}

#ifndef SL1_HYBRID_BYTES
#define SL1_HYBRID_BYTES (2 << 20)
#endif
// Largest preserved set (atoms) at which the hybrid solve moves to the whole-solve
// kernel: one CU then streams at most SL1_HYBRID_BYTES of dense columns per iteration.
int hybrid_atoms(const SolveParams& p) {
    size_t es = 0;
    for (int i = 0; i < p.n_stages; ++i)
        if (p.st[i].kind == kDense) es = std::max(es, p.st[i].dtype == SL1_F64 ? (size_t)8 : (size_t)4);
    if (es == 0) return p.K;
    return (int)std::max<size_t>(16, (size_t)SL1_HYBRID_BYTES / ((size_t)p.N * es));
}

// Whole-solve launches until every signal stopped (or the iteration cap, counting
// the `done` iterations already run by the grid kernels); tail: the hybrid
// solve's kernel for the last, dense, stage with LDS-resident per-atom state;
// parking (p.wg_park >= 0): whole-solve launches until every live signal has
// reached the park stage, or until at most p.wg_park_allow have not (they stop where
// they are), with the hand-over statistics in h_active[4..7].
// Profile: launch times and per-signal phase clocks.
enum WgMode { kWgWhole = 0, kWgTail = 1, kWgPark = 2 };
int run_wg(Workspace* w, const SolveParams& p, const sl1_opts& o, int64_t batch, size_t wlds, bool prof, int dev,
           long long done, int mode) {
    const int per = std::min(wg_iters_per_launch(p), 256 * (o.chunk > 0 ? o.chunk : 16));
    const long long cap = (long long)o.max_iter + 1;
    long long launched = done;
    for (;;) {
        if (prof) HIP_TRY(hipEventRecord(w->ev_a, w->stream));
        if (mode == kWgTail) HIP_TRY(launch_solve_tail(w->dP, (int)batch, wlds, per, w->stream));
        else HIP_TRY(launch_solve_wg(w->dP, (int)batch, wlds, per, w->stream));
        if (prof) HIP_TRY(hipEventRecord(w->ev_b, w->stream));
        launched += per;
        if (mode == kWgPark) HIP_TRY(launch_wg_stat(w->dP, w->stream));
        HIP_TRY(hipMemcpyAsync(w->h_active, w->d_active, mode == kWgPark ? 36 : 4, hipMemcpyDeviceToHost,
                               w->stream));
        HIP_TRY(hipStreamSynchronize(w->stream));
        if (prof) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, w->ev_a, w->ev_b));
            w->wg_ms += ms;
            w->wg_n += 1;
            if (mode == kWgPark) {
                w->park_ms += ms;
                w->park_n += 1;
            }
        }
        if (*w->h_active <= 0 || launched >= cap) break;
        // the park phase ends when every live signal has reached the park stage, or when
        // at most wg_park_allow are short of it (those stopped where they were)
        if (mode == kWgPark && (w->h_active[4 + 2] <= p.wg_park_allow ||
                                w->h_active[0] - w->h_active[8] <= p.wg_park_allow))
            break;
    }
    if (prof) {
        std::vector<long long> ticks((size_t)batch * kWgPhases);
        HIP_TRY(hipMemcpy(ticks.data(), w->d_wgprof, ticks.size() * 8, hipMemcpyDeviceToHost));
        int khz = 0;
        HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        for (int64_t b = 0; b < batch; ++b)
            for (int k = 0; k < kWgPhases; ++k) {
                const double v = (double)ticks[b * kWgPhases + k] / khz;
                if (mode == kWgPark) w->park_phase_ms[k] += v;
                else w->phase_ms[k] += v;
            }
    }
    return SL1_OK;
}

// outputs of a solve, per-signal statuses, hand-back to the caller's stream
// captures `chunk` grid iterations with the launch set of ccfg into graph slot v
int capture_chunk(Workspace* w, const LaunchCfg& ccfg, int chunk, int v) {
    if (w->graph[v]) {
        HIP_TRY(hipGraphExecDestroy(w->graph[v]));
        w->graph[v] = nullptr;
    }
    HIP_TRY(hipStreamSynchronize(w->stream));
    hipStream_t cs;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g;
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < chunk; ++k) {
        if (launch_iter(k & 1, w->dP, ccfg, cs) != hipSuccess) {
            (void)hipStreamEndCapture(cs, &g);
            (void)hipStreamDestroy(cs);
            return SL1_EHIP;
        }
    }
    HIP_TRY(hipStreamEndCapture(cs, &g));
    HIP_TRY(hipStreamDestroy(cs));
    hipError_t e = hipGraphInstantiate(&w->graph[v], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        w->graph[v] = nullptr;
        return SL1_EHIP;
    }
    w->graph_chunk[v] = chunk;
    w->graph_cfg[v] = ccfg;
    return SL1_OK;
}

int finish_solve(Workspace* w, const LaunchCfg& cfg, int64_t batch, double* x, double* gap, double* gap_cert,
                 uint8_t* screened, int32_t* iters, int32_t* stage, hipStream_t us) {
    HIP_TRY(launch_finalize(w->dP, cfg, x, gap, gap_cert, screened, iters, stage, w->d_status, w->stream));
    int result = read_statuses(w, batch);
    const int ord = order_before(w, us);
    if (result < 0) return result;
    if (ord != SL1_OK) return ord;
    if (*w->h_active > 0) result = SL1_MAXITER;
    return result;
}

}  // namespace

extern "C" {

const char* sl1_version(void) { return "stablel1 0.1.0 (gfx950)"; }

const char* sl1_status_str(int s) {
    switch (s) {
        case SL1_OK: return "ok";
        case SL1_MAXITER: return "iteration cap reached before the duality-gap tolerance";
        case SL1_EINVAL: return "invalid argument value";
        case SL1_ESHAPE: return "inconsistent sizes";
        case SL1_EDTYPE: return "unsupported data type combination";
        case SL1_EHIP: return "HIP runtime error";
        case SL1_ENOMEM: return "allocation failed";
        case SL1_ESINGULAR: return "singular support Gram matrix";
        case SL1_ELIMIT: return "outside an implementation limit";
    }
    return "unknown status";
}

static_assert(sizeof(sl1_opts) == 72, "sl1_opts layout (mirrored by the Python binding)");

int sl1_opts_default(sl1_opts* o) {
    if (!o) return SL1_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->Gamma = 0.5;
    o->tol = 1e-6;
    o->margin = 1e-12;
    o->max_iter = 100000;
    o->y_dtype = SL1_F32;
    o->chunk = 16;
    o->flags = 0;
    o->trace = nullptr;
    o->trace_cap = 0;
    o->screen_every = 1;
    o->gemm_signals = kGemmMinSignals;
    o->x0 = nullptr;
    return SL1_OK;
}

int sl1_dict_free(sl1_dict d) {
    if (!d) return SL1_OK;
    if (d->scale) (void)hipFree(d->scale);
    if (d->B) (void)hipFree(d->B);
    if (d->C) (void)hipFree(d->C);
    if (d->eps_eff) (void)hipFree(d->eps_eff);
    if (d->at_norm) (void)hipFree(d->at_norm);
    for (void* q : {(void*)d->fa, (void*)d->fa_ptr, (void*)d->fa_idx, d->fa_val, (void*)d->fa_tptr,
                    (void*)d->fa_tidx, d->fa_tval})
        if (q) (void)hipFree(q);
    delete d;
    return SL1_OK;
}

int sl1_dict_info(sl1_dict d, int64_t* N, int64_t* K, double* eps_max, double* rc_model) {
    if (!d) return SL1_EINVAL;
    if (N) *N = d->N;
    if (K) *K = d->K;
    if (eps_max) *eps_max = d->eps_max_in;
    if (rc_model) *rc_model = d->rc_model;
    return SL1_OK;
}

static int finish_dict_host_eps(sl1_dict_s* d, const double* eps, hipStream_t s) {
    std::vector<double> h(d->K);
    HIP_TRY(hipMemcpyAsync(h.data(), eps, d->K * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double m = 0.0;
    for (double e : h) {
        if (!(e >= 0.0) || !std::isfinite(e)) return SL1_EINVAL;
        m = std::max(m, e);
    }
    d->eps_max_in = m;
    return SL1_OK;
}

int sl1_dict_dense(sl1_dict* out, int dtype, int64_t N, int64_t K, const void* A, const float* col_scale,
                   const double* eps, double q, void* stream) {
    if (!out) return SL1_EINVAL;
    *out = nullptr;
    if (!A || !eps || N < 1 || K < 1 || !valid_bound_norm(q)) return SL1_EINVAL;
    if (dtype_size(dtype) == 0) return SL1_EDTYPE;
    if (N % 4 != 0 || N > kMaxN || K > (int64_t)kMaxSeg * kSeg) return SL1_ELIMIT;
    hipStream_t s = (hipStream_t)stream;
    auto d = std::make_unique<sl1_dict_s>();
    HIP_TRY(hipGetDevice(&d->device));
    d->kind = kDense;
    d->dtype = dtype;
    d->N = N;
    d->K = K;
    d->A = A;
    d->q = q;
    if (dtype == SL1_F64 || dtype == SL1_F32) d->vec = 4;
    else if (dtype == SL1_BF16) d->vec = (N % 8 == 0) ? 8 : 4;
    else d->vec = (N % 16 == 0) ? 16 : 4;
    int st = finish_dict_host_eps(d.get(), eps, s);
    if (st != SL1_OK) return st;
    if (col_scale) {
        if (hipMalloc(&d->scale, K * sizeof(float)) != hipSuccess) return SL1_ENOMEM;
        HIP_TRY(hipMemcpyAsync(d->scale, col_scale, K * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    if (hipMalloc(&d->eps_eff, K * 8) != hipSuccess || hipMalloc(&d->at_norm, K * 8) != hipSuccess) {
        sl1_dict_free(d.release());
        return SL1_ENOMEM;
    }
    int* bad = nullptr;
    if (hipMalloc(&bad, 4) != hipSuccess) return SL1_ENOMEM;
    HIP_TRY(hipMemsetAsync(bad, 0, 4, s));
    const double kappa = rounding_allowance(*d) * bound_norm_factor(*d);
    HIP_TRY(launch_dense_norms(dtype, A, d->scale, (int)N, (int)K, eps, kappa, d->at_norm, d->eps_eff, bad, s));
    int hbad = 0;
    std::vector<double> an(K), ee(K);
    HIP_TRY(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(an.data(), d->at_norm, K * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ee.data(), d->eps_eff, K * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    (void)hipFree(bad);
    if (hbad) {
        sl1_dict_free(d.release());
        return SL1_EINVAL;
    }
    d->at_norm_max = *std::max_element(an.begin(), an.end());
    d->eps_max_eff = *std::max_element(ee.begin(), ee.end());
    d->rc_model = dtype == SL1_BF16 ? 0.5 : (dtype == SL1_FP8_E4M3 ? 0.25 : 1.0);
    *out = d.release();
    return SL1_OK;
}

int sl1_dict_kron(sl1_dict* out, int dtype, int R, int n1, int k1, int n2, int k2, const void* B, const void* C,
                  const double* eps, double q, void* stream) {
    if (!out) return SL1_EINVAL;
    *out = nullptr;
    if (!B || !C || !eps || R < 1 || n1 < 1 || k1 < 1 || n2 < 1 || k2 < 1 || !valid_bound_norm(q)) return SL1_EINVAL;
    if (dtype != SL1_F64 && dtype != SL1_F32 && dtype != SL1_BF16 && dtype != SL1_FP8_E4M3) return SL1_EDTYPE;
    if (n1 % 16 || k1 % 16 || n2 % 16 || k2 % 16) return SL1_ELIMIT;
    const int64_t N = (int64_t)n1 * n2, K = (int64_t)k1 * k2;
    if (N > kMaxN || n1 > (dtype == SL1_F64 ? 128 : 256) || K > (int64_t)kMaxSeg * kSeg) return SL1_ELIMIT;
    hipStream_t s = (hipStream_t)stream;
    auto d = std::make_unique<sl1_dict_s>();
    HIP_TRY(hipGetDevice(&d->device));
    d->kind = kKron;
    d->dtype = dtype;
    d->N = N;
    d->K = K;
    d->q = q;
    d->R = R;
    d->n1 = n1;
    d->k1 = k1;
    d->n2 = n2;
    d->k2 = k2;
    kron_default_shape(*d);
    int st = finish_dict_host_eps(d.get(), eps, s);
    if (st != SL1_OK) return st;
    const size_t es = dtype_size(dtype);
    const size_t nb = (size_t)R * n1 * k1, nc = (size_t)R * n2 * k2;
    if (hipMalloc(&d->B, nb * es) != hipSuccess || hipMalloc(&d->C, nc * es) != hipSuccess ||
        hipMalloc(&d->eps_eff, K * 8) != hipSuccess || hipMalloc(&d->at_norm, K * 8) != hipSuccess) {
        sl1_dict_free(d.release());
        return SL1_ENOMEM;
    }
    HIP_TRY(hipMemcpyAsync(d->B, B, nb * es, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(d->C, C, nc * es, hipMemcpyDeviceToDevice, s));
    // host copies of the factors: atom norms from per-column Gram matrices
    std::vector<unsigned char> hb(nb * es), hc(nc * es);
    HIP_TRY(hipMemcpyAsync(hb.data(), B, nb * es, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hc.data(), C, nc * es, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    auto val = [&](const std::vector<unsigned char>& v, size_t i) -> double {
        if (dtype == SL1_F64) return ((const double*)v.data())[i];
        if (dtype == SL1_F32) return (double)((const float*)v.data())[i];
        if (dtype == SL1_FP8_E4M3) return fp8_host(v[i]);
        return bf16_host(((const uint16_t*)v.data())[i]);
    };
    // non-finite factor entries make every product meaningless
    for (size_t i = 0; i < nb; ++i)
        if (!std::isfinite(val(hb, i))) { sl1_dict_free(d.release()); return SL1_EINVAL; }
    for (size_t i = 0; i < nc; ++i)
        if (!std::isfinite(val(hc, i))) { sl1_dict_free(d.release()); return SL1_EINVAL; }
    // GB[j1][r][r'] = sum_i1 B_r[i1,j1] B_r'[i1,j1] (signed and absolute)
    std::vector<double> GB((size_t)k1 * R * R), GBa((size_t)k1 * R * R), GC((size_t)k2 * R * R), GCa((size_t)k2 * R * R);
    for (int j1 = 0; j1 < k1; ++j1)
        for (int r = 0; r < R; ++r)
            for (int q = 0; q < R; ++q) {
                double s1 = 0, s2 = 0;
                for (int i1 = 0; i1 < n1; ++i1) {
                    const double a = val(hb, ((size_t)r * k1 + j1) * n1 + i1), b = val(hb, ((size_t)q * k1 + j1) * n1 + i1);
                    s1 += a * b;
                    s2 += std::fabs(a) * std::fabs(b);
                }
                GB[((size_t)j1 * R + r) * R + q] = s1;
                GBa[((size_t)j1 * R + r) * R + q] = s2;
            }
    for (int j2 = 0; j2 < k2; ++j2)
        for (int r = 0; r < R; ++r)
            for (int q = 0; q < R; ++q) {
                double s1 = 0, s2 = 0;
                for (int i2 = 0; i2 < n2; ++i2) {
                    const double a = val(hc, ((size_t)r * k2 + j2) * n2 + i2), b = val(hc, ((size_t)q * k2 + j2) * n2 + i2);
                    s1 += a * b;
                    s2 += std::fabs(a) * std::fabs(b);
                }
                GC[((size_t)j2 * R + r) * R + q] = s1;
                GCa[((size_t)j2 * R + r) * R + q] = s2;
            }
    std::vector<double> an(K), ab(K);
    for (int j1 = 0; j1 < k1; ++j1)
        for (int j2 = 0; j2 < k2; ++j2) {
            double s1 = 0, s2 = 0;
            for (int r = 0; r < R; ++r)
                for (int q = 0; q < R; ++q) {
                    s1 += GB[((size_t)j1 * R + r) * R + q] * GC[((size_t)j2 * R + r) * R + q];
                    s2 += GBa[((size_t)j1 * R + r) * R + q] * GCa[((size_t)j2 * R + r) * R + q];
                }
            an[(size_t)j1 * k2 + j2] = std::sqrt(std::max(s1, 0.0));
            ab[(size_t)j1 * k2 + j2] = std::sqrt(std::max(s2, 0.0)) * (1.0 + 1e-12);
        }
    double* d_ab = nullptr;
    int* bad = nullptr;
    if (hipMalloc(&d_ab, K * 8) != hipSuccess || hipMalloc(&bad, 4) != hipSuccess) return SL1_ENOMEM;
    HIP_TRY(hipMemcpyAsync(d->at_norm, an.data(), K * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_ab, ab.data(), K * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(bad, 0, 4, s));
    const double kappa = rounding_allowance(*d) * bound_norm_factor(*d);
    HIP_TRY(launch_eps_fold(eps, d_ab, kappa, (int)K, d->eps_eff, bad, s));
    std::vector<double> ee(K);
    int hbad = 0;
    HIP_TRY(hipMemcpyAsync(ee.data(), d->eps_eff, K * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    (void)hipFree(d_ab);
    (void)hipFree(bad);
    if (hbad) {
        sl1_dict_free(d.release());
        return SL1_EINVAL;
    }
    d->at_norm_max = *std::max_element(an.begin(), an.end());
    d->eps_max_eff = *std::max_element(ee.begin(), ee.end());
    d->rc_model = R * (1.0 / n1 + 1.0 / k2);
    *out = d.release();
    return SL1_OK;
}

int sl1_dict_faust(sl1_dict* out, int dtype, int J, const int64_t* dims, const int64_t* nnz, const int32_t* row_ptr,
                   const int32_t* col_idx, const void* val, const double* eps, double q, void* stream) {
    if (!out) return SL1_EINVAL;
    *out = nullptr;
    if (!dims || !nnz || !row_ptr || !col_idx || !val || !eps || J < 1 || !valid_bound_norm(q)) return SL1_EINVAL;
    if (dtype != SL1_F64 && dtype != SL1_F32) return SL1_EDTYPE;
    if (J > kFaustMax) return SL1_ELIMIT;
    const int64_t N = dims[0], K = dims[J];
    if (N < 4 || N % 4 || N > kFaustMaxDim || K < 1 || K > (int64_t)kMaxSeg * kSeg) return SL1_ELIMIT;
    for (int l = 1; l < J; ++l)
        if (dims[l] < 1 || dims[l] > kFaustMaxDim) return SL1_ELIMIT;
    // the factors' CSR arrays (host), validated: row pointers from 0 to nnz, column
    // indices in range and strictly increasing within a row, finite values
    const size_t es = dtype_size(dtype);
    std::vector<size_t> po(J + 1, 0), zo(J + 1, 0);
    for (int l = 0; l < J; ++l) {
        if (nnz[l] < 0 || nnz[l] > INT32_MAX) return SL1_EINVAL;
        po[l + 1] = po[l] + (size_t)dims[l] + 1;
        zo[l + 1] = zo[l] + (size_t)nnz[l];
    }
    if (zo[J] > (size_t)INT32_MAX) return SL1_ELIMIT;
    auto hval = [&](size_t e) -> double {
        return dtype == SL1_F64 ? ((const double*)val)[e] : (double)((const float*)val)[e];
    };
    for (int l = 0; l < J; ++l) {
        const int32_t* rp = row_ptr + po[l];
        const int32_t* ci = col_idx + zo[l];
        if (rp[0] != 0 || rp[dims[l]] != nnz[l]) return SL1_EINVAL;
        for (int64_t r = 0; r < dims[l]; ++r) {
            if (rp[r + 1] < rp[r]) return SL1_EINVAL;
            for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
                if (ci[e] < 0 || ci[e] >= dims[l + 1] || (e > rp[r] && ci[e] <= ci[e - 1])) return SL1_EINVAL;
                if (!std::isfinite(hval(zo[l] + e))) return SL1_EINVAL;
            }
        }
    }
    hipStream_t s = (hipStream_t)stream;
    auto d = std::make_unique<sl1_dict_s>();
    HIP_TRY(hipGetDevice(&d->device));
    d->kind = kFaust;
    d->dtype = dtype;
    d->N = N;
    d->K = K;
    d->q = q;
    int st = finish_dict_host_eps(d.get(), eps, s);
    if (st != SL1_OK) return st;
    // transposes (CSR of S_l^T; rows of S_l in increasing order give sorted rows)
    std::vector<size_t> tpo(J + 1, 0);
    for (int l = 0; l < J; ++l) tpo[l + 1] = tpo[l] + (size_t)dims[l + 1] + 1;
    std::vector<int32_t> tptr(tpo[J], 0), tidx(zo[J]);
    std::vector<unsigned char> tval(zo[J] * es);
    int sum_terms = 0, maxd = 0;
    for (int l = 0; l < J; ++l) {
        const int32_t* rp = row_ptr + po[l];
        const int32_t* ci = col_idx + zo[l];
        int32_t* tp = tptr.data() + tpo[l];
        for (int32_t e = 0; e < (int32_t)nnz[l]; ++e) tp[ci[e] + 1] += 1;
        int rmax = 0, cmax = 0;
        for (int64_t r = 0; r < dims[l]; ++r) rmax = std::max(rmax, rp[r + 1] - rp[r]);
        for (int64_t c = 0; c < dims[l + 1]; ++c) {
            cmax = std::max(cmax, tp[c + 1]);
            tp[c + 1] += tp[c];
        }
        sum_terms += std::max(rmax, cmax);
        std::vector<int32_t> fill(tp, tp + dims[l + 1]);
        for (int64_t r = 0; r < dims[l]; ++r)
            for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
                const int32_t q = fill[ci[e]]++;
                tidx[zo[l] + q] = (int32_t)r;
                std::memcpy(&tval[(zo[l] + q) * es], (const unsigned char*)val + (zo[l] + e) * es, es);
            }
        maxd = std::max(maxd, (int)dims[l]);
    }
    d->fa_maxd = maxd;
    d->fa_dlast = (int)dims[J - 1];
    d->fa_q = std::max(1, std::min(16, 2048 / d->fa_dlast));
    // ||a~_j|| and ||(|S_1| ... |S_J|) e_j|| in FP64, 64 atoms at a time
    std::vector<double> an(K), ab(K);
    {
        const int64_t BW = 64;
        std::vector<double> vs, va, ws, wa;
        for (int64_t j0 = 0; j0 < K; j0 += BW) {
            const int64_t nb = std::min(BW, K - j0);
            int64_t rows = dims[J - 1];
            vs.assign((size_t)rows * nb, 0.0);
            va.assign((size_t)rows * nb, 0.0);
            const int32_t* tp = tptr.data() + tpo[J - 1];
            for (int64_t q = 0; q < nb; ++q)
                for (int32_t e = tp[j0 + q]; e < tp[j0 + q + 1]; ++e) {
                    const size_t g = zo[J - 1] + e;
                    const double v = dtype == SL1_F64 ? ((const double*)tval.data())[g] : (double)((const float*)tval.data())[g];
                    vs[(size_t)tidx[g] * nb + q] = v;
                    va[(size_t)tidx[g] * nb + q] = std::fabs(v);
                }
            for (int l = J - 2; l >= 0; --l) {
                const int32_t* rp = row_ptr + po[l];
                const int32_t* ci = col_idx + zo[l];
                ws.assign((size_t)dims[l] * nb, 0.0);
                wa.assign((size_t)dims[l] * nb, 0.0);
                for (int64_t r = 0; r < dims[l]; ++r)
                    for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
                        const double v = hval(zo[l] + e), av = std::fabs(v);
                        const double* a = &vs[(size_t)ci[e] * nb];
                        const double* b = &va[(size_t)ci[e] * nb];
                        for (int64_t q = 0; q < nb; ++q) {
                            ws[(size_t)r * nb + q] += v * a[q];
                            wa[(size_t)r * nb + q] += av * b[q];
                        }
                    }
                vs.swap(ws);
                va.swap(wa);
                rows = dims[l];
            }
            for (int64_t q = 0; q < nb; ++q) {
                double s1 = 0.0, s2 = 0.0;
                for (int64_t r = 0; r < rows; ++r) {
                    s1 += vs[(size_t)r * nb + q] * vs[(size_t)r * nb + q];
                    s2 += va[(size_t)r * nb + q] * va[(size_t)r * nb + q];
                }
                an[j0 + q] = std::sqrt(s1);
                ab[j0 + q] = std::sqrt(s2) * (1.0 + 1e-12);
            }
        }
    }
    // device copies
    if (hipMalloc(&d->fa_ptr, po[J] * 4) != hipSuccess || hipMalloc(&d->fa_idx, std::max<size_t>(zo[J], 1) * 4) != hipSuccess ||
        hipMalloc(&d->fa_val, std::max<size_t>(zo[J], 1) * es) != hipSuccess ||
        hipMalloc(&d->fa_tptr, tpo[J] * 4) != hipSuccess || hipMalloc(&d->fa_tidx, std::max<size_t>(zo[J], 1) * 4) != hipSuccess ||
        hipMalloc(&d->fa_tval, std::max<size_t>(zo[J], 1) * es) != hipSuccess || hipMalloc(&d->fa, sizeof(FaustDesc)) != hipSuccess ||
        hipMalloc(&d->eps_eff, K * 8) != hipSuccess || hipMalloc(&d->at_norm, K * 8) != hipSuccess) {
        sl1_dict_free(d.release());
        return SL1_ENOMEM;
    }
    FaustDesc F;
    std::memset(&F, 0, sizeof(F));
    F.J = J;
    for (int l = 0; l <= J; ++l) F.dim[l] = (int)dims[l];
    F.maxd = maxd;
    F.q = d->fa_q;
    for (int l = 0; l < J; ++l) {
        F.fp[l] = (long long)po[l];
        F.fz[l] = (long long)zo[l];
        F.tp[l] = (long long)tpo[l];
        F.tz[l] = (long long)zo[l];
    }
    F.ptr = d->fa_ptr;
    F.idx = d->fa_idx;
    F.val = d->fa_val;
    F.tptr = d->fa_tptr;
    F.tidx = d->fa_tidx;
    F.tval = d->fa_tval;
    HIP_TRY(hipMemcpyAsync(d->fa_ptr, row_ptr, po[J] * 4, hipMemcpyHostToDevice, s));
    if (zo[J]) {
        HIP_TRY(hipMemcpyAsync(d->fa_idx, col_idx, zo[J] * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d->fa_val, val, zo[J] * es, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d->fa_tidx, tidx.data(), zo[J] * 4, hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d->fa_tval, tval.data(), zo[J] * es, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipMemcpyAsync(d->fa_tptr, tptr.data(), tpo[J] * 4, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d->fa, &F, sizeof(F), hipMemcpyHostToDevice, s));
    double* d_ab = nullptr;
    int* bad = nullptr;
    if (hipMalloc(&d_ab, K * 8) != hipSuccess || hipMalloc(&bad, 4) != hipSuccess) {
        if (d_ab) (void)hipFree(d_ab);
        sl1_dict_free(d.release());
        return SL1_ENOMEM;
    }
    HIP_TRY(hipMemcpyAsync(d->at_norm, an.data(), K * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_ab, ab.data(), K * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemsetAsync(bad, 0, 4, s));
    // the chain's FP64 sums have at most sum_l max(row, column nonzeros of S_l) terms
    const double kappa = 2.0 * ((double)sum_terms + (double)J + (double)K + 32.0) * kU64 * bound_norm_factor(*d);
    HIP_TRY(launch_eps_fold(eps, d_ab, kappa, (int)K, d->eps_eff, bad, s));
    std::vector<double> ee(K);
    int hbad = 0;
    HIP_TRY(hipMemcpyAsync(ee.data(), d->eps_eff, K * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    (void)hipFree(d_ab);
    (void)hipFree(bad);
    if (hbad) {
        sl1_dict_free(d.release());
        return SL1_EINVAL;
    }
    d->at_norm_max = *std::max_element(an.begin(), an.end());
    d->eps_max_eff = *std::max_element(ee.begin(), ee.end());
    d->rc_model = (double)zo[J] / ((double)N * (double)K);
    *out = d.release();
    return SL1_OK;
}

// Stable Dynamic Safe set-up (the caller holds w->mu): a_j^T y with the exact
// dictionary for every atom and signal -- the product the footnote to Table I
// allows to form once -- and ||y||^2, both in FP64 into the workspace.  Ends with
// the library stream synchronised, so the pinned parameter block may be rewritten.
int dst_setup(Workspace* w, sl1_dict d, int64_t batch, const void* y, int y_dtype, hipStream_t us) {
    sl1_dict seq[1] = {d};
    double L = 1.0;
    SolveParams tmp;
    std::memset(&tmp, 0, sizeof(tmp));
    int st = prepare(seq, 1, &L, nullptr, y_dtype, tmp);
    if (st != SL1_OK) return st;
    if (!w->d_cy) {
        if (w->borrowed) return SL1_ENOMEM;   // laid out by the caller of a borrowed workspace
        if (hipMalloc(&w->d_cy, (size_t)batch * tmp.K * sizeof(double)) != hipSuccess) return SL1_ENOMEM;
        if (hipMalloc(&w->d_yy, (size_t)batch * sizeof(double)) != hipSuccess) return SL1_ENOMEM;
    }
    SolveParams& p = *w->hP;
    std::memcpy(p.st, tmp.st, sizeof(tmp.st));
    p.n_stages = 1;
    p.N = tmp.N;
    p.K = tmp.K;
    p.batch = (int)batch;
    p.y_f64 = tmp.y_f64;
    p.n1_max = tmp.n1_max;
    p.fwd_fac_lds = tmp.fwd_fac_lds;
    p.max_iter = 0;
    p.trace = nullptr;
    p.trace_cap = 0;
    p.lambda_only = 1;
    p.ista = p.rule = 0;
    p.screen_every = 1;
    p.cy = p.yy = nullptr;
    p.gemm_min = 0;
    p.wg_prof = nullptr;
    p.wg_park = -1;
    p.wg_park_allow = 0;
    p.wg_absent_only = 0;
    p.Gamma = 0.5;
    p.tol = 0.0;
    p.margin = 0.0;
    p.atom_norm = d->at_norm;
    p.y = y;
    p.lam = nullptr;
    LaunchCfg cfg = launch_cfg(*w, p);
    st = check_lds(cfg);
    if (st != SL1_OK) return st;
    if (cfg.lds_fwd > 64 * 1024) HIP_TRY(fwd_lds_attr(cfg.lds_fwd));
    if (cfg.lds_adjk > 64 * 1024) HIP_TRY(adjk_lds_attr(cfg.lds_adjk));
    if (cfg.lds_adjf > 64 * 1024) HIP_TRY(adjf_lds_attr(cfg.lds_adjf));
    if ((st = order_after(w, us)) != SL1_OK) return st;
    HIP_TRY(hipMemcpyAsync(w->dP, &p, sizeof(SolveParams), hipMemcpyHostToDevice, w->stream));
    HIP_TRY(clear_ws(w, w->d_active, 4));
    HIP_TRY(launch_init(w->dP, cfg, w->stream));
    HIP_TRY(launch_fwd_adj(w->dP, cfg, w->stream));
    HIP_TRY(launch_adjoint_out(w->dP, (int)batch, tmp.K, tmp.N, w->d_cy, nullptr, w->stream));
    HIP_TRY(launch_ysq(w->dP, (int)batch, w->d_yy, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    return SL1_OK;
}

// Argument checks shared by both solve entry points (host, synchronous); fills the
// stage descriptors into tmp and the device into *dev.
static int solve_checks(const sl1_dict* seq, int n_stages, const double* L, const double* rc, const double* atom_norm,
                 int64_t batch, const void* y, const double* lambda, const sl1_opts& o, double* x, double* gap,
                 SolveParams& tmp, int* dev) {
    if (!atom_norm || !y || !lambda || !x || !gap || batch < 1) return SL1_EINVAL;
    if (batch > kMaxBatch) return SL1_ELIMIT;
    if (o.max_iter < 0 || !(o.tol >= 0.0) || !std::isfinite(o.Gamma) || !(o.margin >= 0.0)) return SL1_EINVAL;
    if (o.trace && o.trace_cap < 0) return SL1_EINVAL;
    if (o.screen_every < 0 || o.gemm_signals < 0) return SL1_EINVAL;
    if ((o.flags & SL1_FLAG_RULE_DST) && (o.flags & SL1_FLAG_RULE_DOME)) return SL1_EINVAL;
    std::memset(&tmp, 0, sizeof(tmp));
    int st = prepare(seq, n_stages, L, rc, o.y_dtype, tmp);
    if (st != SL1_OK) return st;
    if (seq[n_stages - 1]->eps_max_in != 0.0) return SL1_EINVAL;   // the last stage must be A
    if (current_device(dev) != SL1_OK) return SL1_EHIP;
    if (*dev != seq[0]->device) return SL1_EINVAL;
    return SL1_OK;
}

// Algorithm 1 on workspace w (held and locked by the caller); tmp and dev from solve_checks.
static int solve_impl(Workspace* w, const sl1_dict* seq, int n_stages, const double* atom_norm, int64_t batch,
               const void* y, const double* lambda, const sl1_opts& o, const SolveParams& tmp, int dev, double* x,
               double* gap, double* gap_cert, uint8_t* screened, int32_t* iters, int32_t* stage, void* stream) {
    int st = SL1_OK;
    const bool dst = (o.flags & SL1_FLAG_RULE_DST) != 0;
    const bool dome = (o.flags & SL1_FLAG_RULE_DOME) != 0;
    if (dst || dome) {
        // a^T y is formed with the exact dictionary's dense correlation kernel
        if (seq[n_stages - 1]->kind != kDense) return SL1_ELIMIT;
        st = dst_setup(w, seq[n_stages - 1], batch, y, o.y_dtype, (hipStream_t)stream);
        if (st != SL1_OK) return st;
    }
    SolveParams& p = *w->hP;
    std::memcpy(p.st, tmp.st, sizeof(tmp.st));
    p.n_stages = tmp.n_stages;
    p.N = tmp.N;
    p.K = tmp.K;
    p.batch = (int)batch;
    p.y_f64 = tmp.y_f64;
    p.n1_max = tmp.n1_max;
    p.fwd_fac_lds = tmp.fwd_fac_lds;
    p.max_iter = o.max_iter;
    p.trace = o.trace;
    p.trace_cap = o.trace ? o.trace_cap : 0;
    p.lambda_only = 0;
    p.ista = (o.flags & SL1_FLAG_ISTA) ? 1 : 0;
    p.screen_every = std::max(1, o.screen_every);
    p.rule = dst ? 1 : (dome ? 2 : 0);
    p.cy = (dst || dome) ? w->d_cy : nullptr;
    p.yy = (dst || dome) ? w->d_yy : nullptr;
    p.Gamma = o.Gamma;
    p.tol = o.tol;
    p.margin = o.margin;
    p.atom_norm = atom_norm;
    p.y = y;
    p.lam = lambda;
    const int eng = o.flags & (SL1_FLAG_ENGINE_GRID | SL1_FLAG_ENGINE_WG | SL1_FLAG_ENGINE_HYBRID);
    if (eng & (eng - 1)) return SL1_EINVAL;   // at most one engine flag
    if ((o.flags & SL1_FLAG_GRID_STEP) && (o.flags & SL1_FLAG_GRID_SPLIT_STEP)) return SL1_EINVAL;
    const bool gram = !(o.flags & SL1_FLAG_TAIL_COLUMNS);
    // the dome rule runs in the grid kernels only
    const size_t wlds = dome ? 0 : wg_layout(p, false, 0, false);
    // the tail hand-over needs a dense last stage with l2 bounds whose tail layout fits
    const bool tail_kind = !dome && p.st[p.n_stages - 1].kind == kDense && p.st[p.n_stages - 1].qmode == 0;
    bool tail_fits = tail_kind;
    if (tail_fits) {
        SolveParams probe = p;
        tail_fits = wg_layout(probe, true, 64, gram) != 0;
    }
    bool use_wg = false, hybrid = false;
    if (eng == SL1_FLAG_ENGINE_WG) {
        if (!wlds) return SL1_ELIMIT;
        use_wg = true;
    } else if (eng == SL1_FLAG_ENGINE_HYBRID) {
        if (tail_kind && !tail_fits) return SL1_ELIMIT;
        hybrid = tail_fits;
    } else if (eng == 0) {
        // small dictionaries: one workgroup per signal throughout (a dense stage is
        // cheap for one CU); larger ones: the grid kernels while the preserved sets
        // are large, then the tail kernel
        use_wg = wlds && (int64_t)p.N * p.K <= (1 << 20);
        hybrid = !use_wg && tail_fits;
    }
    const bool prof = (o.flags & SL1_FLAG_PROFILE) != 0;
    p.wg_prof = ((use_wg || hybrid) && prof) ? w->d_wgprof : nullptr;
    p.wg_park = -1;
    p.wg_park_allow = 0;
    p.wg_absent_only = 0;
    LaunchCfg cfg = launch_cfg(*w, p);
    if (!use_wg) {
        st = check_lds(cfg);
        if (st != SL1_OK) return st;
    }
    if (o.flags & SL1_FLAG_NO_GEMM) cfg.g_gemm = 0;
    if (cfg.g_gemm > 0) HIP_TRY(gemm_lds_attr(cfg.lds_gemm));
    if (cfg.lds_fwd > 64 * 1024) HIP_TRY(fwd_lds_attr(cfg.lds_fwd));
    if (cfg.lds_adjk > 64 * 1024) HIP_TRY(adjk_lds_attr(cfg.lds_adjk));
    if (cfg.lds_adjf > 64 * 1024) HIP_TRY(adjf_lds_attr(cfg.lds_adjf));
    p.gemm_min = cfg.g_gemm > 0 ? gemm_min_atoms(p) : 0;
    const int gemm_signals = o.gemm_signals > 0 ? o.gemm_signals : kGemmMinSignals;
    p.gemm_on = p.gemm_min > 0 && batch >= gemm_signals;
    w->last_gemm_min = p.gemm_min;
    w->last_engine = use_wg ? SL1_ENGINE_WG : SL1_ENGINE_GRID;
    w->last_gram_cap = 0;
    hipStream_t us = (hipStream_t)stream;
    if ((st = order_after(w, us)) != SL1_OK) return st;
    HIP_TRY(hipMemcpyAsync(w->dP, &p, sizeof(SolveParams), hipMemcpyHostToDevice, w->stream));
    HIP_TRY(clear_ws(w, w->d_active, 48));
    HIP_TRY(launch_init(w->dP, cfg, w->stream));
    if (o.x0) HIP_TRY(launch_init_x0(w->dP, (int)batch, o.x0, w->stream));
    if (prof) {
        for (int k = 0; k < kGridKernels; ++k) {
            w->prof_ms[k] = 0.0;
            w->prof_n[k] = 0;
        }
        for (int k = 0; k < kWgPhases; ++k) w->phase_ms[k] = w->park_phase_ms[k] = 0.0;
        w->wg_ms = w->park_ms = 0.0;
        w->wg_n = w->park_n = 0;
    }
    if (use_wg) {
        if (prof) HIP_TRY(hipMemsetAsync(w->d_wgprof, 0, (size_t)batch * kWgPhases * 8, w->stream));
        st = run_wg(w, p, o, batch, wlds, prof, dev, 0, kWgWhole);
        if (st != SL1_OK) return st;
        return finish_solve(w, cfg, batch, x, gap, gap_cert, screened, iters, stage, us);
    }
    // iterations alternate between the two control slots: chunks have even length
    const int chunk = o.chunk > 0 ? ((o.chunk + 1) & ~1) : 16;
    const bool use_graph = !(o.flags & SL1_FLAG_NO_GRAPH);
    const int hyb_atoms = hybrid_atoms(p);
    long long launched = 0;
    const long long cap = (long long)o.max_iter + 2LL * chunk + 4;
    if (prof) {
        // one event before and after every kernel of a chunk
        while ((int)w->prof_ev.size() < 2 * kGridKernels * chunk) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            w->prof_ev.push_back(e);
        }
    }
    // launches with no possible work are left out of a chunk: the Kronecker
    // correlations once every live signal is on a dense last stage (stages only
    // advance), the batched product while the host has it switched off
    const bool last_kron = p.st[p.n_stages - 1].kind != kDense;      // a structured last stage
    bool kron_live = cfg.g_adjk > 0 || cfg.adjf_x > 0;
    // hybrid: Kronecker approximations run in the whole-solve kernel (one workgroup
    // per signal with the factors in LDS, no kernel boundary between iterations); a
    // signal stops there at the top of its first iteration on the last stage.  The
    // parked signals then go on in the tail kernel when every preserved set is small
    // enough for it, else in the grid kernels (their lists converted), which hand
    // over to the tail later.  Dense approximations stay on the grid kernels, which
    // spread a large preserved set over the chip.
    bool kron_first = hybrid && wlds && p.n_stages > 1 && !(o.flags & SL1_FLAG_HYBRID_GRID_FIRST);
    for (int i = 0; i + 1 < p.n_stages; ++i) kron_first = kron_first && p.st[i].kind == kKron;
    // per-signal step launches (update of t and forward of t + 1 in one block per
    // signal) replace the chip-wide forward and update launches while every live
    // signal can only be on dense stages: from the start when every stage is dense,
    // after the Kronecker approximations' whole-solve phase otherwise
    // (a batch of fewer than 128 signals would leave most CUs idle: one block per
    // signal streams its whole preserved set, where the split launches spread every
    // signal's segments over the chip)
    bool step_ok = !dome && !(o.flags & SL1_FLAG_GRID_SPLIT_STEP) &&
                   (batch >= 128 || (o.flags & SL1_FLAG_GRID_STEP));
    bool all_dense = true;
    for (int i = 0; i < p.n_stages; ++i) {
        step_ok = step_ok && p.st[i].qmode == 0;
        all_dense = all_dense && p.st[i].kind == kDense;
    }
    bool step_live = step_ok && all_dense;
    bool beside = false;      // late signals of the Kronecker phase in a launch on the second stream
    if (kron_first) {
        w->last_engine = SL1_ENGINE_HYBRID;
        p.wg_park = p.n_stages - 1;
        // a few late signals need not hold the phase for the whole batch: once at most
        // batch / 128 are short of A, the grid kernels start for the others while a
        // whole-solve launch on the second stream goes on with those few (step launches
        // on a dense last stage only; not for a borrowed workspace, which has no stream)
        const bool can_beside = w->stream2 && step_ok && !last_kron && batch >= 128 &&
                                !(o.flags & SL1_FLAG_PARK_ALL);
        p.wg_park_allow = can_beside ? (int)(batch / 128) : 0;
        HIP_TRY(hipMemcpyAsync(w->dP, &p, sizeof(SolveParams), hipMemcpyHostToDevice, w->stream));
        if (prof) HIP_TRY(hipMemsetAsync(w->d_wgprof, 0, (size_t)batch * kWgPhases * 8, w->stream));
        st = run_wg(w, p, o, batch, wlds, prof, dev, 0, kWgPark);
        if (st != SL1_OK) return st;
        SolveParams pw = p;                       // the whole-solve layout, for a launch beside
        pw.wg_park_allow = 0;
        pw.wg_absent_only = 1;
        p.wg_park = -1;
        p.wg_park_allow = 0;
        p.wg_park_allow = 0;
        p.wg_absent_only = 0;
        if (*w->h_active <= 0) return finish_solve(w, cfg, batch, x, gap, gap_cert, screened, iters, stage, us);
        const int* s1 = w->h_active + 4;
        const size_t tlds = wg_layout(p, true, s1[0], gram);
        if (s1[2] == 0 && tlds && (s1[0] <= hyb_atoms || s1[0] <= p.wg_cap_gram)) {
            // the parked state is the tail kernel's input format as it stands
            HIP_TRY(hipMemcpyAsync(w->dP, &p, sizeof(SolveParams), hipMemcpyHostToDevice, w->stream));
            w->last_gram_cap = p.wg_cap_gram;
            if (prof) HIP_TRY(hipMemsetAsync(w->d_wgprof, 0, (size_t)batch * kWgPhases * 8, w->stream));
            st = run_wg(w, p, o, batch, tlds, prof, dev, 0, kWgTail);
            if (st != SL1_OK) return st;
            return finish_solve(w, cfg, batch, x, gap, gap_cert, screened, iters, stage, us);
        }
        if (p.gemm_min > 0) p.gemm_on = s1[3] >= gemm_signals ? 1 : 0;
        beside = can_beside && s1[2] > 0;
        if (beside || (!last_kron && s1[2] == 0)) kron_live = false;
        step_live = step_ok && (beside || s1[2] == 0);
        HIP_TRY(hipMemcpyAsync(w->dP, &p, sizeof(SolveParams), hipMemcpyHostToDevice, w->stream));
        HIP_TRY(launch_wg_to_grid(w->dP, (int)batch, w->stream, beside ? 1 : 0, p.n_stages - 1));
        if (beside) {
            // after the absent marks: the late signals' launch runs to the park stage (or
            // their stop) on the second stream; they join at the first chunk boundary after it
            HIP_TRY(hipMemcpyAsync(w->dP2, &pw, sizeof(SolveParams), hipMemcpyHostToDevice, w->stream));
            HIP_TRY(hipEventRecord(w->ev_j, w->stream));
            HIP_TRY(hipStreamWaitEvent(w->stream2, w->ev_j, 0));
            if (prof) HIP_TRY(hipEventRecord(w->ev_c, w->stream2));
            HIP_TRY(launch_solve_wg(w->dP2, (int)batch, wlds, (int)std::min<long long>((long long)o.max_iter + 1, INT32_MAX),
                                    w->stream2));
            if (prof) HIP_TRY(hipEventRecord(w->ev_d, w->stream2));
            HIP_TRY(hipEventRecord(w->ev_k, w->stream2));
        }
    }
    for (;;) {
        LaunchCfg ccfg = cfg;
        if (!kron_live || step_live) {
            ccfg.g_adjk = 0;
            ccfg.adjf_x = ccfg.adjf_y = ccfg.adjf_z = 0;
        }
        if (!p.gemm_on) ccfg.g_gemm = 0;
        ccfg.step = step_live ? 1 : 0;
        const int v = (ccfg.g_adjk > 0 || ccfg.adjf_x > 0 ? 1 : 0) | (ccfg.g_gemm > 0 ? 2 : 0) | (ccfg.step ? 4 : 0);
        if (prof) {
            for (int it = 0; it < chunk; ++it)
                for (int q = 0; q < kGridKernels; ++q) {
                    const int k = kIterOrder[q];
                    const int e0 = 2 * (kGridKernels * it + k);
                    HIP_TRY(hipEventRecord(w->prof_ev[e0], w->stream));
                    HIP_TRY(launch_one(k, it & 1, w->dP, ccfg, w->stream));
                    HIP_TRY(hipEventRecord(w->prof_ev[e0 + 1], w->stream));
                }
        } else if (use_graph) {
            if (!w->graph[v] || w->graph_chunk[v] != chunk || !cfg_equal(ccfg, w->graph_cfg[v])) {
                st = capture_chunk(w, ccfg, chunk, v);
                if (st != SL1_OK) return st;
            }
            HIP_TRY(hipGraphLaunch(w->graph[v], w->stream));
        } else {
            for (int k = 0; k < chunk; ++k) HIP_TRY(launch_iter(k & 1, w->dP, ccfg, w->stream));
        }
        launched += chunk;
        if (beside) {
            // the late signals join once their launch beside has ended
            HIP_TRY(hipStreamWaitEvent(w->stream, w->ev_k, 0));
            HIP_TRY(launch_wg_to_grid(w->dP, (int)batch, w->stream, 2, p.n_stages - 1));
            beside = false;
            if (prof) {
                HIP_TRY(hipEventSynchronize(w->ev_d));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, w->ev_c, w->ev_d));
                w->wg_ms += ms;
                w->wg_n += 1;
                w->park_ms += ms;
                w->park_n += 1;
            }
        }
        if (prof) {
            HIP_TRY(hipStreamSynchronize(w->stream));
            const bool run[kGridKernels] = {!ccfg.step, ccfg.g_adj > 0, ccfg.g_adjk > 0 || ccfg.adjf_x > 0, !ccfg.step,
                                            ccfg.g_gemm > 0, ccfg.g_gemm > 0, ccfg.step != 0};
            for (int it = 0; it < chunk; ++it)
                for (int k = 0; k < kGridKernels; ++k) {
                    if (!run[k]) continue;
                    float ms = 0.f;
                    const int e0 = 2 * (kGridKernels * it + k);
                    HIP_TRY(hipEventElapsedTime(&ms, w->prof_ev[e0], w->prof_ev[e0 + 1]));
                    w->prof_ms[k] += ms;
                    w->prof_n[k] += 1;
                }
        }
        HIP_TRY(launch_stat(w->dP, w->stream));
        HIP_TRY(hipMemcpyAsync(w->h_active, w->d_active, 32, hipMemcpyDeviceToHost, w->stream));
        HIP_TRY(hipStreamSynchronize(w->stream));
        if (*w->h_active <= 0 || launched > cap) break;
        // the batched correlation product runs in the next chunk only if enough
        // signals qualified in this chunk's last iteration
        if (p.gemm_min > 0) {
            const int on = w->h_active[4 + 3] >= gemm_signals ? 1 : 0;
            if (on != p.gemm_on) {
                p.gemm_on = on;
                HIP_TRY(hipMemcpyAsync(&w->dP->gemm_on, &p.gemm_on, sizeof(int), hipMemcpyHostToDevice, w->stream));
            }
        }
        // hand the remaining iterations to the whole-solve kernel once every live
        // signal is on the last stage with a small preserved set (statistics of
        // the chunk's last forward launch)
        const int* stat1 = w->h_active + 4;
        if (!last_kron && stat1[2] == 0) kron_live = false;
        if (hybrid && stat1[2] == 0) {
            // in Gram mode an iteration costs no N-length work: hand over as soon as
            // the largest preserved set fits the Gram capacity
            const size_t tlds = wg_layout(p, true, stat1[0], gram);
            if (tlds && (stat1[0] <= hyb_atoms || stat1[0] <= p.wg_cap_gram)) {
                HIP_TRY(hipMemcpyAsync(w->dP, &p, sizeof(SolveParams), hipMemcpyHostToDevice, w->stream));
                // after step launches the state of iteration t (correlations formed, update
                // pending) is the tail's input; otherwise a forward launch first folds in
                // the last update
                if (!step_live) HIP_TRY(launch_one(0, 0, w->dP, cfg, w->stream));
                HIP_TRY(launch_to_wg(w->dP, (int)batch, step_live ? 1 : 0, w->stream));
                w->last_engine = SL1_ENGINE_HYBRID;
                w->last_gram_cap = p.wg_cap_gram;
                if (prof) HIP_TRY(hipMemsetAsync(w->d_wgprof, 0, (size_t)batch * kWgPhases * 8, w->stream));
                st = run_wg(w, p, o, batch, tlds, prof, dev, launched, kWgTail);
                if (st != SL1_OK) return st;
                break;
            }
        }
    }
    return finish_solve(w, cfg, batch, x, gap, gap_cert, screened, iters, stage, us);
}

int sl1_solve(const sl1_dict* seq, int n_stages, const double* L, const double* rc, const double* atom_norm,
              int64_t batch, const void* y, const double* lambda, const sl1_opts* opt, double* x, double* gap,
              double* gap_cert, uint8_t* screened, int32_t* iters, int32_t* stage, void* stream) {
    sl1_opts o;
    if (opt) o = *opt;
    else sl1_opts_default(&o);
    SolveParams tmp;
    int dev = 0;
    int st = solve_checks(seq, n_stages, L, rc, atom_norm, batch, y, lambda, o, x, gap, tmp, &dev);
    if (st != SL1_OK) return st;
    std::shared_ptr<Workspace> ws;
    st = get_workspace(dev, (int)batch, tmp.N, tmp.K, &ws);
    if (st != SL1_OK) return st;
    Workspace* w = ws.get();
    std::lock_guard<std::mutex> lk(w->mu);
    return solve_impl(w, seq, n_stages, atom_norm, batch, y, lambda, o, tmp, dev, x, gap, gap_cert, screened, iters,
                      stage, stream);
}

// Device address of `scratch` on device dev (taken on the first call there, with dev
// current), and the mutex that serialises the calls sharing it.
constexpr int kScratchDevices = 64;
std::mutex g_scratch_init_mu;
std::mutex g_scratch_mu[kScratchDevices];
void* g_scratch_ptr[kScratchDevices] = {};

static int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kScratchDevices) return SL1_ELIMIT;
    std::lock_guard<std::mutex> lk(g_scratch_init_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SL1_EHIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SL1_OK;
}

int sl1_solve_noalloc(const sl1_dict* seq, int n_stages, const double* L, const double* rc,
                      const double* atom_norm, int64_t batch, const void* y, const double* lambda,
                      const sl1_opts* opt, double* x, double* gap, double* gap_cert, uint8_t* screened,
                      int32_t* iters, int32_t* stage, void* stream) {
    sl1_opts o;
    if (opt) o = *opt;
    else sl1_opts_default(&o);
    if (o.flags & SL1_FLAG_PROFILE) return SL1_EINVAL;   // profiling records events
    o.flags |= SL1_FLAG_NO_GRAPH;                        // direct launches: no graph to instantiate
    SolveParams tmp;
    int dev = 0;
    int st = solve_checks(seq, n_stages, L, rc, atom_norm, batch, y, lambda, o, x, gap, tmp, &dev);
    if (st != SL1_OK) return st;
    void* base = nullptr;
    if ((st = scratch_address(dev, &base)) != SL1_OK) return st;
    // a view of the fixed array laid out like an allocated workspace of this shape
    Workspace w;
    w.borrowed = true;
    w.device = dev;
    w.batch = (int)batch;
    w.N = tmp.N;
    w.K = tmp.K;
    SolveParams hp;
    std::memset(&hp, 0, sizeof(hp));
    int h_active[16] = {0};
    size_t need = workspace_layout(w, nullptr, nullptr);
    const bool rule_y = (o.flags & (SL1_FLAG_RULE_DST | SL1_FLAG_RULE_DOME)) != 0;
    const size_t o_cy = need;
    if (rule_y) need += al((size_t)batch * tmp.K * 8) + al((size_t)batch * 8);
    if (need > kScratchBytes) return SL1_ELIMIT;
    workspace_layout(w, (char*)base, &hp);
    if (rule_y) {
        w.d_cy = (double*)((char*)base + o_cy);
        w.d_yy = (double*)((char*)base + o_cy + al((size_t)batch * tmp.K * 8));
    }
    w.mem = base;
    w.hP = &hp;
    w.h_active = h_active;
    w.stream = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_scratch_mu[dev]);
    // the array keeps the previous call's contents: start from zeros, as a new workspace does
    HIP_TRY(launch_zero(base, need, w.stream));
    return solve_impl(&w, seq, n_stages, atom_norm, batch, y, lambda, o, tmp, dev, x, gap, gap_cert, screened,
                      iters, stage, stream);
}

static int lambda_pass(sl1_dict d, int64_t batch, const void* y, int y_dtype, double* lam_out, double* g_out,
                       double* z_out, void* stream) {
    if (!d || !y || batch < 1) return SL1_EINVAL;
    if (batch > kMaxBatch) return SL1_ELIMIT;
    sl1_dict seq[1] = {d};
    double L = 1.0;
    SolveParams tmp;
    std::memset(&tmp, 0, sizeof(tmp));
    int st = prepare(seq, 1, &L, nullptr, y_dtype, tmp);
    if (st != SL1_OK) return st;
    int dev = 0;
    if (current_device(&dev) != SL1_OK) return SL1_EHIP;
    if (dev != d->device) return SL1_EINVAL;
    std::shared_ptr<Workspace> ws;
    st = get_workspace(dev, (int)batch, tmp.N, tmp.K, &ws);
    if (st != SL1_OK) return st;
    Workspace* w = ws.get();
    std::lock_guard<std::mutex> lk(w->mu);
    SolveParams& p = *w->hP;
    std::memcpy(p.st, tmp.st, sizeof(tmp.st));
    p.n_stages = 1;
    p.N = tmp.N;
    p.K = tmp.K;
    p.batch = (int)batch;
    p.y_f64 = tmp.y_f64;
    p.n1_max = tmp.n1_max;
    p.fwd_fac_lds = tmp.fwd_fac_lds;
    p.max_iter = 0;
    p.trace = nullptr;
    p.trace_cap = 0;
    p.lambda_only = 1;
    p.ista = p.rule = 0;
    p.screen_every = 1;
    p.cy = p.yy = nullptr;
    p.gemm_min = 0;
    p.wg_prof = nullptr;
    p.wg_park = -1;
    p.wg_park_allow = 0;
    p.wg_absent_only = 0;
    p.Gamma = 0.5;
    p.tol = 0.0;
    p.margin = 0.0;
    p.atom_norm = d->at_norm;
    p.y = y;
    p.lam = nullptr;
    LaunchCfg cfg = launch_cfg(*w, p);
    st = check_lds(cfg);
    if (st != SL1_OK) return st;
    if (cfg.lds_fwd > 64 * 1024) HIP_TRY(fwd_lds_attr(cfg.lds_fwd));
    if (cfg.lds_adjk > 64 * 1024) HIP_TRY(adjk_lds_attr(cfg.lds_adjk));
    if (cfg.lds_adjf > 64 * 1024) HIP_TRY(adjf_lds_attr(cfg.lds_adjf));
    hipStream_t us = (hipStream_t)stream;
    HIP_TRY(hipEventRecord(w->ev_in, us));
    HIP_TRY(hipStreamWaitEvent(w->stream, w->ev_in, 0));
    HIP_TRY(hipMemcpyAsync(w->dP, &p, sizeof(SolveParams), hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipMemsetAsync(w->d_active, 0, 4, w->stream));
    HIP_TRY(launch_init(w->dP, cfg, w->stream));
    HIP_TRY(launch_fwd_adj(w->dP, cfg, w->stream));
    // the per-signal status always comes back; lambda'_max lands in scratch when not asked for
    double* lam_dst = lam_out ? lam_out : (double*)w->d_times;
    HIP_TRY(launch_lambda_out(w->dP, (int)batch, lam_dst, w->d_status, w->stream));
    if (g_out) HIP_TRY(launch_adjoint_out(w->dP, (int)batch, tmp.K, tmp.N, g_out, z_out, w->stream));
    std::vector<int32_t> hs(batch);
    HIP_TRY(hipMemcpyAsync(hs.data(), w->d_status, batch * 4, hipMemcpyDeviceToHost, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    HIP_TRY(hipEventRecord(w->ev_out, w->stream));
    HIP_TRY(hipStreamWaitEvent(us, w->ev_out, 0));
    for (int32_t v : hs)
        if (v < 0) return v;
    return SL1_OK;
}

int sl1_lambda_max(sl1_dict d, int64_t batch, const void* y, int y_dtype, double* out, void* stream) {
    if (!out) return SL1_EINVAL;
    return lambda_pass(d, batch, y, y_dtype, out, nullptr, nullptr, stream);
}

int sl1_dict_adjoint(sl1_dict d, int64_t batch, const void* y, int y_dtype, double* out, double* z_used,
                     void* stream) {
    if (!out) return SL1_EINVAL;
    return lambda_pass(d, batch, y, y_dtype, nullptr, out, z_used, stream);
}

// Device time of one correlation launch with stage descriptor sd over the whole atom
// set, for batch signals y = ybuf (the caller holds w->mu; launches on w->stream).
static int time_adj(Workspace* w, const SolveParams& tmp, const StageDesc& sd, int64_t batch, const void* ybuf,
                    int reps, double* ms_out) {
    SolveParams& p = *w->hP;
    std::memcpy(p.st, tmp.st, sizeof(tmp.st));
    p.st[0] = sd;
    p.n_stages = 1;
    p.N = tmp.N;
    p.K = tmp.K;
    p.batch = (int)batch;
    p.y_f64 = tmp.y_f64;
    p.n1_max = tmp.n1_max;
    p.fwd_fac_lds = tmp.fwd_fac_lds;
    p.max_iter = 0;
    p.trace = nullptr;
    p.trace_cap = 0;
    p.lambda_only = 1;
    p.ista = p.rule = 0;
    p.screen_every = 1;
    p.cy = p.yy = nullptr;
    p.gemm_min = 0;
    p.wg_prof = nullptr;
    p.wg_park = -1;
    p.wg_park_allow = 0;
    p.wg_absent_only = 0;
    p.tol = 0.0;
    p.margin = 0.0;
    p.atom_norm = sd.at_norm;
    p.y = ybuf;
    p.lam = nullptr;
    LaunchCfg cfg = launch_cfg(*w, p);
    int st = check_lds(cfg);
    if (st != SL1_OK) return st;
    if (cfg.lds_fwd > 64 * 1024) HIP_TRY(fwd_lds_attr(cfg.lds_fwd));
    if (cfg.lds_adjk > 64 * 1024) HIP_TRY(adjk_lds_attr(cfg.lds_adjk));
    if (cfg.lds_adjf > 64 * 1024) HIP_TRY(adjf_lds_attr(cfg.lds_adjf));
    HIP_TRY(hipMemcpyAsync(w->dP, &p, sizeof(SolveParams), hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipMemsetAsync(w->d_active, 0, 4, w->stream));
    HIP_TRY(launch_init(w->dP, cfg, w->stream));
    HIP_TRY(launch_fwd_adj(w->dP, cfg, w->stream));
    for (int k = 0; k < 3; ++k) HIP_TRY(launch_adj_only(w->dP, cfg, w->stream));
    HIP_TRY(hipEventRecord(w->ev_a, w->stream));
    for (int k = 0; k < reps; ++k) HIP_TRY(launch_adj_only(w->dP, cfg, w->stream));
    HIP_TRY(hipEventRecord(w->ev_b, w->stream));
    HIP_TRY(hipEventSynchronize(w->ev_b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, w->ev_a, w->ev_b));
    *ms_out = ms / reps;
    return SL1_OK;
}

// Shared set-up of the timing calls: stage descriptors, the workspace, synthetic signals
// y = 1 (the cost of a correlation launch over every atom does not depend on y).
struct TimingSetup {
    SolveParams tmp;
    std::shared_ptr<Workspace> ws;
    void* ybuf = nullptr;
    ~TimingSetup() {
        if (ybuf) (void)hipFree(ybuf);
    }
};

static int timing_setup(const sl1_dict* seq, int n_stages, int64_t batch, TimingSetup& T) {
    if (!seq || n_stages < 1 || batch < 1) return SL1_EINVAL;
    if (batch > kMaxBatch) return SL1_ELIMIT;
    std::vector<double> Ls(n_stages, 1.0);
    std::memset(&T.tmp, 0, sizeof(T.tmp));
    int st = prepare(seq, n_stages, Ls.data(), nullptr, SL1_F64, T.tmp);
    if (st != SL1_OK) return st;
    int dev = 0;
    if (current_device(&dev) != SL1_OK) return SL1_EHIP;
    st = get_workspace(dev, (int)batch, T.tmp.N, T.tmp.K, &T.ws);
    if (st != SL1_OK) return st;
    if (hipMalloc(&T.ybuf, (size_t)batch * T.tmp.N * 8) != hipSuccess) return SL1_ENOMEM;
    return SL1_OK;
}

static int timing_fill_y(Workspace* w, TimingSetup& T, int64_t batch, hipStream_t us) {
    std::vector<double> hy((size_t)batch * T.tmp.N, 1.0);
    if ((order_after(w, us)) != SL1_OK) return SL1_EHIP;
    HIP_TRY(hipMemcpyAsync(T.ybuf, hy.data(), hy.size() * 8, hipMemcpyHostToDevice, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    return SL1_OK;
}

int sl1_measure_rc(const sl1_dict* seq, int n_stages, int64_t batch, double* rc_out, void* stream) {
    if (!rc_out) return SL1_EINVAL;
    TimingSetup T;
    int st = timing_setup(seq, n_stages, batch, T);
    if (st != SL1_OK) return st;
    Workspace* w = T.ws.get();
    std::lock_guard<std::mutex> lk(w->mu);
    hipStream_t us = (hipStream_t)stream;
    if ((st = timing_fill_y(w, T, batch, us)) != SL1_OK) return st;
    std::vector<double> times(n_stages, 0.0);
    for (int i = 0; i < n_stages; ++i)
        if ((st = time_adj(w, T.tmp, T.tmp.st[i], batch, T.ybuf, 20, &times[i])) != SL1_OK) return st;
    HIP_TRY(hipStreamSynchronize(w->stream));
    if ((st = order_before(w, us)) != SL1_OK) return st;
    const double ref = times[n_stages - 1];
    for (int i = 0; i < n_stages; ++i) rc_out[i] = ref > 0 ? times[i] / ref : 1.0;
    return SL1_OK;
}

int sl1_dict_kron_tile(sl1_dict d, int kt2, int kt1) {
    if (!d || d->kind != kKron || !kron_shape_ok(*d, kt2, kt1)) return SL1_EINVAL;
    d->kt2 = kt2;
    d->kt1 = kt1;
    return SL1_OK;
}

int sl1_tune_kron(const sl1_dict* seq, int n_stages, int64_t batch, int32_t* shape_out, double* ms_out,
                  void* stream) {
    TimingSetup T;
    int st = timing_setup(seq, n_stages, batch, T);
    if (st != SL1_OK) return st;
    Workspace* w = T.ws.get();
    std::lock_guard<std::mutex> lk(w->mu);
    hipStream_t us = (hipStream_t)stream;
    if ((st = timing_fill_y(w, T, batch, us)) != SL1_OK) return st;
    static const int kCand[] = {16, 32, 64, 128};
    for (int i = 0; i < n_stages; ++i) {
        sl1_dict_s& d = *seq[i];
        if (shape_out) shape_out[2 * i] = shape_out[2 * i + 1] = 0;
        if (ms_out) ms_out[i] = 0.0;
        if (d.kind != kKron) continue;
        int best2 = d.kt2, best1 = d.kt1;
        double best = -1.0;
        for (int kt2 : kCand)
            for (int kt1 : kCand) {
                if (!kron_shape_ok(d, kt2, kt1) || kt2 * kt1 < 512) continue;
                StageDesc sd = T.tmp.st[i];
                sd.kt2 = kt2;
                sd.kt1 = kt1;
                double ms = 0.0;
                st = time_adj(w, T.tmp, sd, batch, T.ybuf, 20, &ms);
                if (st == SL1_ELIMIT) continue;            // the launch's LDS does not fit
                if (st != SL1_OK) return st;
                if (best < 0.0 || ms < best) {
                    best = ms;
                    best2 = kt2;
                    best1 = kt1;
                }
            }
        d.kt2 = best2;
        d.kt1 = best1;
        if (shape_out) {
            shape_out[2 * i] = best2;
            shape_out[2 * i + 1] = best1;
        }
        if (ms_out) ms_out[i] = best;
    }
    HIP_TRY(hipStreamSynchronize(w->stream));
    return order_before(w, us);
}

// Device clock stamps (start, convergence) of each signal of the last solve of
// this shape, for time-to-gap measurements; out: host, 2*batch int64, and the
// clock rate in kHz.
int sl1_last_solve_clock(int64_t batch, int64_t N, int64_t K, long long* out, double* rate_khz) {
    int dev = 0;
    if (current_device(&dev) != SL1_OK) return SL1_EHIP;
    std::shared_ptr<Workspace> ws;
    {
        std::lock_guard<std::mutex> lk(g_ws_mu);
        auto it = g_ws.find(std::make_tuple(dev, (int)batch, (int)N, (int)K));
        if (it == g_ws.end()) return SL1_EINVAL;
        ws = it->second;
    }
    Workspace* w = ws.get();
    std::lock_guard<std::mutex> lk(w->mu);
    HIP_TRY(launch_time_out(w->dP, (int)batch, w->d_times, w->stream));
    HIP_TRY(hipMemcpyAsync(out, w->d_times, batch * 16, hipMemcpyDeviceToHost, w->stream));
    HIP_TRY(hipStreamSynchronize(w->stream));
    int khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    *rate_khz = khz;
    return SL1_OK;
}

int sl1_last_solve_profile(int64_t batch, int64_t N, int64_t K, double* ms, long long* launches) {
    if (!ms || !launches) return SL1_EINVAL;
    int dev = 0;
    if (current_device(&dev) != SL1_OK) return SL1_EHIP;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find(std::make_tuple(dev, (int)batch, (int)N, (int)K));
    if (it == g_ws.end()) return SL1_EINVAL;
    for (int k = 0; k < kGridKernels; ++k) {
        ms[k] = it->second->prof_ms[k];
        launches[k] = it->second->prof_n[k];
    }
    return SL1_OK;
}

int sl1_last_solve_phases(int64_t batch, int64_t N, int64_t K, int32_t* engine, double* phase_ms,
                          long long* wg_launches, int32_t* gram_cap, int32_t* gemm_min) {
    if (!engine) return SL1_EINVAL;
    int dev = 0;
    if (current_device(&dev) != SL1_OK) return SL1_EHIP;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    auto it = g_ws.find(std::make_tuple(dev, (int)batch, (int)N, (int)K));
    if (it == g_ws.end()) return SL1_EINVAL;
    const Workspace& w = *it->second;
    *engine = w.last_engine;
    if (phase_ms) {
        for (int k = 0; k < kWgPhases; ++k) {
            phase_ms[k] = w.phase_ms[k];
            phase_ms[kWgPhases + 2 + k] = w.park_phase_ms[k];
        }
        phase_ms[kWgPhases] = w.wg_ms;
        phase_ms[kWgPhases + 1] = w.park_ms;
        phase_ms[2 * kWgPhases + 2] = (double)w.park_n;
    }
    if (wg_launches) *wg_launches = w.wg_n;
    if (gram_cap) *gram_cap = w.last_gram_cap;
    if (gemm_min) *gemm_min = w.last_gemm_min;
    return SL1_OK;
}

__attribute__((visibility("hidden"))) int sl1_grad_impl_dense_info(sl1_dict_s* d, int* kind, int* dtype, int64_t* N, int64_t* K, const void** A,
                             const float** scale) {
    if (!d) return SL1_EINVAL;
    *kind = d->kind;
    *dtype = d->dtype;
    *N = d->N;
    *K = d->K;
    *A = d->A;
    *scale = d->scale;
    return SL1_OK;
}

}  // extern "C"
