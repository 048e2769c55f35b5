// api.cpp -- host runtime and C ABI of libkzk (plan, workspace, launches).
#include "../../include/kzk.h"
#include "internal.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <new>
#include <vector>

using kzk::InstDesc;
using kzk::TauItem;
using kzk::YItem;

namespace {

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2i(int v) { int l = 0; while ((1 << l) < v) ++l; return l; }
// K with n_tau = 7 * 2^(K+1), 4 <= K <= 9 (M = n_tau/2 = 7 * 2^K, 112 .. 3584), else 0
int gen_k(int n_tau) {
    if (n_tau % 14 != 0 || !pow2(n_tau / 14)) return 0;
    const int k = ilog2i(n_tau / 14);
    return k >= 4 && k <= 9 ? k : 0;
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct kzk_plan {
    int n_inst = 0;
    int dtype = KZK_F64;
    size_t esz = 8;                       // bytes per real
    hipStream_t stream = nullptr;
    int device = 0;
    std::vector<kzk_params> params;
    std::vector<std::vector<double>> Dsched, nlsched;
    std::vector<InstDesc> desc;
    std::vector<size_t> u_off;            // n_inst + 1 real offsets
    size_t state_elems = 0, tab_elems = 0;
    int ntw = 0, log2_ntw = 0;
    int y_threads = 0;
    int y_grid = 0;                       // persistent y-pass blocks (resident at once)
    int tau_prog = 0;                     // every instance has M/16 >= W and M >= 256 (tau-pass pair indexing)
    int gk = 0;                           // > 0: every instance has M = 7 * 2^gk (mixed-radix tau-pass)
    int y_full = 0;                       // every instance has W n_y = 16 y_threads and n_y >= 512 (full y tiles)
    int y_ntl = 0;                        // FP64 state arrays above 64 MiB: non-temporal y-pass loads
    int max_ny = 0;                       // largest n_y of the plan (8192 needs full tiles of 512+ threads)
    bool any_D_sched = false;
    int scheme = 0;                       // 0: ExpRK22, 1: exponential Euler (every solve)
    bool any_reg = false;                 // some solve uses the regularised multiplier
    // transport by the random velocity field (every solve or none): the
    // physical field and transverse part of b per stage, its tau-spectrum,
    // velocity tables at the nodes, and the work list of the transverse pass
    bool transport = false;
    bool s64 = false;                     // FP32 plan whose spectral state U and stage value P are FP64
    void *dUph = nullptr, *dByp = nullptr, *dBys = nullptr;
    kzk::YwItem* dYw = nullptr;
    int n_yw_items = 0;
    long long steps_limit = -1;           // -1: unlimited (constant coefficients)

    void *dC = nullptr, *dB = nullptr, *dP = nullptr, *dU = nullptr, *dTab = nullptr, *dTw = nullptr;
    void* dSig = nullptr;                 // flux-difference symbols, sum of M over the solves
    InstDesc* dDesc = nullptr;
    TauItem* dTau = nullptr;    // tau-pass work list (tau_threads * 16 / M lines per item)
    TauItem* dTauAdj = nullptr; // adjoint tau-pass work list (TAU_THREADS * 16 / M lines per item)
    YItem* dY = nullptr;
    int n_tau_items = 0, n_tau_adj_items = 0, n_y_items = 0, max_tau_items = 0;
    int tau_threads = kzk::TAU_THREADS;   // tau-pass block size
    int tau_mr = 4;                       // tau-transform radix schedule: log2 of the largest radix (4 or 3)
    void* dTwSt = nullptr;      // per-stage Stockham twiddles
    unsigned* dStatus = nullptr;
    double* dSched = nullptr;
    std::vector<void*> owned;             // everything hipMalloc'ed, freed in destroy
    // plans of kzk_step_noalloc carve their device memory out of the static
    // scratch array instead (bump allocation, nothing to free)
    char* arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;

    bool graph_on = false;
    hipGraphExec_t gexec = nullptr;
    const void* g_u = nullptr;
    int g_first = -1, g_n = -1;

    // per-kernel timing with HIP events (kzk_profile_enable): launches outside
    // the step loop always, those of step s when s % prof_every == 0
    bool prof = false;
    int prof_every = 1;
    bool prof_now = false;
    struct Ev { int kind; hipEvent_t a, b; };
    std::vector<Ev> ev_used;
    std::vector<hipEvent_t> ev_pool;

    // adjoint workspace (allocated on first use, grown on demand)
    void *dL = nullptr, *dM = nullptr, *dR = nullptr, *dCk = nullptr, *dUn = nullptr, *dUs = nullptr;
    size_t adj_ckpt_cap = 0, adj_seg_cap = 0;
};

namespace {

kzk_status dev_alloc(kzk_plan* p, void** out, size_t bytes) {
    *out = nullptr;
    if (bytes == 0) bytes = 256;
    if (p->arena) {
        const size_t off = (p->arena_used + 255) & ~(size_t)255;
        if (off > p->arena_cap || bytes > p->arena_cap - off) return KZK_ERR_SIZE;
        *out = p->arena + off;
        p->arena_used = off + bytes;
        return KZK_OK;
    }
    if (hipMalloc(out, bytes) != hipSuccess) {
        (void)hipGetLastError();
        *out = nullptr;
        return KZK_ERR_OOM;
    }
    p->owned.push_back(*out);
    return KZK_OK;
}

// Free one buffer of dev_alloc (the plan's stream must have finished with it).
void dev_free(kzk_plan* p, void*& q) {
    if (!q) return;
    auto it = std::find(p->owned.begin(), p->owned.end(), q);
    if (it != p->owned.end()) {
        p->owned.erase(it);
        (void)hipFree(q);
    }
    q = nullptr;
}

void drop_graph(kzk_plan* p) {
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
    p->g_u = nullptr;
    p->g_first = p->g_n = -1;
}

hipEvent_t take_event(kzk_plan* p) {
    if (!p->ev_pool.empty()) {
        hipEvent_t e = p->ev_pool.back();
        p->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one launch with events when profiling is on.
struct ProfScope {
    kzk_plan* p;
    int kind;
    hipEvent_t a = nullptr;
    ProfScope(kzk_plan* p_, int kind_) : p(p_), kind(kind_) {
        if (p->prof && p->prof_now && (a = take_event(p))) (void)hipEventRecord(a, p->stream);
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = take_event(p);
        if (!b) { p->ev_pool.push_back(a); return; }
        (void)hipEventRecord(b, p->stream);
        p->ev_used.push_back({kind, a, b});
    }
};

kzk_status check_params(const kzk_params& q) {
    if ((!pow2(q.n_tau) && !gen_k(q.n_tau)) || !pow2(q.n_y)) return KZK_ERR_SIZE;
    if (q.n_tau < 32 || q.n_tau > 8192 || q.n_y < 16 || q.n_y > 8192) return KZK_ERR_SIZE;
    if (!(q.L_tau > 0) || !(q.L_y > 0) || !(q.h > 0) || !std::isfinite(q.h)) return KZK_ERR_ARG;
    if (q.dtype != KZK_F32 && q.dtype != KZK_F64) return KZK_ERR_ARG;
    if (!(q.A >= 0) || !std::isfinite(q.A) || !std::isfinite(q.D) || !std::isfinite(q.nl)) return KZK_ERR_ARG;
    if (!(q.weno_eps > 0)) return KZK_ERR_ARG;
    if (q.lf_scope != 0) return KZK_ERR_ARG;
    if (q.cfl_max < 0) return KZK_ERR_ARG;
    if ((q.D_step || q.nl_node) && q.n_steps_max < 0) return KZK_ERR_ARG;
    if (q.scheme != 0 && q.scheme != 1) return KZK_ERR_ARG;
    if (!(q.reg_eps >= 0) || !std::isfinite(q.reg_eps)) return KZK_ERR_ARG;
    if (q.vel != 0 && q.vel != 1) return KZK_ERR_ARG;
    if (q.state_fp64 != 0 && q.state_fp64 != 1) return KZK_ERR_ARG;
    if (q.state_fp64 && q.dtype == KZK_F32 && q.reg_eps > 0) return KZK_ERR_ARG;
    if (q.vel == 1) {
        if (q.vel_modes < 1 || !q.vel_phi || !q.vel_theta || q.n_steps_max < 1 || q.n_steps_max > 65534)
            return KZK_ERR_ARG;
        if (!(q.vel_lambda > 0) || !(q.vel_c0 > 0) || !(q.vel_sigma_u >= 0) || !std::isfinite(q.vel_lambda) ||
            !std::isfinite(q.vel_c0) || !std::isfinite(q.vel_sigma_u))
            return KZK_ERR_ARG;
    }
    return KZK_OK;
}

// Default y-pass block size: the smallest supported one whose column tiles
// are at least 32 bytes wide (W complex values) in every instance, so that
// the tau-pass reads and writes row segments of 32 bytes or more; smaller
// blocks use less LDS, so more of them share a compute unit and their load,
// transform and store phases overlap.
int default_y_threads(const kzk_plan* p) {
    const int cands[3] = {256, 512, 1024};
    int last = 0;
    for (int nt : cands) {
        if (!kzk::y_threads_supported(p->dtype == KZK_F64, nt) || nt * 16 < p->max_ny) continue;
        last = nt;
        bool wide = true;
        for (const InstDesc& d : p->desc) {
            const int W = std::min(nt * 16 / d.n_y, d.M);
            if (W < d.M && (size_t)W * 2 * p->esz < 32) wide = false;
        }
        if (wide) return nt;
    }
    return last;
}

// Default tau-pass block size: 256 threads (two blocks of 64 KB per compute
// unit in FP32, whose load, transform and store phases interleave); the
// autotuner also tries TAU_THREADS_WIDE in FP32.
int default_tau_threads(const kzk_plan*) { return kzk::TAU_THREADS; }

// Transport (vel = 1): the work arrays, the transverse pass's work list and
// the velocity tables of every solve at the nodes x_n = x0 + n h,
// n = 0 .. n_steps_max (Algorithm 1, evaluated on the device in FP64 from the
// per-mode constants built here: K_n lambda with K_n equispaced in
// [0.1/L, 9/L], L = 4 lambda, and |U~(K_n)| / c0 = sqrt(E(K_n)/N) / c0 with
// E(K) = sigma_u^2 K^3 L^4 exp(-(K L/2)^2) / 8).
kzk_status setup_transport(kzk_plan* p, const kzk_params* params) {
    const size_t ub = p->u_off[p->n_inst] * p->esz;
    kzk_status st;
    if ((st = dev_alloc(p, &p->dUph, ub)) != KZK_OK || (st = dev_alloc(p, &p->dByp, ub)) != KZK_OK ||
        (st = dev_alloc(p, &p->dBys, p->state_elems * 2 * p->esz)) != KZK_OK)
        return st;
    std::vector<kzk::YwItem> items;
    for (int i = 0; i < p->n_inst; ++i)
        for (int k0 = 0; k0 < p->desc[i].n_tau; k0 += kzk::YW_THREADS)
            for (int j0 = 0; j0 < p->desc[i].n_y; j0 += kzk::YW_SEG) items.push_back({i, k0, j0});
    p->n_yw_items = (int)items.size();
    if ((st = dev_alloc(p, (void**)&p->dYw, sizeof(kzk::YwItem) * items.size())) != KZK_OK) return st;
    if (hipMemcpy(p->dYw, items.data(), sizeof(kzk::YwItem) * items.size(), hipMemcpyHostToDevice) != hipSuccess)
        return KZK_ERR_DEVICE;
    for (int i = 0; i < p->n_inst; ++i) {
        const kzk_params& q = params[i];
        const int N = q.vel_modes, nodes = q.n_steps_max + 1, ny = q.n_y;
        const double L = 4.0 * q.vel_lambda, kmin = 0.1 / L, kmax = 9.0 / L;
        std::vector<double> m(5 * (size_t)N);
        for (int n = 0; n < N; ++n) {
            const double K = N > 1 ? kmin + (kmax - kmin) * (double)n / (double)(N - 1) : kmin;
            const double E = 0.125 * q.vel_sigma_u * q.vel_sigma_u * K * K * K * L * L * L * L *
                             std::exp(-(K * L / 2.0) * (K * L / 2.0));
            m[n] = K * q.vel_lambda;
            m[N + n] = std::sqrt(E / (double)N) / q.vel_c0;
            m[2 * N + n] = std::cos(q.vel_theta[n]);
            m[3 * N + n] = std::sin(q.vel_theta[n]);
            m[4 * N + n] = q.vel_phi[n];
        }
        void *dm = nullptr, *tab = nullptr, *amax = nullptr;
        if ((st = dev_alloc(p, &dm, sizeof(double) * m.size())) != KZK_OK ||
            (st = dev_alloc(p, &tab, sizeof(double) * 3 * (size_t)ny * nodes)) != KZK_OK ||
            (st = dev_alloc(p, &amax, sizeof(double) * nodes)) != KZK_OK)
            return st;
        if (hipMemcpy(dm, m.data(), sizeof(double) * m.size(), hipMemcpyHostToDevice) != hipSuccess)
            return KZK_ERR_DEVICE;
        p->desc[i].vel_tab = static_cast<const double*>(tab);
        p->desc[i].vel_amax = static_cast<const double*>(amax);
        // the kernels read n_y and y0, dy of instance i from the descriptors
        if (hipMemcpy(p->dDesc + i, &p->desc[i], sizeof(InstDesc), hipMemcpyHostToDevice) != hipSuccess)
            return KZK_ERR_DEVICE;
        if (kzk::launch_velocity(p->dDesc, i, static_cast<const double*>(dm), N, q.x0, q.h, nodes,
                                 static_cast<double*>(tab), static_cast<double*>(amax), p->stream) != hipSuccess)
            return KZK_ERR_DEVICE;
    }
    return hipStreamSynchronize(p->stream) == hipSuccess ? KZK_OK : KZK_ERR_DEVICE;
}

// Descriptors, work lists and tables for the current y-pass and tau-pass
// block sizes.
kzk_status layout(kzk_plan* p) {
    std::vector<TauItem> tau, tau_adj;
    std::vector<YItem> ys;
    for (int i = 0; i < p->n_inst; ++i) {
        InstDesc& d = p->desc[i];
        // column tiles of W modes, W a power of two dividing M (2^K for M = 7 * 2^K)
        int W = std::min(p->y_threads * 16 / d.n_y, p->gk ? (1 << p->gk) : d.M);
        d.W = W;
        d.log2W = ilog2i(W);
        // lines of M/16 threads; with M = 7 * 2^K they sit in groups of 2^(K-1)
        d.rows_per_tau_block = p->gk ? p->tau_threads >> (p->gk - 1) : p->tau_threads * 16 / d.M;
        const int rows_adj = p->gk ? kzk::TAU_THREADS >> (p->gk - 1) : kzk::TAU_THREADS * 16 / d.M;
        for (int r = 0; r < d.n_y; r += d.rows_per_tau_block) tau.push_back({i, r});
        for (int r = 0; r < d.n_y; r += rows_adj) tau_adj.push_back({i, r});
        for (int m = 0; m < d.M; m += W) ys.push_back({i, m});
    }
    // the item arrays are sized for the largest case at create (W >= 1,
    // TAU_THREADS-thread tau blocks)
    if ((int)tau.size() > p->max_tau_items || (int)tau_adj.size() > p->max_tau_items) return KZK_ERR_STATE;
    p->n_tau_items = (int)tau.size();
    p->n_tau_adj_items = (int)tau_adj.size();
    p->n_y_items = (int)ys.size();
    p->tau_prog = p->gk ? 0 : 1;
    for (const InstDesc& d : p->desc)
        if (d.M / 16 < d.W || d.M < 256) p->tau_prog = 0;
    p->y_full = 1;
    for (const InstDesc& d : p->desc)
        if (d.W < 1 || d.W * d.n_y != 16 * p->y_threads || d.n_y < 512) p->y_full = 0;
    // 8192-row columns: full tiles only, in the variant that loads their twiddles per stage
    if (p->max_ny > 4096) {
        if (!p->y_full) return KZK_ERR_SIZE;
        p->y_full = 2;
    }
    p->y_grid = kzk::y_resident_blocks(p->dtype == KZK_F64, p->s64, p->y_threads, p->y_full, p->device);
    if (p->y_grid <= 0) return KZK_ERR_DEVICE;
    if (hipMemcpy(p->dDesc, p->desc.data(), sizeof(InstDesc) * p->n_inst, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->dTau, tau.data(), sizeof(TauItem) * tau.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->dTauAdj, tau_adj.data(), sizeof(TauItem) * tau_adj.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->dY, ys.data(), sizeof(YItem) * ys.size(), hipMemcpyHostToDevice) != hipSuccess)
        return KZK_ERR_DEVICE;
    return KZK_OK;
}

kzk_status build_tables(kzk_plan* p, int step, bool only_scheduled) {
    for (int i = 0; i < p->n_inst; ++i) {
        bool sched = p->desc[i].D_step != nullptr;
        if (only_scheduled && !sched) continue;
        int st = sched ? std::min<long long>(step, std::max<long long>(0, (long long)p->Dsched[i].size() - 1)) : 0;
        ProfScope ps(p, KZK_KIND_TABLES);
        hipError_t e = p->dtype == KZK_F32
            ? kzk::launch_tables<float>(p->dDesc, i, p->desc[i].W * p->desc[i].Nh, p->desc[i].M / p->desc[i].W,
                                        p->dTab, st, p->stream)
            : kzk::launch_tables<double>(p->dDesc, i, p->desc[i].W * p->desc[i].Nh, p->desc[i].M / p->desc[i].W,
                                         p->dTab, st, p->stream);
        if (e != hipSuccess) return KZK_ERR_DEVICE;
    }
    return KZK_OK;
}

// tiled = 1: spectra in the column-tile layout of the y-pass (internal arrays);
// tiled = 0: row-major spectra (the single-operator transform entries).
hipError_t tau(kzk_plan* p, int mode, const void* u_in, void* u_out, const void* Cin, void* Bout, int node,
               int tiled = 1) {
    ProfScope ps(p, mode == 2 ? KZK_KIND_TAU : KZK_KIND_TRANSFORM);
    if (p->dtype == KZK_F32)
        return kzk::launch_tau<float>(mode, p->tau_threads, p->dDesc, p->dTau, p->n_tau_items, (const float*)u_in,
                                      (float*)u_out, Cin, Bout, p->dTw, p->dTwSt, p->log2_ntw, node, tiled,
                                      p->tau_prog, p->gk, p->tau_mr, p->dStatus, p->stream);
    return kzk::launch_tau<double>(mode, p->tau_threads, p->dDesc, p->dTau, p->n_tau_items, (const double*)u_in,
                                   (double*)u_out, Cin, Bout, p->dTw, p->dTwSt, p->log2_ntw, node, tiled,
                                   p->tau_prog, p->gk, p->tau_mr, p->dStatus, p->stream);
}

// step: the ExpRK22 step, for instances with a D schedule (the y-pass
// computes their multipliers; the others read the tables built at create).
hipError_t ypass(kzk_plan* p, int stage, int step = 0) {
    ProfScope ps(p, stage == 1 ? KZK_KIND_Y1 : stage == 2 ? KZK_KIND_Y2 : KZK_KIND_TRANSFORM);
    const void* by = stage > 0 && p->transport ? p->dBys : nullptr;
    if (p->dtype == KZK_F32)
        return kzk::launch_y<float>(stage, p->s64, p->y_ntl, p->y_threads, p->y_full, p->dDesc, p->dY, p->n_y_items,
                                    p->y_grid, p->dC, p->dB, by, p->dP, p->dU, p->dTab, p->dTwSt, step, p->stream);
    return kzk::launch_y<double>(stage, 0, p->y_ntl, p->y_threads, p->y_full, p->dDesc, p->dY, p->n_y_items, p->y_grid,
                                 p->dC, p->dB, by, p->dP, p->dU, p->dTab, p->dTwSt, step, p->stream);
}

// The mean tau-mode column of the solves with the regularised multiplier,
// after y-pass stage `stage` of step s (stage 2 only with transport).
hipError_t dc_column(kzk_plan* p, int stage, int step) {
    if (!p->any_reg || (stage == 2 && !p->transport)) return hipSuccess;
    ProfScope ps(p, stage == 1 ? KZK_KIND_Y1 : KZK_KIND_Y2);
    const void* by = p->transport ? p->dBys : nullptr;
    if (p->dtype == KZK_F32)
        return kzk::launch_dc<float>(stage, p->dDesc, p->n_inst, p->dC, p->dP, p->dU, by, p->dTwSt, step, p->stream);
    return kzk::launch_dc<double>(stage, p->dDesc, p->n_inst, p->dC, p->dP, p->dU, by, p->dTwSt, step, p->stream);
}

// b at node x_node with transport (Sec. 3.4 eq. (21)-(22)): the tau-pass
// leaves the spectrum of the tau face fluxes (axial and Burgers terms) in dB
// and the physical field in dUph; the transverse pass writes its part of b
// (WENO5 of U_perp u along y plus the source) to dByp, whose tau-transform
// is dBys.  The y-pass then takes sigma_m dB + dBys.
kzk_status transport_b(kzk_plan* p, int node) {
    if (tau(p, 3, nullptr, p->dUph, p->dC, p->dB, node) != hipSuccess) return KZK_ERR_DEVICE;
    {
        ProfScope ps(p, KZK_KIND_TRANSPORT);
        hipError_t e = p->dtype == KZK_F32
            ? kzk::launch_yweno<float>(p->dDesc, p->dYw, p->n_yw_items, (const float*)p->dUph, (float*)p->dByp, node,
                                       p->dStatus, p->stream)
            : kzk::launch_yweno<double>(p->dDesc, p->dYw, p->n_yw_items, (const double*)p->dUph, (double*)p->dByp,
                                        node, p->dStatus, p->stream);
        if (e != hipSuccess) return KZK_ERR_DEVICE;
    }
    if (tau(p, 0, p->dByp, nullptr, nullptr, p->dBys, 0) != hipSuccess) return KZK_ERR_DEVICE;
    return KZK_OK;
}

// b at a stage node: the fused tau-pass, or the three passes of transport.
kzk_status stage_b(kzk_plan* p, int node) {
    if (p->transport) return transport_b(p, node);
    return tau(p, 2, nullptr, nullptr, p->dC, p->dB, node) == hipSuccess ? KZK_OK : KZK_ERR_DEVICE;
}

// Steps s .. s+n-1 on the spectral state (dU, with dC its tau-spectrum per y-row).
// ExpRK22 (Algorithm 2): tau-pass at x_n, y-pass stage 1, tau-pass at x_{n+1},
// y-pass stage 2.  Exponential Euler: its step is the first stage, U* = E U +
// h Phi1 B, which y-pass stage 1 leaves as C~*; the state U is its y-transform
// (y-pass stage 0).
kzk_status enqueue_steps(kzk_plan* p, int first, int n) {
    kzk_status st;
    for (int s = first; s < first + n; ++s) {
        p->prof_now = s % p->prof_every == 0;
        if ((st = stage_b(p, s)) != KZK_OK) return st;
        if (ypass(p, 1, s) != hipSuccess) return KZK_ERR_DEVICE;
        if (dc_column(p, 1, s) != hipSuccess) return KZK_ERR_DEVICE;
        if (p->scheme == 1) {
            if (ypass(p, 0) != hipSuccess) return KZK_ERR_DEVICE;
            continue;
        }
        if ((st = stage_b(p, s + 1)) != KZK_OK) return st;
        if (ypass(p, 2, s) != hipSuccess) return KZK_ERR_DEVICE;
        if (dc_column(p, 2, s) != hipSuccess) return KZK_ERR_DEVICE;
    }
    p->prof_now = true;
    return KZK_OK;
}

hipError_t tau_adj(kzk_plan* p, int stage, const void* Tin, const void* Rin, const void* ustore, void* out, int node) {
    ProfScope ps(p, KZK_KIND_ADJ_TAU);
    if (p->dtype == KZK_F32)
        return kzk::launch_tau_adj<float>(stage, p->dDesc, p->dTauAdj, p->n_tau_adj_items, Tin, Rin,
                                          (const float*)ustore, out, p->dTw, p->dTwSt, p->log2_ntw, node, p->gk,
                                          p->dStatus, p->stream);
    return kzk::launch_tau_adj<double>(stage, p->dDesc, p->dTauAdj, p->n_tau_adj_items, Tin, Rin,
                                       (const double*)ustore, out, p->dTw, p->dTwSt, p->log2_ntw, node, p->gk,
                                       p->dStatus, p->stream);
}

hipError_t y_adj(kzk_plan* p, int stage, const void* In, void* Lh, void* Tout, void* Rout) {
    ProfScope ps(p, KZK_KIND_ADJ_Y);
    if (p->dtype == KZK_F32)
        return kzk::launch_y_adj<float>(stage, p->y_threads, p->max_ny > 4096, p->dDesc, p->dY, p->n_y_items, In,
                                        Lh, Tout, Rout, p->dTab, p->dTwSt, p->stream);
    return kzk::launch_y_adj<double>(stage, p->y_threads, p->max_ny > 4096, p->dDesc, p->dY, p->n_y_items, In, Lh,
                                     Tout, Rout, p->dTab, p->dTwSt, p->stream);
}

// u -> state: tau-spectrum per row (dC), then the full spectrum (dU).
kzk_status enqueue_forward(kzk_plan* p, const void* u) {
    if (tau(p, 0, u, nullptr, nullptr, p->dC, 0) != hipSuccess) return KZK_ERR_DEVICE;
    if (ypass(p, 0) != hipSuccess) return KZK_ERR_DEVICE;
    return KZK_OK;
}

kzk_status enqueue_march(kzk_plan* p, void* u, int first, int n) {
    if (enqueue_forward(p, u) != KZK_OK) return KZK_ERR_DEVICE;
    kzk_status st = enqueue_steps(p, first, n);
    if (st != KZK_OK) return st;
    if (tau(p, 1, nullptr, u, p->dC, nullptr, 0) != hipSuccess) return KZK_ERR_DEVICE;
    return KZK_OK;
}

kzk_status check_range(const kzk_plan* p, long long first, long long n) {
    if (first < 0 || n < 0) return KZK_ERR_ARG;
    if (p->steps_limit >= 0 && first + n > p->steps_limit) return KZK_ERR_STATE;
    return KZK_OK;
}

}  // namespace

extern "C" {

const char* kzk_status_str(kzk_status s) {
    // callers may pass any integer: read the bits as an int, not as the enum
    // (a value outside the enumerators is not a valid kzk_status in C++)
    static_assert(sizeof(kzk_status) == sizeof(int32_t), "kzk_status is passed as a 32-bit int");
    int32_t v;
    std::memcpy(&v, &s, sizeof(v));
    switch (v) {
    case KZK_OK: return "ok";
    case KZK_ERR_ARG: return "invalid argument";
    case KZK_ERR_SIZE: return "grid size not supported";
    case KZK_ERR_OOM: return "out of device memory";
    case KZK_ERR_DEVICE: return "HIP error";
    case KZK_ERR_CFL: return "CFL limit exceeded";
    case KZK_ERR_NONFINITE: return "non-finite value in the field";
    case KZK_ERR_STATE: return "invalid state or step range";
    }
    return "unknown status";
}

void kzk_destroy(kzk_plan* p) {
    if (!p) return;
    drop_graph(p);
    for (auto& e : p->ev_used) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    for (auto e : p->ev_pool) (void)hipEventDestroy(e);
    for (void* q : p->owned) (void)hipFree(q);
    delete p;
}

}  // extern "C"

namespace {

// kzk_create, with the device memory taken from [arena, arena + arena_cap)
// when arena is not null (KZK_ERR_SIZE if it does not fit there).
kzk_status create_plan(const kzk_params* params, int32_t n_inst, void* hip_stream, char* arena, size_t arena_cap,
                       kzk_plan** out) {
    if (!out) return KZK_ERR_ARG;
    *out = nullptr;
    if (!params || n_inst < 1) return KZK_ERR_ARG;
    for (int i = 0; i < n_inst; ++i) {
        kzk_status st = check_params(params[i]);
        if (st != KZK_OK) return st;
        if (params[i].dtype != params[0].dtype || params[i].scheme != params[0].scheme ||
            params[i].vel != params[0].vel || params[i].state_fp64 != params[0].state_fp64)
            return KZK_ERR_ARG;
        // n_tau = 7 * 2^(K+1): one tau length for the whole plan
        if ((gen_k(params[i].n_tau) || gen_k(params[0].n_tau)) && params[i].n_tau != params[0].n_tau)
            return KZK_ERR_SIZE;
    }
    kzk_plan* p = new (std::nothrow) kzk_plan();
    if (!p) return KZK_ERR_OOM;
    p->scheme = params[0].scheme;
    p->transport = params[0].vel == 1;
    p->gk = gen_k(params[0].n_tau);
    p->s64 = params[0].state_fp64 == 1 && params[0].dtype == KZK_F32;
    p->arena = arena;
    p->arena_cap = arena ? arena_cap : 0;
    p->n_inst = n_inst;
    p->dtype = params[0].dtype;
    p->esz = p->dtype == KZK_F32 ? 4 : 8;
    p->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&p->device);
    p->params.assign(params, params + n_inst);
    p->Dsched.resize(n_inst);
    p->nlsched.resize(n_inst);
    p->desc.resize(n_inst);
    p->u_off.resize(n_inst + 1);

    size_t so = 0, uo = 0, to = 0, nsched = 0;
    int ntw = 0, max_tau_items = 0, max_y_items = 0;
    for (int i = 0; i < n_inst; ++i) {
        const kzk_params& q = params[i];
        InstDesc& d = p->desc[i];
        std::memset(&d, 0, sizeof(d));
        d.n_tau = q.n_tau;
        d.n_y = q.n_y;
        p->max_ny = std::max(p->max_ny, q.n_y);
        d.M = q.n_tau / 2;
        d.Nh = q.n_y / 2 + 1;
        d.off_state = (long long)so;
        d.off_u = (long long)uo;
        d.off_tab = (long long)to;
        d.tab_size = (long long)d.M * d.Nh;
        d.dtau = q.L_tau / q.n_tau;
        d.h = q.h;
        d.L_tau = q.L_tau;
        d.L_y = q.L_y;
        d.A = q.A;
        d.weno_eps = q.weno_eps;
        d.D_const = q.D;
        d.nl_const = q.nl;
        d.cfl_max = q.cfl_max > 0 ? q.cfl_max : 1.0;
        d.scheme = q.scheme;
        d.reg_eps = q.reg_eps;
        if (q.reg_eps > 0) p->any_reg = true;
        d.vel = q.vel;
        d.y0 = q.y0;
        d.dy = q.L_y / q.n_y;
        p->u_off[i] = uo;
        so += (size_t)d.M * q.n_y;
        uo += (size_t)q.n_tau * q.n_y;
        to += (size_t)d.M * d.Nh;
        ntw = std::max(ntw, std::max(q.n_tau, q.n_y));
        const int rows256 = p->gk ? kzk::TAU_THREADS >> (p->gk - 1) : kzk::TAU_THREADS * 16 / d.M;
        max_tau_items += (q.n_y + rows256 - 1) / rows256;
        max_y_items += d.M;   // W >= 1
        if (q.D_step) {
            p->Dsched[i].assign(q.D_step, q.D_step + q.n_steps_max);
            p->any_D_sched = true;
        }
        if (q.nl_node) p->nlsched[i].assign(q.nl_node, q.nl_node + q.n_steps_max + 1);
        // the schedules, and with transport the velocity tables (nodes 0 .. n_steps_max), bound the steps
        if (q.D_step || q.nl_node || q.vel == 1) {
            long long lim = q.n_steps_max;
            p->steps_limit = p->steps_limit < 0 ? lim : std::min(p->steps_limit, lim);
        }
        nsched += p->Dsched[i].size() + p->nlsched[i].size();
    }
    p->u_off[n_inst] = uo;
    p->state_elems = so;
    p->tab_elems = to;
    // FP64 spectral state (FP64 plans, or FP32 with state_fp64): above a
    // quarter of the 256 MB Infinity Cache per array (a step streams about
    // six such arrays) the y-passes load the state non-temporally; below
    // it, where the arrays largely stay cached, cached loads are faster.
    {
        constexpr size_t NTL_MIN_BYTES = (size_t)64 << 20;
        const bool s64state = p->dtype == KZK_F64 || p->s64;
        p->y_ntl = s64state && p->state_elems * 16 > NTL_MIN_BYTES;
    }
    for (int i = 0; i < n_inst; ++i) p->desc[i].tab_stride = (long long)to;
    // the tau-pass twiddle table: e^{-2 pi i k / 2^log2_ntw}, or with
    // n_tau = 7 * 2^(K+1) the table e^{-2 pi i k / n_tau} of that length
    if (p->gk) ntw = params[0].n_tau;
    p->ntw = ntw;
    p->log2_ntw = p->gk ? 0 : ilog2i(ntw);

    const size_t cz = 2 * p->esz;   // bytes per complex
    kzk_status st = KZK_OK;
    const size_t czs = p->s64 ? 2 * sizeof(double) : cz;   // bytes per complex of the state and stage value
    if ((st = dev_alloc(p, &p->dC, so * cz)) != KZK_OK || (st = dev_alloc(p, &p->dB, so * cz)) != KZK_OK ||
        (st = dev_alloc(p, &p->dP, so * czs)) != KZK_OK || (st = dev_alloc(p, &p->dU, so * czs)) != KZK_OK ||
        (st = dev_alloc(p, &p->dTab, 3 * to * cz)) != KZK_OK ||
        (st = dev_alloc(p, &p->dTw, (size_t)ntw * cz)) != KZK_OK ||
        (st = dev_alloc(p, (void**)&p->dDesc, sizeof(InstDesc) * n_inst)) != KZK_OK ||
        (st = dev_alloc(p, (void**)&p->dTau, sizeof(TauItem) * max_tau_items)) != KZK_OK ||
        (st = dev_alloc(p, (void**)&p->dTauAdj, sizeof(TauItem) * max_tau_items)) != KZK_OK ||
        (st = dev_alloc(p, &p->dTwSt, (size_t)kzk::stage_twiddle_entries() * cz)) != KZK_OK ||
        (st = dev_alloc(p, (void**)&p->dY, sizeof(YItem) * max_y_items)) != KZK_OK ||
        (st = dev_alloc(p, (void**)&p->dStatus, 256)) != KZK_OK ||
        (st = dev_alloc(p, (void**)&p->dSched, sizeof(double) * (nsched + 1))) != KZK_OK) {
        kzk_destroy(p);
        return st;
    }
    p->max_tau_items = max_tau_items;

    // coefficient schedules
    {
        std::vector<double> all;
        all.reserve(nsched);
        std::vector<size_t> offD(n_inst), offN(n_inst);
        for (int i = 0; i < n_inst; ++i) {
            offD[i] = all.size();
            all.insert(all.end(), p->Dsched[i].begin(), p->Dsched[i].end());
            offN[i] = all.size();
            all.insert(all.end(), p->nlsched[i].begin(), p->nlsched[i].end());
        }
        if (!all.empty() &&
            hipMemcpy(p->dSched, all.data(), sizeof(double) * all.size(), hipMemcpyHostToDevice) != hipSuccess) {
            kzk_destroy(p);
            return KZK_ERR_DEVICE;
        }
        for (int i = 0; i < n_inst; ++i) {
            p->desc[i].D_step = p->Dsched[i].empty() ? nullptr : p->dSched + offD[i];
            p->desc[i].nl_node = p->nlsched[i].empty() ? nullptr : p->dSched + offN[i];
        }
    }
    // flux-difference symbols sigma_m = -(2 sin^2(pi m/n_tau) + i sin(2 pi m/n_tau)) / dtau
    // (FP64, half-angle form for the low modes; m = 0 zero), in the working precision
    {
        size_t tot = 0;
        for (int i = 0; i < n_inst; ++i) tot += (size_t)p->desc[i].M;
        std::vector<double> sg(2 * tot);
        size_t o = 0;
        for (int i = 0; i < n_inst; ++i) {
            const InstDesc& d = p->desc[i];
            for (int m = 0; m < d.M; ++m, ++o) {
                const double a = M_PI * (double)m / (double)d.n_tau;
                const double sh = std::sin(a), ch = std::cos(a);
                sg[2 * o] = m ? -2.0 * sh * sh / d.dtau : 0.0;
                sg[2 * o + 1] = m ? -2.0 * sh * ch / d.dtau : 0.0;
            }
        }
        hipError_t e = hipSuccess;
        if ((st = dev_alloc(p, &p->dSig, sg.size() * p->esz)) != KZK_OK) { kzk_destroy(p); return st; }
        if (p->dtype == KZK_F32) {
            std::vector<float> f(sg.begin(), sg.end());
            e = hipMemcpy(p->dSig, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice);
        } else {
            e = hipMemcpy(p->dSig, sg.data(), sg.size() * sizeof(double), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) { kzk_destroy(p); return KZK_ERR_DEVICE; }
        o = 0;
        for (int i = 0; i < n_inst; ++i) {
            p->desc[i].sigma = (const char*)p->dSig + o * 2 * p->esz;
            o += (size_t)p->desc[i].M;
        }
    }
    // twiddles exp(-2 pi i k / ntw) in FP64, stored in the working precision
    // (ntw = 2^log2_ntw, or n_tau = 7 * 2^(K+1))
    {
        std::vector<double> tw(2 * (size_t)ntw);
        for (int k = 0; k < ntw; ++k) {
            double a = 2.0 * M_PI * (double)k / (double)ntw;
            tw[2 * k] = std::cos(a);
            tw[2 * k + 1] = -std::sin(a);
        }
        hipError_t e;
        if (p->dtype == KZK_F32) {
            std::vector<float> f(tw.begin(), tw.end());
            e = hipMemcpy(p->dTw, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice);
        } else {
            e = hipMemcpy(p->dTw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) { kzk_destroy(p); return KZK_ERR_DEVICE; }
        std::vector<double> st64(2 * (size_t)kzk::stage_twiddle_entries());
        kzk::stage_twiddles(st64.data());
        if (p->dtype == KZK_F32) {
            std::vector<float> f(st64.begin(), st64.end());
            e = hipMemcpy(p->dTwSt, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice);
        } else {
            e = hipMemcpy(p->dTwSt, st64.data(), st64.size() * sizeof(double), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) { kzk_destroy(p); return KZK_ERR_DEVICE; }
    }
    if (p->transport && (st = setup_transport(p, params)) != KZK_OK) {
        kzk_destroy(p);
        return st;
    }
    if (hipMemset(p->dStatus, 0, 256) != hipSuccess) { kzk_destroy(p); return KZK_ERR_DEVICE; }
    p->y_threads = default_y_threads(p);
    p->tau_threads = default_tau_threads(p);
    if ((st = layout(p)) != KZK_OK || (st = build_tables(p, 0, false)) != KZK_OK) {
        kzk_destroy(p);
        return st;
    }
    if (hipStreamSynchronize(p->stream) != hipSuccess) { kzk_destroy(p); return KZK_ERR_DEVICE; }
    *out = p;
    return KZK_OK;
}

}  // namespace

extern "C" {

kzk_status kzk_create(const kzk_params* params, int32_t n_inst, void* hip_stream, kzk_plan** out) {
    return create_plan(params, n_inst, hip_stream, nullptr, 0, out);
}

kzk_status kzk_set_stream(kzk_plan* p, void* s) {
    if (!p) return KZK_ERR_ARG;
    p->stream = (hipStream_t)s;
    return KZK_OK;
}

kzk_status kzk_set_graph(kzk_plan* p, int32_t enable) {
    if (!p) return KZK_ERR_ARG;
    p->graph_on = enable != 0;
    if (!p->graph_on) drop_graph(p);
    return KZK_OK;
}

int32_t kzk_get_y_threads(const kzk_plan* p) { return p ? p->y_threads : 0; }

int32_t kzk_get_tau_threads(const kzk_plan* p) { return p ? p->tau_threads : 0; }

kzk_status kzk_set_tau_threads(kzk_plan* p, int32_t threads) {
    if (!p) return KZK_ERR_ARG;
    if (threads == 0) threads = default_tau_threads(p);
    if (!kzk::tau_threads_supported(p->dtype == KZK_F64, threads)) return KZK_ERR_ARG;
    if (p->gk && threads != kzk::TAU_THREADS) return KZK_ERR_ARG;   // lengths 7 * 2^K: one block size
    if (hipStreamSynchronize(p->stream) != hipSuccess) return KZK_ERR_DEVICE;
    drop_graph(p);
    p->tau_threads = threads;
    kzk_status st = layout(p);
    if (st != KZK_OK) return st;
    return hipStreamSynchronize(p->stream) == hipSuccess ? KZK_OK : KZK_ERR_DEVICE;
}


int32_t kzk_get_tau_fft_radix(const kzk_plan* p) { return p ? 1 << p->tau_mr : 0; }

kzk_status kzk_set_tau_fft_radix(kzk_plan* p, int32_t radix) {
    if (!p) return KZK_ERR_ARG;
    if (radix == 0) radix = 16;
    if (radix != 16 && radix != 8) return KZK_ERR_ARG;
    if (p->gk && radix != 16) return KZK_ERR_ARG;   // lengths 7 * 2^K: one schedule
    if (hipStreamSynchronize(p->stream) != hipSuccess) return KZK_ERR_DEVICE;
    drop_graph(p);
    p->tau_mr = radix == 16 ? 4 : 3;
    return KZK_OK;
}

kzk_status kzk_set_y_threads(kzk_plan* p, int32_t threads) {
    if (!p) return KZK_ERR_ARG;
    if (threads == 0) threads = default_y_threads(p);
    if (!kzk::y_threads_supported(p->dtype == KZK_F64, threads)) return KZK_ERR_ARG;
    if (threads * 16 < p->max_ny) return KZK_ERR_ARG;   // a column tile holds at least one column
    if (hipStreamSynchronize(p->stream) != hipSuccess) return KZK_ERR_DEVICE;
    drop_graph(p);
    const int old = p->y_threads;
    p->y_threads = threads;
    kzk_status st = layout(p);
    if (st != KZK_OK) {
        // not a layout this plan can take (8192-row columns without full tiles): keep the previous one
        p->y_threads = old;
        if (layout(p) != KZK_OK) return KZK_ERR_STATE;
        return st;
    }
    st = build_tables(p, 0, false);
    if (st != KZK_OK) return st;
    return hipStreamSynchronize(p->stream) == hipSuccess ? KZK_OK : KZK_ERR_DEVICE;
}

size_t kzk_inst_offset(const kzk_plan* p, int32_t i) {
    if (!p || i < 0 || i > p->n_inst) return (size_t)-1;
    return p->u_off[i];
}

kzk_status kzk_step(kzk_plan* p, void* u, int32_t first, int32_t n) {
    if (!p || !u) return KZK_ERR_ARG;
    kzk_status st = check_range(p, first, n);
    if (st != KZK_OK) return st;
    if (n == 0) return KZK_OK;
    if (!p->graph_on || p->prof) return enqueue_march(p, u, first, n);
    if (!p->stream) return KZK_ERR_STATE;   // the legacy default stream cannot be captured
    if (!(p->gexec && p->g_u == u && p->g_first == first && p->g_n == n)) {
        drop_graph(p);
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return KZK_ERR_DEVICE;
        kzk_status cs = enqueue_march(p, u, first, n);
        hipError_t e = hipStreamEndCapture(p->stream, &g);
        if (cs != KZK_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return cs != KZK_OK ? cs : KZK_ERR_DEVICE;
        }
        e = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) { p->gexec = nullptr; return KZK_ERR_DEVICE; }
        p->g_u = u;
        p->g_first = first;
        p->g_n = n;
    }
    return hipGraphLaunch(p->gexec, p->stream) == hipSuccess ? KZK_OK : KZK_ERR_DEVICE;
}

kzk_status kzk_profile_enable(kzk_plan* p, int32_t every) {
    if (!p || every < 0) return KZK_ERR_ARG;
    p->prof = every != 0;
    p->prof_every = every > 0 ? every : 1;
    p->prof_now = true;
    return KZK_OK;
}

kzk_status kzk_profile_read(kzk_plan* p, double* ms, int32_t* count, int32_t n_kinds) {
    if (!p || !ms || !count || n_kinds < 0) return KZK_ERR_ARG;
    for (int k = 0; k < n_kinds; ++k) { ms[k] = 0; count[k] = 0; }
    if (hipStreamSynchronize(p->stream) != hipSuccess) return KZK_ERR_DEVICE;
    kzk_status st = KZK_OK;
    for (auto& e : p->ev_used) {
        float t = 0;
        if (hipEventElapsedTime(&t, e.a, e.b) != hipSuccess) st = KZK_ERR_DEVICE;
        if (e.kind < n_kinds) { ms[e.kind] += t; count[e.kind] += 1; }
        p->ev_pool.push_back(e.a);
        p->ev_pool.push_back(e.b);
    }
    p->ev_used.clear();
    return st;
}

kzk_status kzk_poll(kzk_plan* p) {
    if (!p) return KZK_ERR_ARG;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return KZK_ERR_DEVICE;
    unsigned s = 0;
    if (hipMemcpy(&s, p->dStatus, sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess) return KZK_ERR_DEVICE;
    if (s) {
        if (hipMemset(p->dStatus, 0, sizeof(unsigned)) != hipSuccess) return KZK_ERR_DEVICE;
        if (hipDeviceSynchronize() != hipSuccess) return KZK_ERR_DEVICE;
    }
    if (s & kzk::ST_NONFINITE) return KZK_ERR_NONFINITE;
    if (s & kzk::ST_CFL) return KZK_ERR_CFL;
    return KZK_OK;
}

kzk_status kzk_eval_b(kzk_plan* p, const void* u, int32_t node, void* b) {
    if (!p || !u || !b) return KZK_ERR_ARG;
    if (node < 0 || (p->steps_limit >= 0 && node > p->steps_limit)) return KZK_ERR_STATE;
    if (tau(p, 0, u, nullptr, nullptr, p->dC, 0) != hipSuccess) return KZK_ERR_DEVICE;
    kzk_status st = stage_b(p, node);
    if (st != KZK_OK) return st;
    // the tau-pass leaves the spectrum of the face fluxes: apply the difference
    // (and add the transverse part of b with transport)
    const void* by = p->transport ? p->dBys : nullptr;
    for (int i = 0; i < p->n_inst; ++i) {
        const long long n = (long long)p->desc[i].M * p->desc[i].n_y;
        if ((p->dtype == KZK_F32 ? kzk::launch_flux_diff<float>(p->dDesc, i, n, p->dB, by, p->stream)
                                 : kzk::launch_flux_diff<double>(p->dDesc, i, n, p->dB, by, p->stream)) != hipSuccess)
            return KZK_ERR_DEVICE;
    }
    if (tau(p, 1, nullptr, b, p->dB, nullptr, 0) != hipSuccess) return KZK_ERR_DEVICE;
    return KZK_OK;
}

kzk_status kzk_tau_forward(kzk_plan* p, const void* u, void* spec) {
    if (!p || !u || !spec) return KZK_ERR_ARG;
    return tau(p, 0, u, nullptr, nullptr, spec, 0, 0) == hipSuccess ? KZK_OK : KZK_ERR_DEVICE;
}

kzk_status kzk_tau_inverse(kzk_plan* p, const void* spec, void* u) {
    if (!p || !u || !spec) return KZK_ERR_ARG;
    return tau(p, 1, nullptr, u, spec, nullptr, 0, 0) == hipSuccess ? KZK_OK : KZK_ERR_DEVICE;
}

kzk_status kzk_read_tables(kzk_plan* p, int32_t inst, void* out) {
    if (!p || !out || inst < 0 || inst >= p->n_inst) return KZK_ERR_ARG;
    const InstDesc& d = p->desc[inst];
    const size_t cz = 2 * p->esz, n = (size_t)d.tab_size;
    std::vector<char> tile(3 * n * cz), lin(3 * n * cz);
    if (hipStreamSynchronize(p->stream) != hipSuccess) return KZK_ERR_DEVICE;
    for (int t = 0; t < 3; ++t)
        if (hipMemcpy(tile.data() + t * n * cz, (char*)p->dTab + ((size_t)t * d.tab_stride + d.off_tab) * cz, n * cz,
                      hipMemcpyDeviceToHost) != hipSuccess)
            return KZK_ERR_DEVICE;
    for (int t = 0; t < 3; ++t)
        for (int m = 0; m < d.M; ++m)
            for (int q = 0; q < d.Nh; ++q) {
                const int c = m & (d.W - 1);
                const size_t src = (size_t)(m - c) * d.Nh + (size_t)q * d.W + c;
                const size_t dst = (size_t)m * d.Nh + q;
                std::memcpy(lin.data() + (t * n + dst) * cz, tile.data() + (t * n + src) * cz, cz);
            }
    return hipMemcpy(out, lin.data(), lin.size(), hipMemcpyHostToDevice) == hipSuccess ? KZK_OK : KZK_ERR_DEVICE;
}

}  // extern "C"

namespace {

// Grow the adjoint workspace: three spectra, ckpt physical fields for u^n
// and for u*, and nseg checkpoints of the spectral state.
kzk_status adjoint_workspace(kzk_plan* p, size_t ckpt, size_t nseg) {
    const size_t cz = 2 * p->esz, sb = p->state_elems * cz, ub = p->u_off[p->n_inst] * p->esz;
    if (!p->dL) {
        kzk_status st;
        if ((st = dev_alloc(p, &p->dL, sb)) != KZK_OK || (st = dev_alloc(p, &p->dM, sb)) != KZK_OK ||
            (st = dev_alloc(p, &p->dR, sb)) != KZK_OK)
            return st;
    }
    // a larger request replaces the old buffers (freed once the stream is idle)
    if (ckpt > p->adj_ckpt_cap || nseg > p->adj_seg_cap) {
        if (hipStreamSynchronize(p->stream) != hipSuccess) return KZK_ERR_DEVICE;
    }
    if (ckpt > p->adj_ckpt_cap) {
        dev_free(p, p->dUn);
        dev_free(p, p->dUs);
        p->adj_ckpt_cap = 0;
        kzk_status st;
        if ((st = dev_alloc(p, &p->dUn, ckpt * ub)) != KZK_OK || (st = dev_alloc(p, &p->dUs, ckpt * ub)) != KZK_OK)
            return st;
        p->adj_ckpt_cap = ckpt;
    }
    if (nseg > p->adj_seg_cap) {
        dev_free(p, p->dCk);
        p->adj_seg_cap = 0;
        kzk_status st = dev_alloc(p, &p->dCk, 2 * nseg * sb);
        if (st != KZK_OK) return st;
        p->adj_seg_cap = nseg;
    }
    return KZK_OK;
}

}  // namespace

namespace {

// Key of a plan in the tuning cache: device architecture, dtype, scheme and
// every solve's grid (and whether its multipliers are evaluated per step).
std::string tune_key(const kzk_plan* p) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) arch = prop.gcnArchName;
    std::string k = "kzk2|" + arch + (p->dtype == KZK_F32 ? "|f32|" : "|f64|") + std::to_string(p->scheme);
    for (const InstDesc& d : p->desc)
        k += "|" + std::to_string(d.n_tau) + "x" + std::to_string(d.n_y) + (d.D_step ? "s" : "") +
             (d.reg_eps > 0 ? "r" : "");
    return k;
}

// Look the key up in the cache file: the last line
// "<key> <y_threads> <tau_threads> <tau_fft_radix> <ms>" wins.
bool tune_lookup(const char* path, const std::string& key, int* yt, int* tt, int* rx) {
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    bool found = false;
    std::vector<char> line(1 << 16);
    while (std::fgets(line.data(), (int)line.size(), f)) {
        const char* sp = std::strchr(line.data(), ' ');
        if (!sp || (size_t)(sp - line.data()) != key.size() || std::strncmp(line.data(), key.c_str(), key.size()))
            continue;
        int a = 0, b = 0, c = 0;
        if (std::sscanf(sp + 1, "%d %d %d", &a, &b, &c) == 3) {
            *yt = a;
            *tt = b;
            *rx = c;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void tune_store(const char* path, const std::string& key, int yt, int tt, int rx, float ms) {
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %.4f\n", key.c_str(), yt, tt, rx, (double)ms);
    std::fclose(f);
}

}  // namespace

extern "C" int32_t kzk_autotune(kzk_plan* p, const void* u, int32_t n_trial) {
    if (!p || !u || n_trial < 1) return -(int32_t)KZK_ERR_ARG;
    if (p->steps_limit >= 0 && n_trial > p->steps_limit) n_trial = (int32_t)p->steps_limit;
    if (n_trial < 1) return -(int32_t)KZK_ERR_STATE;
    const char* cache = std::getenv("KZK_TUNE_CACHE");
    const std::string key = tune_key(p);
    kzk_status st = KZK_OK;
    // tau-pass block sizes this plan can take (one with n_tau = 7 * 2^(K+1))
    auto tau_ok = [&](int t) {
        return kzk::tau_threads_supported(p->dtype == KZK_F64, t) && (!p->gk || t == kzk::TAU_THREADS);
    };
    auto radix_ok = [&](int r) { return r == 16 || (r == 8 && !p->gk); };
    if (cache && *cache) {
        int yt = 0, tt = 0, rx = 0;
        if (tune_lookup(cache, key, &yt, &tt, &rx) && kzk::y_threads_supported(p->dtype == KZK_F64, yt) &&
            tau_ok(tt) && radix_ok(rx)) {
            if ((st = kzk_set_y_threads(p, yt)) != KZK_OK || (st = kzk_set_tau_threads(p, tt)) != KZK_OK ||
                (st = kzk_set_tau_fft_radix(p, rx)) != KZK_OK)
                return -(int32_t)st;
            return yt;
        }
    }
    const int ycands[3] = {1024, 512, 256};
    const int tcands[2] = {kzk::TAU_THREADS_WIDE, kzk::TAU_THREADS};
    const int rcands[2] = {16, 8};
    int best_y = p->y_threads, best_t = p->tau_threads, best_r = 1 << p->tau_mr;
    float best_ms = 1e30f;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -(int32_t)KZK_ERR_DEVICE;
    const bool prof = p->prof;
    p->prof = false;
    for (int c : ycands) {
        if (!kzk::y_threads_supported(p->dtype == KZK_F64, c) || c * 16 < p->max_ny) continue;
        if ((st = kzk_set_y_threads(p, c)) != KZK_OK) {
            if (st == KZK_ERR_SIZE) { st = KZK_OK; continue; }   // a layout this plan cannot take
            break;
        }
        for (int t : tcands) {
            if (!tau_ok(t)) continue;
            if ((st = kzk_set_tau_threads(p, t)) != KZK_OK) break;
            for (int r : rcands) {
                if (!radix_ok(r)) continue;
                if ((st = kzk_set_tau_fft_radix(p, r)) != KZK_OK) break;
                // one untimed step to warm up, then n_trial timed steps, on the plan's own state
                if ((st = enqueue_forward(p, u)) != KZK_OK) break;
                if ((st = enqueue_steps(p, 0, 1)) != KZK_OK) break;
                if ((st = enqueue_forward(p, u)) != KZK_OK) break;
                (void)hipEventRecord(a, p->stream);
                if ((st = enqueue_steps(p, 0, n_trial)) != KZK_OK) break;
                (void)hipEventRecord(b, p->stream);
                if (hipEventSynchronize(b) != hipSuccess) { st = KZK_ERR_DEVICE; break; }
                float ms = 0;
                (void)hipEventElapsedTime(&ms, a, b);
                if (ms < best_ms) { best_ms = ms; best_y = c; best_t = t; best_r = r; }
            }
            if (st != KZK_OK) break;
        }
        if (st != KZK_OK) break;
    }
    p->prof = prof;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipMemset(p->dStatus, 0, sizeof(unsigned));   // trial steps ran on scratch state
    if (st != KZK_OK) return -(int32_t)st;
    if ((st = kzk_set_y_threads(p, best_y)) != KZK_OK || (st = kzk_set_tau_threads(p, best_t)) != KZK_OK ||
        (st = kzk_set_tau_fft_radix(p, best_r)) != KZK_OK)
        return -(int32_t)st;
    if (cache && *cache) tune_store(cache, key, best_y, best_t, best_r, best_ms / (float)n_trial);
    return best_y;
}

extern "C" kzk_status kzk_adjoint(kzk_plan* p, const void* u0, const void* lam, int32_t first, int32_t n,
                                  int32_t ckpt, void* grad) {
    if (!p || !u0 || !lam || !grad || ckpt < 0) return KZK_ERR_ARG;
    // ExpRK22, zeroed mean, Burgers b, state in the working precision
    if (p->scheme != 0 || p->any_reg || p->transport || p->s64) return KZK_ERR_ARG;
    kzk_status st = check_range(p, first, n);
    if (st != KZK_OK) return st;
    const size_t cz = 2 * p->esz, sb = p->state_elems * cz, ub = p->u_off[p->n_inst] * p->esz;
    if (n == 0) {
        if (grad != lam && hipMemcpyAsync(grad, lam, ub, hipMemcpyDeviceToDevice, p->stream) != hipSuccess)
            return KZK_ERR_DEVICE;
        return KZK_OK;
    }
    int K = std::min<int>(ckpt, n);
    if (ckpt == 0) {
        // the longest checkpoint interval whose stored stage inputs (2 K fields)
        // and checkpoints (2 spectral states per segment) fit in half of the
        // device memory free now; K = n stores the whole march (no recomputation)
        size_t fr = 0, total = 0;
        if (hipMemGetInfo(&fr, &total) != hipSuccess) return KZK_ERR_DEVICE;
        const size_t budget = fr / 2;
        K = 1;
        for (int k = n; k >= 1; k = k > 1 ? (k + 1) / 2 : 0) {
            const size_t segs = (size_t)((n + k - 1) / k);
            if (2 * (size_t)k * ub + 2 * segs * sb <= budget) { K = k; break; }
        }
    }
    const int nseg = (n + K - 1) / K;
    if ((st = adjoint_workspace(p, (size_t)K, (size_t)nseg)) != KZK_OK) return st;
    char* ck = (char*)p->dCk;
    char* Un = (char*)p->dUn;
    char* Us = (char*)p->dUs;

    // Steps s0 .. s1-1 storing u^n and u* in physical space (stage inputs of
    // the nonlinear term, needed by its Jacobians).
    auto stored_steps = [&](int s0, int s1) -> kzk_status {
        for (int s = s0; s < s1; ++s) {
            if (tau(p, 3, nullptr, Un + (size_t)(s - s0) * ub, p->dC, p->dB, s) != hipSuccess) return KZK_ERR_DEVICE;
            if (ypass(p, 1, s) != hipSuccess) return KZK_ERR_DEVICE;
            if (tau(p, 3, nullptr, Us + (size_t)(s - s0) * ub, p->dC, p->dB, s + 1) != hipSuccess)
                return KZK_ERR_DEVICE;
            if (ypass(p, 2, s) != hipSuccess) return KZK_ERR_DEVICE;
        }
        return KZK_OK;
    };
    // forward sweep, keeping the spectral state at the start of every segment;
    // the last segment stores its stage inputs right away (it is the first one
    // the backward sweep needs, so it is not recomputed)
    if ((st = enqueue_forward(p, u0)) != KZK_OK) return st;
    for (int g = 0; g < nseg; ++g) {
        const int s0 = first + g * K, s1 = std::min(s0 + K, first + n);
        if (g == nseg - 1) {
            if ((st = stored_steps(s0, s1)) != KZK_OK) return st;
            break;
        }
        if (hipMemcpyAsync(ck + (size_t)(2 * g) * sb, p->dU, sb, hipMemcpyDeviceToDevice, p->stream) != hipSuccess ||
            hipMemcpyAsync(ck + (size_t)(2 * g + 1) * sb, p->dC, sb, hipMemcpyDeviceToDevice, p->stream) != hipSuccess)
            return KZK_ERR_DEVICE;
        if ((st = enqueue_steps(p, s0, s1 - s0)) != KZK_OK) return st;
    }
    // adjoint state L~ = tau-spectrum of dL/du at the end
    if (tau(p, 0, lam, nullptr, nullptr, p->dL, 0) != hipSuccess) return KZK_ERR_DEVICE;
    for (int g = nseg - 1; g >= 0; --g) {
        const int s0 = first + g * K, s1 = std::min(s0 + K, first + n);
        if (g < nseg - 1) {
            if (hipMemcpyAsync(p->dU, ck + (size_t)(2 * g) * sb, sb, hipMemcpyDeviceToDevice, p->stream) != hipSuccess ||
                hipMemcpyAsync(p->dC, ck + (size_t)(2 * g + 1) * sb, sb, hipMemcpyDeviceToDevice, p->stream) !=
                    hipSuccess)
                return KZK_ERR_DEVICE;
            // recompute the segment, storing u^n and u*
            if ((st = stored_steps(s0, s1)) != KZK_OK) return st;
        }
        // adjoint steps back through the segment
        for (int s = s1 - 1; s >= s0; --s) {
            if (p->any_D_sched && (st = build_tables(p, s, true)) != KZK_OK) return st;
            if (y_adj(p, 1, p->dL, p->dP, p->dB, nullptr) != hipSuccess) return KZK_ERR_DEVICE;
            if (tau_adj(p, 1, p->dB, nullptr, Us + (size_t)(s - s0) * ub, p->dM, s + 1) != hipSuccess)
                return KZK_ERR_DEVICE;
            if (y_adj(p, 2, p->dM, p->dP, p->dB, p->dR) != hipSuccess) return KZK_ERR_DEVICE;
            if (tau_adj(p, 2, p->dB, p->dR, Un + (size_t)(s - s0) * ub, p->dL, s) != hipSuccess)
                return KZK_ERR_DEVICE;
        }
    }
    if (tau(p, 1, nullptr, grad, p->dL, nullptr, 0) != hipSuccess) return KZK_ERR_DEVICE;
    return KZK_OK;
}


// ------------------------------------------------------------------ march without allocation
// Device memory of kzk_step_noalloc: one array per GPU (each device holds its
// own copy from the library's load on that device until the process ends).
// Host code never passes the array's name to a kernel or a copy: it takes the
// device address from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[KZK_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the scratch array on the current device.
kzk_status scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        (void)hipGetLastError();
        return KZK_ERR_DEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return KZK_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return KZK_OK;
}

}  // namespace

extern "C" kzk_status kzk_step_noalloc(const kzk_params* params, int32_t n_inst, void* hip_stream, void* u_dev,
                                       int32_t first_step, int32_t n_steps) {
    if (!params || !u_dev || n_inst < 1) return KZK_ERR_ARG;
    void* base = nullptr;
    kzk_status st = scratch_address(&base);
    if (st != KZK_OK) return st;
    kzk_plan* p = nullptr;
    st = create_plan(params, n_inst, hip_stream, static_cast<char*>(base), KZK_NOALLOC_SCRATCH_BYTES, &p);
    if (st != KZK_OK) return st;
    st = kzk_step(p, u_dev, first_step, n_steps);
    const kzk_status ps = kzk_poll(p);   // synchronises: the scratch is free again on return
    kzk_destroy(p);
    return st != KZK_OK ? st : ps;
}
