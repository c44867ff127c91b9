// Host side of the C ABI: plan construction (geometry, tables, prior, Jacobi
// diagonal, scratch), per-batch work schedules, and the PCG driver that
// enqueues the HIP kernels.  No arithmetic of the solve runs here: every step
// of an apply or a solve is a kernel launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "wmcao.h"
#include "wmcao_internal.hpp"

using namespace wm;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define WM_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(WMCAO_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

// Device allocation owned by a plan or a schedule.
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

struct Sched {
    // Item lists per stage, on the device (shared by the frame-prefix views
    // of the allocation-free solve).
    std::shared_ptr<DevBuf> buf;
    int frames = 0;                     // frames of a single-plan schedule
    const Item* coarse = nullptr;       // every layer (analysis)
    int n_coarse = 0;
    const Item* coarse_syn = nullptr;   // layers whose synthesis tiles do not rebuild LL_k0
    int n_coarse_syn = 0;
    // dynamic LDS sizes, [0] for FP32 and [1] for FP64 arithmetic (LDS tiles
    // follow the arithmetic type)
    int lds_idwt_lvl[2][WM_MAXLEV + 1] = {};   // the level-k synthesis tiles
    const Item* tiled[WM_MAXLEV + 1] = {};
    int n_tiled[WM_MAXLEV + 1] = {};
    const Item* sensor = nullptr;
    int n_sensor = 0;
    const Item* proj = nullptr;
    int n_proj = 0;
    const Item* wgt = nullptr;          // noise-weighting items (bands of wgt_rows node rows)
    int n_wgt = 0;
    const Item* proj_ap = nullptr;      // projection items of an operator apply (banded plans)
    int n_proj_ap = 0;
    const Item* papply = nullptr;       // one item per small sensor: projection and weighting
    int n_papply = 0;
    const Item* adj = nullptr;
    int n_adj = 0;
    int lds_adj[2] = {};
    int adj_taps = 2;      // fast-path taps of the adjoint (largest over the plans)
    const Item* vec = nullptr;
    int n_vec = 0;
    int maxk0 = 0;
    int lds_idwt[2] = {};  // the whole-band synthesis
    int lds_fdwt[2] = {};  // the whole-band analysis
    int lds_sensor = 0;
    int lds_weights = 0;   // dynamic LDS of k_weights
    int lds_project = 0;   // dynamic LDS of k_project
    int max_layers = 0;    // most layers of a plan of the schedule
    int tile = 32;
    // algorithmic bytes one launch of each stage moves (all frames of the job)
    double b_idwt_coarse = 0, b_idwt_tile[WM_MAXLEV + 1] = {};
    double b_fdwt_tile[2][WM_MAXLEV + 1] = {}, b_fdwt_coarse[2] = {};   // [plain, apply]
    double b_sensor[3] = {};                                              // [apply, rhs, fwd]
    double b_project = 0, b_adjoint = 0;
    double b_init = 0, b_update_r = 0, b_update_p = 0, b_replace = 0;
};

// Per-plan kernel timing with HIP events on the launch stream.
struct Profiler {
    bool on = false;
    std::vector<std::tuple<int, hipEvent_t, hipEvent_t, double>> rec;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    void clear() {
        for (auto& r : rec) {
            pool.push_back(std::get<1>(r));
            pool.push_back(std::get<2>(r));
        }
        rec.clear();
    }
    ~Profiler() {
        clear();
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

thread_local Profiler* g_prof = nullptr;

// Launch through f, bracketed by events when a profiler is active.
template <class F>
void timed(int kind, double bytes, hipStream_t s, F&& f) {
    if (!g_prof || !g_prof->on) {
        f();
        return;
    }
    hipEvent_t a = g_prof->get(), b = g_prof->get();
    (void)hipEventRecord(a, s);
    f();
    (void)hipEventRecord(b, s);
    g_prof->rec.emplace_back(kind, a, b, bytes);
}

struct ProfScope {
    Profiler* prev;
    explicit ProfScope(Profiler* p) : prev(g_prof) { g_prof = p; }
    ~ProfScope() { g_prof = prev; }
};

}  // namespace

struct wmcao_plan_s {
    int device = 0;
    wmcao_dtype dtype = WMCAO_F64;
    size_t esz = 8;       // bytes of a PCG vector element (T)
    int op64 = 1;         // operator type F: 1 double, 0 float
    size_t osz = 8;       // bytes of an operator element (F)
    int L = 0, W = 0, levels = 0;
    int max_batch = 1;
    int tile = 32;
    int lds_budget = 64 * 1024;
    int resid_replace = 0;
    PlanDev host{};
    PlanDev* dev = nullptr;
    std::vector<std::unique_ptr<DevBuf>> allocs;
    void* vb = nullptr;
    void* vr = nullptr;
    void* vp = nullptr;
    void* vq = nullptr;
    void* vphi = nullptr;
    void* vll = nullptr;
    void* vnode = nullptr;
    void* vfp = nullptr;
    double* vu = nullptr;
    double* vspart = nullptr;
    double* part = nullptr;
    double* scal = nullptr;
    int* status = nullptr;
    double* jac_d = nullptr;
    int64_t n = 0, n_slopes = 0, n_nodes = 0, ll_size = 0;
    int64_t n_fp = 0;   // layer pixels some sensor node's bilinear stencil touches
    int64_t n_fpimg = 0;  // values of the adjoint footprint images of one frame
    int64_t n_spart = 0;  // doubles of the per-band slope sums of one frame
    int lds_adjoint[2] = {};  // staged rows + row-pass buffer of the adjoint, FP32 / FP64 arithmetic
    int c64 = 7;              // stages computing in FP64 (C_IDWT | C_ADJ | C_FDWT)
    int adj_lds = ADJ_LDS;    // LDS budget of one adjoint work item
    int adj_taps = 2;     // most nodes feeding one footprint row or column (2 to 4)
    std::vector<int64_t> layer_off, slope_off;
    std::map<std::pair<int, int>, std::unique_ptr<Sched>> sched;   // by (first frame, frames)
    Sched* full_sched = nullptr;     // max_batch frames, built with the plan
    int streams = 2;                 // concurrent parts a large solve may run as (1..4)
    hipStream_t side[3] = {};        // streams of parts 2..4
    hipEvent_t ev_fork = nullptr, ev_join[3] = {};
    // captured graph of one wmcao_solve_graph argument set, and the event
    // recorded after its latest replay
    hipGraphExec_t gexec = nullptr;
    hipEvent_t gdone = nullptr;
    std::tuple<const void*, void*, int, int, int, double*, int*, void*> gkey{};
    std::mutex mu;
    Profiler prof;

    void* alloc(size_t bytes, int* rc) {
        auto b = std::make_unique<DevBuf>();
        if (bytes == 0) bytes = 16;
        hipError_t e = hipMalloc(&b->p, bytes);
        if (e != hipSuccess) {
            *rc = fail(WMCAO_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
            return nullptr;
        }
        void* p = b->p;
        allocs.push_back(std::move(b));
        return p;
    }
};

namespace {

// ------------------------------------------------------------ db3 filter ----
// Daubechies' 6-tap orthonormal scaling filter (closed form of Daubechies
// 1988 for three vanishing moments) and its quadrature mirror.
void db3_filters(double* h, double* g) {
    const double s10 = std::sqrt(10.0);
    const double q = std::sqrt(5.0 + 2.0 * s10);
    const double c = 1.0 / (16.0 * std::sqrt(2.0));
    h[0] = (1.0 + s10 + q) * c;
    h[1] = (5.0 + s10 + 3.0 * q) * c;
    h[2] = (10.0 - 2.0 * s10 + 2.0 * q) * c;
    h[3] = (10.0 - 2.0 * s10 - 2.0 * q) * c;
    h[4] = (5.0 + s10 - 3.0 * q) * c;
    h[5] = (1.0 + s10 - q) * c;
    for (int n = 0; n < 6; ++n) g[n] = ((n & 1) ? -1.0 : 1.0) * h[5 - n];
}

// 1-D periodic synthesis of a length-M vector from its low half a and high
// half d: x[(2k+n) mod M] += h_n a_k + g_n d_k.
void synth1(const double* h, const double* g, const std::vector<double>& in, int M,
            std::vector<double>& out) {
    std::fill(out.begin(), out.begin() + M, 0.0);
    const int H = M / 2;
    for (int k = 0; k < H; ++k)
        for (int n = 0; n < 6; ++n) out[(2 * k + n) % M] += h[n] * in[k] + g[n] * in[H + k];
}

// Prototype basis vector of an N-periodic k-level 1-D transform: the
// synthesis of a unit coefficient at position 0 of the level-k low band
// (type 0) or detail band (type 1).
std::vector<double> prototype(const double* h, const double* g, int N, int k, int type) {
    std::vector<double> x(N, 0.0), tmp(N, 0.0);
    x[type ? (N >> k) : 0] = 1.0;
    for (int lev = k; lev >= 1; --lev) {
        const int M = N >> (lev - 1);
        synth1(h, g, x, M, tmp);
        std::copy(tmp.begin(), tmp.begin() + M, x.begin());
    }
    return x;
}

int upload(wmcao_plan_s* p, const void* host, size_t bytes, void** out) {
    int rc = WMCAO_OK;
    void* d = p->alloc(bytes, &rc);
    if (!d) return rc;
    if (bytes) WM_HIP(hipMemcpy(d, host, bytes, hipMemcpyHostToDevice));
    *out = d;
    return WMCAO_OK;
}

template <class V>
int upload_vec(wmcao_plan_s* p, const std::vector<V>& v, const V** out) {
    void* d = nullptr;
    int rc = upload(p, v.data(), v.size() * sizeof(V), &d);
    *out = static_cast<const V*>(d);
    return rc;
}

// ------------------------------------------------------------- schedules ----
struct JobSpec {
    wmcao_plan_s* plan;
    int count;
    int first = 0;   // frames first .. first + count - 1 of the plan's batch
};

int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Items for every stage of a job of several plans: frame-major order inside
// each plan, plans in order.  The FDWT pass of one frame writes one <p, Ap>
// partial per tile, layer by layer; each layer's whole-band block adds its
// layer's tile partials to its own and writes the layer total after them
// (the consumer sums L totals); the vector passes use one slot per chunk.
int build_sched(const std::vector<JobSpec>& jobs, int tile, Sched* S) {
    std::vector<Item> coarse, coarse_syn, sensor, vec, proj, adj, wgt, proj_ap, papply;
    int lds_lvl[2][WM_MAXLEV + 1] = {};
    std::vector<Item> tiled[WM_MAXLEV + 1];
    int maxk0 = 0, lds_i[2] = {}, lds_f[2] = {}, lds_s = 0, lds_a[2] = {}, lds_w = 0, lds_p = 0, taps_a = 2;
    for (int jp = 0; jp < static_cast<int>(jobs.size()); ++jp) {
        const wmcao_plan_s* P = jobs[jp].plan;
        // a plan whose sensors are all small projects and weights them in one
        // block per sensor (k_sensor); the others in bands (k_project, k_weights)
        bool fused = true;
        for (int m = 0; m < P->W; ++m) fused = fused && P->host.wfs[m].nn <= SENSOR_FUSE_NN;
        for (int f = jobs[jp].first; f < jobs[jp].first + jobs[jp].count; ++f) {
            // <p, Ap> partials: one per analysis tile, numbered layer by layer,
            // then one total per layer (written by the layer's whole-band block)
            int slot = 0, first[WM_MAXL], cnt[WM_MAXL];
            for (int l = 0; l < P->L; ++l) {
                const LayerInfo& Ly = P->host.layer[l];
                first[l] = slot;
                for (int k = 1; k <= Ly.k0; ++k) {
                    const int M = Ly.N >> (k - 1);
                    const int nt = ceil_div(M, tile);
                    for (int t = 0; t < nt * nt; ++t) tiled[k].push_back(Item{jp, f, l, t, slot++, 0, 0, 0});
                    maxk0 = std::max(maxk0, k);
                }
                cnt[l] = slot - first[l];
            }
            const int tile_slots = slot;
            for (int l = 0; l < P->L; ++l) {
                coarse.push_back(Item{jp, f, l, 0, tile_slots + l, first[l], cnt[l], 0});
                const LayerInfo& Ly = P->host.layer[l];
                if (!Ly.fuse) coarse_syn.push_back(coarse.back());
                const int N = Ly.N, M0 = N >> Ly.k0;
                for (int c = 0; c < 2; ++c) {
                    const int esz_c = c ? 8 : 4;
                    if (Ly.fuse) lds_lvl[c][Ly.k0] = std::max(lds_lvl[c][Ly.k0], M0 * M0 * esz_c);
                    lds_i[c] = std::max(lds_i[c], M0 * M0 * esz_c);
                    lds_f[c] = std::max(lds_f[c], M0 * M0 * esz_c);
                }
            }
            for (int m = 0; m < P->W; ++m)
                for (int l = 0; l < P->L; ++l) {
                    const int br = P->host.fp_br[m][l];
                    const int nb = br > 0 ? ceil_div(P->host.fp_h[m][l], br) : 0;
                    for (int b = 0; b < nb; ++b) adj.push_back(Item{jp, f, m, l, b, 0, 0, 0});
                }
            for (int c = 0; c < 2; ++c) lds_a[c] = std::max(lds_a[c], P->lds_adjoint[c]);
            taps_a = std::max(taps_a, P->adj_taps);
            for (int m = 0; m < P->W; ++m) {
                sensor.push_back(Item{jp, f, m, 0, 0, 0, 0, 0});
                const int nb = ceil_div(P->host.wfs[m].nn, P->host.proj_rows);
                for (int b = 0; b < nb; ++b) proj.push_back(Item{jp, f, m, b, 0, 0, 0, 0});
                if (fused) {
                    papply.push_back(Item{jp, f, m, 0, 0, 0, 0, 0});
                } else {
                    for (int b = 0; b < nb; ++b) proj_ap.push_back(Item{jp, f, m, b, 0, 0, 0, 0});
                    const int nbw = ceil_div(P->host.wfs[m].nn, P->host.wgt_rows);
                    for (int b = 0; b < nbw; ++b) wgt.push_back(Item{jp, f, m, b, 0, 0, 0, 0});
                }
                const int nn = P->host.wfs[m].nn;
                lds_s = std::max(lds_s, static_cast<int>(nn * nn * sizeof(double)));
                lds_w = std::max(lds_w, weights_lds_bytes(nn, P->host.wfs[m].n_sub, P->host.wgt_rows));
                lds_p = std::max(lds_p, proj_lds_bytes(P->L, nn, P->host.proj_rows));
            }
            const int nch = static_cast<int>((P->n + P->host.vec_chunk - 1) / P->host.vec_chunk);
            for (int c = 0; c < nch; ++c) vec.push_back(Item{jp, f, 0, c, c, 0, 0, 0});
        }
        // bytes each launch reads and writes as designed (see the kernel table
        // in the design notes): e per PCG vector element, o per operator element
        const double e = static_cast<double>(P->esz) * jobs[jp].count;
        const double o = static_cast<double>(P->osz) * jobs[jp].count;
        const double Q = static_cast<double>(P->n_nodes), n = static_cast<double>(P->n);
        bool gathers_tile = false, gathers_coarse = false;
        // low-pass scratch bands in each stage's arithmetic type
        const double c8i = ((P->c64 & 1) ? 8.0 : 4.0) * jobs[jp].count;
        const double c8f = ((P->c64 & 4) ? 8.0 : 4.0) * jobs[jp].count;
        for (int l = 0; l < P->L; ++l) {
            const LayerInfo& Ly = P->host.layer[l];
            const double M0 = Ly.N >> Ly.k0, B0 = M0 * M0;
            if (Ly.fuse)   // the level-k0 tiles read the coarse block instead of LL_k0
                S->b_idwt_tile[Ly.k0] += B0 * e - B0 * c8i;
            else
                S->b_idwt_coarse += B0 * e + B0 * (Ly.k0 ? c8i : o);
            for (int a = 0; a < 2; ++a) S->b_fdwt_coarse[a] += (Ly.k0 ? B0 * c8f : 0) + B0 * e + (a ? B0 * e : 0);
            gathers_coarse = gathers_coarse || Ly.k0 == 0;
            for (int k = 1; k <= Ly.k0; ++k) {
                const double M = Ly.N >> (k - 1), Hq = (M / 2) * (M / 2);
                S->b_idwt_tile[k] += Hq * c8i + 3 * Hq * e + M * M * (k > 1 ? c8i : o);
                for (int a = 0; a < 2; ++a)
                    S->b_fdwt_tile[a][k] += (k > 1 ? M * M * c8f : 0) + Hq * c8f + 3 * Hq * e + (a ? 3 * Hq * e : 0);
                gathers_tile = gathers_tile || k == 1;
            }
        }
        const double F = static_cast<double>(P->n_fpimg);
        for (int a = 0; a < 2; ++a) {
            if (gathers_tile) S->b_fdwt_tile[a][1] += F * o;
            if (gathers_coarse) S->b_fdwt_coarse[a] += F * o;
        }
        S->b_adjoint += (Q + F) * o;
        const double u8 = 8.0 * jobs[jp].count;     // node fields of the projection are FP64
        S->b_project += P->n_fp * o + Q * u8;
        S->b_sensor[0] += Q * u8 + Q * o;
        S->b_sensor[1] += P->n_slopes * e + Q * o;
        S->b_sensor[2] += Q * u8 + P->n_slopes * e;
        S->b_init += 5 * n * e;
        S->b_update_r += 4 * n * e;
        S->b_update_p += 6 * n * e;
        S->b_replace += 4 * n * e;
    }
    std::vector<Item> all;
    std::vector<size_t> offs;
    auto add = [&](const std::vector<Item>& v) {
        offs.push_back(all.size());
        all.insert(all.end(), v.begin(), v.end());
    };
    add(coarse);
    add(coarse_syn);
    add(sensor);
    add(vec);
    add(proj);
    add(adj);
    for (int k = 1; k <= WM_MAXLEV; ++k) add(tiled[k]);
    add(wgt);
    add(proj_ap);
    add(papply);
    S->buf = std::make_shared<DevBuf>();
    const size_t bytes = std::max<size_t>(all.size(), 1) * sizeof(Item);
    hipError_t e = hipMalloc(&S->buf->p, bytes);
    if (e != hipSuccess) return fail(WMCAO_ERR_OOM, "schedule allocation failed");
    WM_HIP(hipMemcpy(S->buf->p, all.data(), all.size() * sizeof(Item), hipMemcpyHostToDevice));
    const Item* base = static_cast<const Item*>(S->buf->p);
    S->coarse = base + offs[0];
    S->n_coarse = static_cast<int>(coarse.size());
    S->coarse_syn = base + offs[1];
    S->n_coarse_syn = static_cast<int>(coarse_syn.size());
    S->sensor = base + offs[2];
    S->n_sensor = static_cast<int>(sensor.size());
    S->vec = base + offs[3];
    S->n_vec = static_cast<int>(vec.size());
    S->proj = base + offs[4];
    S->n_proj = static_cast<int>(proj.size());
    S->adj = base + offs[5];
    S->n_adj = static_cast<int>(adj.size());
    S->wgt = base + offs[6 + WM_MAXLEV];
    S->n_wgt = static_cast<int>(wgt.size());
    S->proj_ap = base + offs[7 + WM_MAXLEV];
    S->n_proj_ap = static_cast<int>(proj_ap.size());
    S->papply = base + offs[8 + WM_MAXLEV];
    S->n_papply = static_cast<int>(papply.size());
    for (int c = 0; c < 2; ++c) S->lds_adj[c] = lds_a[c];
    S->adj_taps = taps_a;
    for (int c = 0; c < 2; ++c)
        for (int k = 0; k <= WM_MAXLEV; ++k) S->lds_idwt_lvl[c][k] = lds_lvl[c][k];
    for (int k = 1; k <= WM_MAXLEV; ++k) {
        S->tiled[k] = base + offs[5 + k];
        S->n_tiled[k] = static_cast<int>(tiled[k].size());
    }
    S->maxk0 = maxk0;
    for (int c = 0; c < 2; ++c) {
        S->lds_idwt[c] = lds_i[c];
        S->lds_fdwt[c] = lds_f[c];
    }
    S->lds_sensor = lds_s;
    S->lds_weights = lds_w;
    S->lds_project = lds_p;
    for (const JobSpec& j : jobs) S->max_layers = std::max(S->max_layers, j.plan->L);
    S->tile = tile;
    return WMCAO_OK;
}

std::mutex g_multi_mu;
// packed schedules by job shape: (plan, frames, first frame) per job
std::map<std::vector<std::tuple<const void*, int, int>>, std::unique_ptr<Sched>> g_multi_cache;

// Captured multi-plan solves, keyed by every argument that the graph bakes in.
struct MultiGraphKey {
    std::vector<std::tuple<const void*, const void*, const void*, int>> args;   // plan, slopes, coeffs, count
    int n_iter = 0, warm = 0;
    void* stream = nullptr;
    bool operator<(const MultiGraphKey& o) const {
        return std::tie(args, n_iter, warm, stream) < std::tie(o.args, o.n_iter, o.warm, o.stream);
    }
};
constexpr size_t MULTI_GRAPH_CACHE = 64;
// A cached capture, the event recorded after its latest replay (so that it is
// destroyed only once that replay has finished) and its last use, for
// least-recently-used eviction.
struct CachedGraph {
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    uint64_t last_use = 0;
};
std::map<MultiGraphKey, CachedGraph> g_multi_graphs;
uint64_t g_graph_clock = 0;

void destroy_cached(CachedGraph& g) {
    if (g.done) {
        (void)hipEventSynchronize(g.done);
        (void)hipEventDestroy(g.done);
    }
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    g = CachedGraph{};
}

// Schedule of frames first .. first + batch - 1 of a plan (cached).
int get_sched(wmcao_plan_s* p, int batch, Sched** out, int first = 0) {
    const std::pair<int, int> key(first, batch);
    auto it = p->sched.find(key);
    if (it != p->sched.end()) {
        *out = it->second.get();
        return WMCAO_OK;
    }
    auto S = std::make_unique<Sched>();
    int rc = build_sched({JobSpec{p, batch, first}}, p->tile, S.get());
    if (rc) return rc;
    S->frames = batch;
    *out = S.get();
    p->sched[key] = std::move(S);
    return WMCAO_OK;
}

// A solve runs as up to `streams` concurrent parts of its frames when each
// part holds at least SPLIT_MIN_UNKNOWNS coefficients: the kernels of one part
// fill the gaps the others' leave (E-ELT frames, two parts: 7 % faster at 6
// frames, 9 % at 8 to 16, 8 % at 32, 5 % at 64; 4 frames, 0.75 M per half,
// gain nothing).  Smaller parts are launch-bound and can lose (128 frames of
// the 8 m system, 0.79 M per half: 18 % slower), so they stay on one stream.
constexpr int64_t SPLIT_MIN_UNKNOWNS = 1024 * 1024;

int parts_of(const wmcao_plan_s* p, int batch) {
    for (int k = std::min(p->streams, batch); k >= 2; --k)
        if (static_cast<int64_t>(batch / k) * p->n >= SPLIT_MIN_UNKNOWNS) return k;
    return 1;
}

// First frame of part i of k.
int part_first(int batch, int k, int i) { return static_cast<int>(static_cast<int64_t>(batch) * i / k); }

// The plan's streams for parts 2..k and their fork/join events, created on
// first use (outside any graph capture: callers prepare them before capturing).
int ensure_side(wmcao_plan_s* p, int k = 2) {
    if (!p->ev_fork) WM_HIP(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    for (int i = 0; i + 1 < k; ++i) {
        if (p->side[i]) continue;
        WM_HIP(hipStreamCreateWithFlags(&p->side[i], hipStreamNonBlocking));
        WM_HIP(hipEventCreateWithFlags(&p->ev_join[i], hipEventDisableTiming));
    }
    return WMCAO_OK;
}

// Everything a solve of this batch needs that allocates (schedules, streams).
int prepare_solve(wmcao_plan_s* p, int batch) {
    Sched* S = nullptr;
    const int k = parts_of(p, batch);
    if (k == 1) return get_sched(p, batch, &S);
    int rc = WMCAO_OK;
    for (int i = 0; i < k && !rc; ++i) {
        const int f0 = part_first(batch, k, i), f1 = part_first(batch, k, i + 1);
        rc = get_sched(p, f1 - f0, &S, f0);
    }
    if (!rc) rc = ensure_side(p, k);
    return rc;
}

JobPlan make_jobplan(wmcao_plan_s* p, int nframes) {
    JobPlan J{};
    J.P = p->dev;
    J.vec[V_B] = p->vb;
    J.vec[V_R] = p->vr;
    J.vec[V_P] = p->vp;
    J.vec[V_Q] = p->vq;
    J.vec[V_PHI] = p->vphi;
    J.vec[V_LL] = p->vll;
    J.vec[V_NODE] = p->vnode;
    J.vec[V_U] = p->vu;
    J.vec[V_FP] = p->vfp;
    J.vec[V_SPART] = p->vspart;
    J.stride[V_SPART] = p->n_spart;
    J.stride[V_U] = p->n_nodes;
    J.stride[V_FP] = p->n_fpimg;
    for (int v : {V_X, V_B, V_R, V_P, V_Q, V_PHI}) J.stride[v] = p->n;
    J.stride[V_LL] = p->ll_size;
    J.stride[V_NODE] = p->n_nodes;
    J.stride[V_SLOPES] = p->n_slopes;
    J.part = p->part;
    J.alpha = p->scal;
    J.status = p->status;
    J.resid = nullptr;
    J.resid_ld = 0;
    J.nframes = nframes;
    return J;
}

// ------------------------------------------------------- stage drivers ----
// T: PCG vector type of the plans of the job; S: their operator storage type;
// c64: stages computing in FP64 (C_IDWT, C_ADJ, C_FDWT bits; all of them when
// S is double).
enum : int { C_IDWT = 1, C_ADJ = 2, C_FDWT = 4 };
// Stages of an FP32-storage operator that compute in FP64 unless the plan
// says otherwise: the forward transform, whose detail coefficients are small
// differences of the summed P^T image (single-precision arithmetic there moved
// E-ELT iterates by 2.5e-5; FP64 there alone by 3.8e-6, measured), while
// W^-1 and P^T run in FP32.
constexpr int DEFAULT_FP64_STAGES = C_FDWT;

// Calls f.template operator()<C>() with C = double if the stage bit is set in
// c64 (or S is double), else float.
template <class S, class Fn>
void with_compute(int c64, int bit, Fn&& f) {
    if (std::is_same<S, double>::value || (c64 & bit))
        f.template operator()<double>();
    else
        f.template operator()<float>();
}

template <class T, class S>
void run_idwt(const JobArgs& a, const Sched& Sc, int in_vec, int out_vec, int c64, hipStream_t s) {
    with_compute<S>(c64, C_IDWT, [&]<class C>() {
        if (Sc.n_coarse_syn > 0)
            timed(WMCAO_K_IDWT_COARSE, Sc.b_idwt_coarse, s, [&] {
                launch_idwt_coarse<T, S, C>(a, Sc.coarse_syn, Sc.n_coarse_syn, in_vec, out_vec,
                                            Sc.lds_idwt[sizeof(C) == 8], s);
            });
        for (int k = Sc.maxk0; k >= 1; --k)
            timed(WMCAO_K_IDWT_TILE, Sc.b_idwt_tile[k], s, [&] {
                launch_idwt_tile<T, S, C>(a, Sc.tiled[k], Sc.n_tiled[k], k, in_vec, out_vec, Sc.tile,
                                          Sc.lds_idwt_lvl[sizeof(C) == 8][k], s);
            });
    });
}

template <class T, class S>
void run_fdwt(const JobArgs& a, const Sched& Sc, int src, int in_vec, int out_vec, int epi,
              int aux_vec, int c64, hipStream_t s) {
    with_compute<S>(c64, C_FDWT, [&]<class C>() {
        for (int k = 1; k <= Sc.maxk0; ++k)
            timed(WMCAO_K_FDWT_TILE, Sc.b_fdwt_tile[epi == EPI_APPLY][k], s, [&] {
                launch_fdwt_tile<T, S, C>(a, Sc.tiled[k], Sc.n_tiled[k], k, src, in_vec, out_vec, epi,
                                          aux_vec, Sc.tile, s);
            });
        timed(WMCAO_K_FDWT_COARSE, Sc.b_fdwt_coarse[epi == EPI_APPLY], s, [&] {
            launch_fdwt_coarse<T, S, C>(a, Sc.coarse, Sc.n_coarse, src, in_vec, out_vec, epi, aux_vec,
                                        Sc.lds_fdwt[sizeof(C) == 8], s);
        });
    });
}

template <class T, class S>
void run_adjoint(const JobArgs& a, const Sched& Sc, int c64, hipStream_t s) {
    with_compute<S>(c64, C_ADJ, [&]<class C>() {
        timed(WMCAO_K_ADJOINT, Sc.b_adjoint, s, [&] {
            launch_adjoint<T, S, C>(a, Sc.adj, Sc.n_adj, V_NODE, V_FP, Sc.lds_adj[sizeof(C) == 8],
                                    Sc.adj_taps, s);
        });
    });
}

// y = A x for every frame of the job (x_vec, y_vec are vector kinds).
template <class T, class S>
void run_apply(const JobArgs& a, const Sched& Sc, int x_vec, int y_vec, int c64, hipStream_t s) {
    run_idwt<T, S>(a, Sc, x_vec, V_PHI, c64, s);
    if (Sc.n_proj_ap > 0) {
        timed(WMCAO_K_PROJECT, Sc.b_project, s, [&] {
            launch_project<T, S>(a, Sc.proj_ap, Sc.n_proj_ap, V_PHI, 1, Sc.lds_project, Sc.max_layers, s);
        });
        timed(WMCAO_K_WEIGHTS, Sc.b_sensor[0], s,
              [&] { launch_weights<T, S>(a, Sc.wgt, Sc.n_wgt, V_NODE, Sc.lds_weights, s); });
    }
    if (Sc.n_papply > 0)
        timed(WMCAO_K_SENSOR, Sc.b_sensor[0], s, [&] {
            launch_sensor<T, S>(a, Sc.papply, Sc.n_papply, SM_PAPPLY, V_PHI, V_NODE, Sc.lds_sensor, s);
        });
    run_adjoint<T, S>(a, Sc, c64, s);
    run_fdwt<T, S>(a, Sc, SRC_PT, V_FP, y_vec, EPI_APPLY, x_vec, c64, s);
}

template <class T, class S>
void run_rhs(const JobArgs& a, const Sched& Sc, int slopes_vec, int b_vec, int c64, hipStream_t s) {
    timed(WMCAO_K_SENSOR, Sc.b_sensor[1], s, [&] {
        launch_sensor<T, S>(a, Sc.sensor, Sc.n_sensor, SM_RHS, slopes_vec, V_NODE, Sc.lds_sensor, s);
    });
    run_adjoint<T, S>(a, Sc, c64, s);
    run_fdwt<T, S>(a, Sc, SRC_PT, V_FP, b_vec, EPI_NONE, b_vec, c64, s);
}

template <class T, class S>
void run_solve(const JobArgs& a, const Sched& Sc, int n_iter, int warm, int resid_replace, int c64,
               hipStream_t s) {
    run_rhs<T, S>(a, Sc, V_SLOPES, V_B, c64, s);
    if (warm) run_apply<T, S>(a, Sc, V_X, V_Q, c64, s);
    timed(WMCAO_K_INIT, Sc.b_init, s, [&] { launch_init<T>(a, Sc.vec, Sc.n_vec, warm, s); });
    for (int it = 0; it < n_iter; ++it) {
        // rho of this iteration comes from the residual's partials on the
        // first iteration and after a replacement, else from k_update_p
        const bool replaced = resid_replace > 0 && it > 0 && it % resid_replace == 0;
        if (replaced) {
            run_apply<T, S>(a, Sc, V_X, V_Q, c64, s);
            timed(WMCAO_K_REPLACE_R, Sc.b_replace, s, [&] { launch_replace_r<T>(a, Sc.vec, Sc.n_vec, it, s); });
        }
        run_apply<T, S>(a, Sc, V_P, V_Q, c64, s);
        const int fresh = it == 0 || replaced;
        timed(WMCAO_K_UPDATE_R, Sc.b_update_r, s,
              [&] { launch_update_r<T>(a, Sc.vec, Sc.n_vec, it, fresh, s); });
        timed(WMCAO_K_UPDATE_P, Sc.b_update_p, s, [&] { launch_update_p<T>(a, Sc.vec, Sc.n_vec, it, s); });
    }
}

// Calls f.template operator()<T, S>() with the vector and operator storage
// types of a plan: (double, double), (float, double) or (float, float).
template <class Fn>
void with_types(const wmcao_plan_s* p, Fn&& f) {
    if (p->dtype == WMCAO_F64)
        f.template operator()<double, double>();
    else if (p->op64)
        f.template operator()<float, double>();
    else
        f.template operator()<float, float>();
}

int check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(WMCAO_ERR_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return WMCAO_OK;
}

int check_batch(wmcao_plan_s* p, int batch) {
    if (!p) return fail(WMCAO_ERR_INVALID_ARG, "plan is NULL");
    if (batch < 1 || batch > p->max_batch)
        return fail(WMCAO_ERR_INVALID_ARG, "batch must be in 1..max_batch");
    return WMCAO_OK;
}

struct DevGuard {
    int prev = -1;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DevGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int enqueue_solve(wmcao_plan_s* p, const void* slopes, void* coeffs, int batch, int n_iter,
                  int warm, double* resid, int* status, hipStream_t s) {
    int rc = prepare_solve(p, batch);
    if (rc) return rc;
    JobArgs a{};
    a.njp = 1;
    a.jp[0] = make_jobplan(p, batch);
    a.jp[0].vec[V_X] = coeffs;
    a.jp[0].vec[V_SLOPES] = const_cast<void*>(slopes);
    if (status) a.jp[0].status = status;
    a.jp[0].resid = resid;
    a.jp[0].resid_ld = n_iter + 1;
    auto run = [&](const Sched& S, hipStream_t st) {
        with_types(p, [&]<class T, class Sv>() { run_solve<T, Sv>(a, S, n_iter, warm, p->resid_replace, p->c64, st); });
    };
    const int k = parts_of(p, batch);
    if (k == 1) {
        Sched* S = nullptr;
        rc = get_sched(p, batch, &S);
        if (rc) return rc;
        run(*S, s);
        return check_launch();
    }
    // k parts: parts 2..k fork onto the plan's streams after everything the
    // caller queued before, and the caller's stream waits for them to end
    Sched* Sp[4] = {};
    for (int i = 0; i < k && !rc; ++i) {
        const int f0 = part_first(batch, k, i), f1 = part_first(batch, k, i + 1);
        rc = get_sched(p, f1 - f0, &Sp[i], f0);
    }
    if (rc) return rc;
    WM_HIP(hipEventRecord(p->ev_fork, s));
    for (int i = 1; i < k; ++i) WM_HIP(hipStreamWaitEvent(p->side[i - 1], p->ev_fork, 0));
    run(*Sp[0], s);
    for (int i = 1; i < k; ++i) run(*Sp[i], p->side[i - 1]);
    for (int i = 1; i < k; ++i) {
        WM_HIP(hipEventRecord(p->ev_join[i - 1], p->side[i - 1]));
        WM_HIP(hipStreamWaitEvent(s, p->ev_join[i - 1], 0));
    }
    return check_launch();
}

// Multi-plan solve enqueue (caller holds g_multi_mu).  prepare_only: validate
// and build the schedule without launching (before a graph capture).
int enqueue_multi(const wmcao_plan_t* plans, const void* const* slopes, void* const* coeffs,
                  const int* counts, int n_plans, int n_iter, int warm_start, hipStream_t s,
                  bool prepare_only = false) {
    if (!plans || !slopes || !coeffs || !counts) return fail(WMCAO_ERR_INVALID_ARG, "NULL argument");
    if (n_plans < 1 || n_plans > WM_MAXJP) return fail(WMCAO_ERR_INVALID_ARG, "n_plans out of range");
    if (n_iter < 0) return fail(WMCAO_ERR_INVALID_ARG, "n_iter < 0");
    const wmcao_dtype dt = plans[0] ? plans[0]->dtype : WMCAO_F32;
    std::vector<JobSpec> jobs;
    for (int i = 0; i < n_plans; ++i) {
        int rc = check_batch(plans[i], counts[i]);
        if (rc) return rc;
        if (plans[i]->dtype != dt) return fail(WMCAO_ERR_INVALID_ARG, "plans must share the dtype");
        if (!slopes[i] || !coeffs[i]) return fail(WMCAO_ERR_INVALID_ARG, "NULL buffer");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return fail(WMCAO_ERR_INVALID_ARG, "a plan appears twice");
        jobs.push_back(JobSpec{plans[i], counts[i]});
    }
    // one schedule per distinct job shape, dropped when one of its plans is destroyed
    std::vector<std::unique_lock<std::mutex>> locks;
    for (auto& j : jobs) locks.emplace_back(j.plan->mu);
    DevGuard g(plans[0]->device);
    const int tile = plans[0]->tile;
    for (auto& j : jobs)
        if (j.plan->tile != tile) return fail(WMCAO_ERR_INVALID_ARG, "plans must share the tile size");
    auto packed = [&](const std::vector<JobSpec>& js, Sched** out) -> int {
        std::vector<std::tuple<const void*, int, int>> key;
        for (auto& j : js) key.emplace_back(j.plan, j.count, j.first);
        auto it = g_multi_cache.find(key);
        if (it != g_multi_cache.end()) {
            *out = it->second.get();
            return WMCAO_OK;
        }
        auto sp = std::make_unique<Sched>();
        int rc = build_sched(js, tile, sp.get());
        if (rc) return rc;
        *out = sp.get();
        g_multi_cache[key] = std::move(sp);
        return WMCAO_OK;
    };
    int rr = 0;
    for (int i = 0; i < n_plans; ++i) rr = std::max(rr, plans[i]->resid_replace);
    auto args_for = [&](const std::vector<JobSpec>& js, const std::vector<int>& ids) {
        JobArgs a{};
        a.njp = static_cast<int>(ids.size());
        for (int k = 0; k < a.njp; ++k) {
            const int i = ids[k];
            a.jp[k] = make_jobplan(plans[i], counts[i]);
            a.jp[k].vec[V_X] = coeffs[i];
            a.jp[k].vec[V_SLOPES] = const_cast<void*>(slopes[i]);
        }
        return a;
    };
    auto run = [&](const JobArgs& a, const Sched& Sx, const wmcao_plan_s* typ, hipStream_t st) {
        with_types(typ, [&]<class T, class Sv>() { run_solve<T, Sv>(a, Sx, n_iter, warm_start, rr, typ->c64, st); });
    };
    // Groups of one launch sequence each: plans of one operator type share
    // kernels, so plans of both types run as two groups, the second on the
    // first plan's side stream.  Within a single group, each plan's frames
    // split into two concurrent halves under the rule of a single-plan solve:
    // every plan allows two streams and a half holds at least
    // SPLIT_MIN_UNKNOWNS coefficients.
    std::vector<JobSpec> grp[2];
    std::vector<int> idx[2];
    // operator type of a plan: FP64 storage, or FP32 storage with its FP64 stages
    auto op_key = [](const wmcao_plan_s* q) { return q->op64 ? 8 : q->c64; };
    int keys[2] = {op_key(plans[0]), -1};
    for (int i = 0; i < n_plans; ++i) {
        const int k = op_key(plans[i]);
        if (k != keys[0] && keys[1] < 0) keys[1] = k;
        if (k != keys[0] && k != keys[1])
            return fail(WMCAO_ERR_INVALID_ARG, "packed plans may use at most two operator types");
    }
    const bool mixed_ops = keys[1] >= 0;
    if (mixed_ops) {
        for (int i = 0; i < n_plans; ++i) {
            const int g = op_key(plans[i]) == keys[0] ? 0 : 1;
            grp[g].push_back(JobSpec{plans[i], counts[i], 0});
            idx[g].push_back(i);
        }
    } else {
        int64_t total = 0;
        bool two = true;
        for (auto& j : jobs) {
            total += static_cast<int64_t>(j.count) * j.plan->n;
            two = two && j.plan->streams > 1;
        }
        std::vector<JobSpec> half[2];
        std::vector<int> hidx[2];
        for (int i = 0; i < n_plans; ++i) {
            const int c1 = counts[i] / 2, c0 = counts[i] - c1;
            half[0].push_back(JobSpec{plans[i], c0, 0});
            hidx[0].push_back(i);
            if (c1 > 0) {
                half[1].push_back(JobSpec{plans[i], c1, c0});
                hidx[1].push_back(i);
            }
        }
        const bool split = two && total / 2 >= SPLIT_MIN_UNKNOWNS && !half[1].empty();
        if (split) {
            for (int g = 0; g < 2; ++g) {
                grp[g] = half[g];
                idx[g] = hidx[g];
            }
        } else {
            grp[0] = jobs;
            for (int i = 0; i < n_plans; ++i) idx[0].push_back(i);
        }
    }
    const bool two_groups = !grp[1].empty();
    // a plan limited to one stream keeps both groups on the caller's stream
    bool side_ok = true;
    for (int i = 0; i < n_plans; ++i) side_ok = side_ok && plans[i]->streams > 1;
    Sched* S[2] = {nullptr, nullptr};
    int rc = packed(grp[0], &S[0]);
    if (!rc && two_groups) rc = packed(grp[1], &S[1]);
    if (!rc && two_groups && side_ok) rc = ensure_side(plans[0], 2);
    if (rc) return rc;
    if (prepare_only) return WMCAO_OK;
    if (!two_groups || !side_ok) {
        run(args_for(grp[0], idx[0]), *S[0], plans[idx[0][0]], s);
        if (two_groups) run(args_for(grp[1], idx[1]), *S[1], plans[idx[1][0]], s);
        return check_launch();
    }
    wmcao_plan_s* p0 = plans[0];
    WM_HIP(hipEventRecord(p0->ev_fork, s));
    WM_HIP(hipStreamWaitEvent(p0->side[0], p0->ev_fork, 0));
    run(args_for(grp[0], idx[0]), *S[0], plans[idx[0][0]], s);
    run(args_for(grp[1], idx[1]), *S[1], plans[idx[1][0]], p0->side[0]);
    WM_HIP(hipEventRecord(p0->ev_join[0], p0->side[0]));
    WM_HIP(hipStreamWaitEvent(s, p0->ev_join[0], 0));
    return check_launch();
}

// ------------------------------------------------ allocation-free solve ----
// Scratch of wmcao_solve_noalloc lives in `scratch`, a file-scope device array
// of NOALLOC_BYTES: every GPU the library runs on holds its own copy until the
// process ends.  Host code reaches it only through the device address that
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in, not a device address), looked up once per device.
std::mutex g_noalloc_mu;
constexpr int NOALLOC_DEVICES = 64;
void* g_noalloc_ptr[NOALLOC_DEVICES] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[wm::NOALLOC_BYTES];

namespace {

// Device address of `scratch` on device dev (which must be current).
int noalloc_base(int dev, char** out) {
    if (dev < 0 || dev >= NOALLOC_DEVICES) return fail(WMCAO_ERR_UNSUPPORTED, "device index too large");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(WMCAO_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_noalloc_ptr[dev] = ptr;
    }
    *out = static_cast<char*>(g_noalloc_ptr[dev]);
    return WMCAO_OK;
}

// Carves the per-frame scratch of a solve of `batch` frames out of base (or,
// with base NULL, only measures it): the PCG vectors b, r, p, A p, the
// operator scratch, the slope sums, the partial sums and the per-frame scalars
// and status.  Returns the bytes needed.
size_t carve_noalloc(const wmcao_plan_s* p, int batch, char* base, JobPlan* J) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* q = base ? base + off : nullptr;
        off += (bytes + 255) & ~size_t(255);
        return static_cast<void*>(q);
    };
    const size_t B = static_cast<size_t>(batch);
    void* vb = take(p->n * p->esz * B);
    void* vr = take(p->n * p->esz * B);
    void* vp = take(p->n * p->esz * B);
    void* vq = take(p->n * p->esz * B);
    void* vphi = take(p->n * p->osz * B);
    void* vll = take(p->ll_size * 8 * B);
    void* vnode = take(p->n_nodes * p->osz * B);
    void* vu = take(p->n_nodes * 8 * B);
    void* vfp = take(p->n_fpimg * p->osz * B);
    void* vsp = take(p->n_spart * 8 * B);
    void* part = take(sizeof(double) * NPT * p->host.slots * B);
    void* scal = take(sizeof(double) * 4 * B);
    void* status = take(sizeof(int) * B);
    if (J && base) {
        J->vec[V_B] = vb;
        J->vec[V_R] = vr;
        J->vec[V_P] = vp;
        J->vec[V_Q] = vq;
        J->vec[V_PHI] = vphi;
        J->vec[V_LL] = vll;
        J->vec[V_NODE] = vnode;
        J->vec[V_U] = vu;
        J->vec[V_FP] = vfp;
        J->vec[V_SPART] = vsp;
        J->part = static_cast<double*>(part);
        J->alpha = static_cast<double*>(scal);
        J->status = static_cast<int*>(status);
    }
    return off;
}

}  // namespace

// =================================================================== ABI ====
extern "C" {

const char* wmcao_strerror(int code) {
    switch (code) {
        case WMCAO_OK: return "ok";
        case WMCAO_ERR_INVALID_ARG: return "invalid argument";
        case WMCAO_ERR_SIZE: return "unsupported size (layer grid must be divisible by 2^levels)";
        case WMCAO_ERR_FOOTPRINT: return "a sensor node projects outside a layer grid";
        case WMCAO_ERR_UNSUPPORTED: return "unsupported wavelet or sensor size";
        case WMCAO_ERR_OOM: return "out of memory";
        case WMCAO_ERR_HIP: return "HIP runtime error";
        case WMCAO_ERR_BREAKDOWN: return "CG breakdown (p^T A p <= 0 or non-finite)";
        default: return "unknown error";
    }
}

const char* wmcao_last_error(void) { return g_last_error.c_str(); }

int wmcao_plan(const wmcao_pupil* pupil, const wmcao_layer* layers, int n_layers,
               const wmcao_wfs* wfs, int n_wfs, wmcao_wavelet wavelet, int levels,
               const wmcao_options* opts, wmcao_plan_t* out) {
    g_last_error.clear();
    if (!out) return fail(WMCAO_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!pupil || !layers || !wfs || !opts) return fail(WMCAO_ERR_INVALID_ARG, "NULL argument");
    if (n_layers < 1 || n_layers > WM_MAXL) return fail(WMCAO_ERR_INVALID_ARG, "n_layers out of range");
    if (n_wfs < 1 || n_wfs > WM_MAXW) return fail(WMCAO_ERR_INVALID_ARG, "n_wfs out of range");
    if (wavelet.family != 0 || wavelet.order != 3)
        return fail(WMCAO_ERR_UNSUPPORTED, "only Daubechies order 3 is built");
    if (levels < 0 || levels > WM_MAXLEV) return fail(WMCAO_ERR_SIZE, "levels out of range");
    if (opts->dtype != WMCAO_F32 && opts->dtype != WMCAO_F64)
        return fail(WMCAO_ERR_INVALID_ARG, "dtype");
    if (opts->max_batch < 1) return fail(WMCAO_ERR_INVALID_ARG, "max_batch < 1");
    if (!(opts->alpha > 0.0) || !(opts->r0_m > 0.0) || !(opts->L0_m > 0.0))
        return fail(WMCAO_ERR_INVALID_ARG, "alpha, r0 and L0 must be positive");
    if (opts->tile != 0 && opts->tile != 16 && opts->tile != 32 && opts->tile != 64)
        return fail(WMCAO_ERR_INVALID_ARG, "tile must be 0, 16, 32 or 64");
    if (opts->precond != 0 && opts->precond != 1) return fail(WMCAO_ERR_INVALID_ARG, "precond");
    if (opts->resid_replace_every < 0) return fail(WMCAO_ERR_INVALID_ARG, "resid_replace_every < 0");
    if (opts->streams < 0 || opts->streams > 4) return fail(WMCAO_ERR_INVALID_ARG, "streams must be 0..4");
    if (opts->op_precision != 0 && opts->op_precision != 32 && opts->op_precision != 64)
        return fail(WMCAO_ERR_INVALID_ARG, "op_precision must be 0, 32 or 64");
    if (opts->dtype == WMCAO_F64 && opts->op_precision == 32)
        return fail(WMCAO_ERR_INVALID_ARG, "FP64 plans have FP64 operators");
    if (opts->op_fp64_stages < -1 || opts->op_fp64_stages > 7)
        return fail(WMCAO_ERR_INVALID_ARG, "op_fp64_stages must be -1 or a mask of 1, 2 and 4");
    if (opts->proj_rows != 0 && (opts->proj_rows < PROJ_ROWS_MIN || opts->proj_rows > PROJ_ROWS_MAX))
        return fail(WMCAO_ERR_INVALID_ARG, "proj_rows must be 0 or " + std::to_string(PROJ_ROWS_MIN) +
                                               " .. " + std::to_string(PROJ_ROWS_MAX));
    if (opts->vec_chunk != 0 && opts->vec_chunk != 1024 && opts->vec_chunk != 2048 &&
        opts->vec_chunk != 4096 && opts->vec_chunk != 8192)
        return fail(WMCAO_ERR_INVALID_ARG, "vec_chunk must be 0, 1024, 2048, 4096 or 8192");
    if (opts->adj_lds != 0 && (opts->adj_lds < 8 * 1024 || opts->adj_lds > 96 * 1024))
        return fail(WMCAO_ERR_INVALID_ARG, "adj_lds must be 0 or 8 KiB .. 96 KiB");
    if (!(pupil->diameter_m > 0.0) || pupil->obstruction_ratio < 0.0 || pupil->obstruction_ratio >= 1.0)
        return fail(WMCAO_ERR_INVALID_ARG, "pupil");
    bool seen_ngs = false;
    for (int m = 0; m < n_wfs; ++m) {
        const wmcao_wfs& w = wfs[m];
        if (w.n_sub < 1 || w.n_sub > WM_NSUB_MAX) return fail(WMCAO_ERR_UNSUPPORTED, "n_sub out of range");
        if (w.tt_aggregate < 0 || w.tt_aggregate > 4 || (w.tt_aggregate && w.n_sub % w.tt_aggregate))
            return fail(WMCAO_ERR_INVALID_ARG, "tt_aggregate must be 0..4 and divide n_sub");
        if (w.kind != 0 && w.kind != 1) return fail(WMCAO_ERR_INVALID_ARG, "kind must be 0 or 1");
        if (w.kind == 1 && (w.tt_aggregate || w.is_lgs))
            return fail(WMCAO_ERR_INVALID_ARG, "phase sensors are natural-star and not aggregated");
        if (!w.cinv_blocks && !(w.sigma > 0.0)) return fail(WMCAO_ERR_INVALID_ARG, "sigma must be > 0");
        if (w.is_lgs) {
            if (seen_ngs) return fail(WMCAO_ERR_INVALID_ARG, "laser guide stars must come first");
            if (!(w.lgs_height_m > 0.0)) return fail(WMCAO_ERR_INVALID_ARG, "lgs_height_m");
        } else {
            seen_ngs = true;
        }
    }
    for (int l = 0; l < n_layers; ++l) {
        const int N = layers[l].n;
        if (levels > 0 && (N < 6 || N % (1 << levels) != 0 || (N >> (levels - 1)) < 6))
            return fail(WMCAO_ERR_SIZE, "layer size must be divisible by 2^levels and N/2^(levels-1) >= 6");
        if (N < 2) return fail(WMCAO_ERR_SIZE, "layer size must be at least 2");
        if (!(layers[l].spacing_m > 0.0) || !(layers[l].cn2_weight > 0.0))
            return fail(WMCAO_ERR_INVALID_ARG, "layer spacing and weight must be positive");
        for (int m = 0; m < n_wfs; ++m)
            if (wfs[m].is_lgs && layers[l].altitude_m >= wfs[m].lgs_height_m)
                return fail(WMCAO_ERR_INVALID_ARG, "layer above a laser guide star");
    }

    auto p = std::make_unique<wmcao_plan_s>();
    int rc = WMCAO_OK;
    if (hipGetDevice(&p->device) != hipSuccess) return fail(WMCAO_ERR_HIP, "no HIP device");
    static std::once_flag once;
    std::call_once(once, [] { configure_kernels(); });
    p->dtype = opts->dtype;
    p->esz = opts->dtype == WMCAO_F32 ? 4 : 8;
    {
        int64_t n_total = 0;
        for (int l = 0; l < n_layers; ++l) n_total += static_cast<int64_t>(layers[l].n) * layers[l].n;
        // default: FP64 operators below 2^17 unknowns (launch-bound solves whose
        // iterates are most sensitive to rounding), FP32 above
        const int op = opts->dtype == WMCAO_F64 ? 64
                       : opts->op_precision ? opts->op_precision
                       : (n_total < (int64_t(1) << 17) ? 64 : 32);
        p->op64 = op == 64 ? 1 : 0;
        p->osz = p->op64 ? 8 : 4;
        p->c64 = p->op64 ? (C_IDWT | C_ADJ | C_FDWT)
                 : opts->op_fp64_stages >= 0 ? opts->op_fp64_stages : DEFAULT_FP64_STAGES;
    }
    p->L = n_layers;
    p->W = n_wfs;
    p->levels = levels;
    p->max_batch = opts->max_batch;
    p->tile = opts->tile ? opts->tile : 32;
    // LDS of the whole-band wavelet block (FP64): 32 KB keeps it at <= 64 x 64
    p->lds_budget = opts->lds_budget > 0 ? opts->lds_budget : 8 * 1024;
    p->lds_budget = std::min(p->lds_budget, 128 * 1024);
    p->resid_replace = opts->resid_replace_every;
    p->streams = opts->streams ? opts->streams : 2;
    PlanDev& H = p->host;
    H.L = n_layers;
    H.W = n_wfs;
    H.levels = levels;
    H.dtype = opts->dtype;
    H.op64 = p->op64;
    H.proj_rows = opts->proj_rows ? opts->proj_rows : PROJ_ROWS;
    H.wgt_rows = std::min(H.proj_rows, WGT_ROWS_MAX);
    H.vec_chunk = opts->vec_chunk ? opts->vec_chunk : VEC_CHUNK;
    p->adj_lds = opts->adj_lds ? opts->adj_lds : ADJ_LDS;
    H.precond = opts->precond;
    H.alpha = opts->alpha;
    db3_filters(H.h, H.g);

    // ---- layers ---------------------------------------------------------
    int64_t off = 0, lloff = 0;
    // Levels 1..k0 run as tiled launches, the rest in one whole-band block.
    // A layer needs the fewest k0 whose block fits the LDS budget; all layers
    // take the largest of these, so that no tiled launch waits for a layer
    // whose tiles rebuild its coarse block while the others' are plain (a
    // batch-1 E-ELT solve 0.89 -> 0.83 ms with 128- and 256-pixel layers).
    auto min_k0 = [&](int N) {
        int k0 = 0;
        while (k0 < levels - 1) {
            const int64_t M0 = N >> k0;
            if (M0 * M0 * 8 <= p->lds_budget && M0 * M0 <= 1024 * WM_QMAX) break;
            ++k0;
        }
        return k0;
    };
    int k0_all = 0;
    for (int l = 0; l < n_layers; ++l) k0_all = std::max(k0_all, min_k0(layers[l].n));
    for (int l = 0; l < n_layers; ++l) {
        LayerInfo& Ly = H.layer[l];
        const int N = layers[l].n;
        Ly.N = N;
        Ly.coff = off;
        off += static_cast<int64_t>(N) * N;
        const int k0 = k0_all;
        const int64_t M0 = N >> k0;
        if (M0 * M0 * 8 > 128 * 1024 || M0 * M0 > 1024 * WM_QMAX)
            return fail(WMCAO_ERR_UNSUPPORTED, "layer too large for the wavelet kernels");
        Ly.k0 = k0;
        Ly.fuse = k0 >= 1 && M0 * M0 * 8 <= FUSE_LDS;
        for (int k = 1; k <= k0; ++k) {
            Ly.ll_off[k] = lloff;
            lloff += static_cast<int64_t>(N >> k) * (N >> k);
        }
        // prior (eq. (13)): D = d^2 (L0^-11/3 + nu_k^11/3) / c_rho, nu_k = 2^-k / d;
        // without a wavelet transform (levels = 0) the regulariser is the identity
        const double d = layers[l].spacing_m;
        const double c_rho = 0.023 * layers[l].cn2_weight * std::pow(opts->r0_m, -5.0 / 3.0);
        Ly.D[0] = 1.0;
        for (int k = 1; k <= levels; ++k) {
            const double nu = std::ldexp(1.0, -k) / d;
            Ly.D[k - 1] = d * d * (std::pow(opts->L0_m, -11.0 / 3.0) + std::pow(nu, 11.0 / 3.0)) / c_rho;
        }
    }
    // the projection addresses a frame's pixels with 32-bit byte offsets (FP64 at most)
    if (off * 8 >= (int64_t(1) << 31))
        return fail(WMCAO_ERR_UNSUPPORTED, "layers too large: a frame's pixels must stay under 2 GiB");
    p->n = off;
    p->ll_size = lloff;
    H.n = off;
    H.ll_size = lloff;
    p->layer_off.resize(n_layers + 1);
    for (int l = 0; l < n_layers; ++l) p->layer_off[l] = H.layer[l].coff;
    p->layer_off[n_layers] = off;

    // ---- sensors --------------------------------------------------------
    std::vector<int> ix0, jy0;
    std::vector<char> hitx, hity;                 // per (sensor, layer): pixels reached
    int pix_tab_off[WM_MAXW][WM_MAXL] = {};
    std::vector<double> txd, tyd, blocksd;
    int64_t soff = 0, noff = 0;
    p->slope_off.assign(1, 0);
    struct WfsHost { std::vector<int> act, cell_of, cell_count, maskmap; };
    std::vector<WfsHost> wh(n_wfs);
    const double Dp = pupil->diameter_m;
    for (int m = 0; m < n_wfs; ++m) {
        const wmcao_wfs& w = wfs[m];
        WfsInfo& I = H.wfs[m];
        const int ns = w.n_sub, nn = ns + 1;
        const double dsub = Dp / ns;
        I.n_sub = ns;
        I.nn = nn;
        I.agg = w.tt_aggregate;
        I.kind = w.kind;
        I.remove_tt = w.kind == 1 ? 0 : w.remove_tt < 0 ? (w.is_lgs ? 1 : 0) : (w.remove_tt ? 1 : 0);
        I.in_precond = w.in_precond < 0 ? ((ns > 2 && w.tt_aggregate == 0) ? 1 : 0) : (w.in_precond ? 1 : 0);
        // pupil: centre of subaperture (i, j) in the closed annulus
        const double ro2 = 0.25 * Dp * Dp, ri2 = 0.25 * Dp * Dp * pupil->obstruction_ratio * pupil->obstruction_ratio;
        WfsHost& X = wh[m];
        X.maskmap.assign(ns * ns, -1);
        for (int i = 0; i < ns; ++i)
            for (int j = 0; j < ns; ++j) {
                const double cx = (i + 0.5 - ns / 2.0) * dsub, cy = (j + 0.5 - ns / 2.0) * dsub;
                const double r2 = cx * cx + cy * cy;
                if (r2 <= ro2 && r2 >= ri2) X.act.push_back(i * ns + j);
            }
        I.S_fine = static_cast<int>(X.act.size());
        if (I.S_fine == 0) return fail(WMCAO_ERR_INVALID_ARG, "sensor without active subapertures");
        if (I.S_fine > 1024 * WM_QMAX || nn * nn > 1024 * WM_QMAX)
            return fail(WMCAO_ERR_UNSUPPORTED, "sensor too large");
        if (static_cast<int64_t>(nn) * nn * 8 > 150 * 1024)
            return fail(WMCAO_ERR_UNSUPPORTED, "sensor node field exceeds LDS");
        if (I.kind == 1) {
            // phase sensor: nodes that are corners of active subapertures
            std::vector<char> on(nn * nn, 0);
            for (int q = 0; q < I.S_fine; ++q) {
                const int i = X.act[q] / ns, j = X.act[q] % ns;
                on[i * nn + j] = on[(i + 1) * nn + j] = on[i * nn + j + 1] = on[(i + 1) * nn + j + 1] = 1;
            }
            X.act.clear();
            X.maskmap.assign(nn * nn, -1);
            for (int e = 0; e < nn * nn; ++e)
                if (on[e]) {
                    X.maskmap[e] = static_cast<int>(X.act.size());
                    X.act.push_back(e);
                }
            X.cell_of.assign(1, 0);
            X.cell_count.assign(1, 0);
            I.S = static_cast<int>(X.act.size());
            I.S_fine = I.S;
        } else if (I.agg) {
            const int k = I.agg, b = ns / k;
            std::vector<int> cell_id(k * k, -1);
            for (int q = 0; q < I.S_fine; ++q) {
                const int i = X.act[q] / ns, j = X.act[q] % ns;
                const int c = (i / b) * k + (j / b);
                cell_id[c] = 0;
            }
            int nc = 0;
            for (int c = 0; c < k * k; ++c)
                if (cell_id[c] == 0) cell_id[c] = nc++;
            X.cell_count.assign(nc, 0);
            X.cell_of.resize(I.S_fine);
            for (int q = 0; q < I.S_fine; ++q) {
                const int i = X.act[q] / ns, j = X.act[q] % ns;
                const int c = cell_id[(i / b) * k + (j / b)];
                X.cell_of[q] = c;
                X.cell_count[c]++;
                X.maskmap[X.act[q]] = c;
            }
            I.S = nc;
        } else {
            for (int q = 0; q < I.S_fine; ++q) X.maskmap[X.act[q]] = q;
            X.cell_of.assign(1, 0);
            X.cell_count.assign(1, 0);
            I.S = I.S_fine;
        }
        for (int q = 0; q < I.S; ++q) {
            if (w.cinv_blocks) {
                blocksd.push_back(w.cinv_blocks[3 * q]);
                blocksd.push_back(w.cinv_blocks[3 * q + 1]);
                blocksd.push_back(w.cinv_blocks[3 * q + 2]);
            } else {
                const double iv = 1.0 / (w.sigma * w.sigma);
                blocksd.push_back(iv);
                blocksd.push_back(0.0);
                blocksd.push_back(iv);
            }
        }
        I.soff = soff;
        I.boff = static_cast<int64_t>(blocksd.size() / 3) - I.S;
        for (int k = 0; k < 3; ++k) {
            I.bsum[k] = 0.0;
            for (int q = 0; q < I.S; ++q) I.bsum[k] += blocksd[3 * (I.boff + q) + k];
        }
        I.sp_off = static_cast<int>(p->n_spart);
        p->n_spart += static_cast<int64_t>(ceil_div(nn, H.proj_rows)) * SP_K;
        soff += (I.kind == 1 ? 1 : 2) * I.S;
        p->slope_off.push_back(soff);
        I.node_off = noff;
        noff += static_cast<int64_t>(nn) * nn;
        // projection tables per layer (Sec. 2.1): sample at s * r + theta * h
        for (int l = 0; l < n_layers; ++l) {
            const double hl = layers[l].altitude_m;
            const double s = w.is_lgs ? 1.0 - hl / w.lgs_height_m : 1.0;
            const int N = layers[l].n;
            const double d = layers[l].spacing_m;
            // node i at x_i = (i - n_sub/2) d_sub, seen at s x_i + theta h; in
            // grid units u = x / d + N/2 = pa i + pb
            const double pa = s * dsub / d;
            H.pa[m][l] = pa;
            H.pia[m][l] = 1.0 / pa;
            H.node_tab_off[m][l] = static_cast<int>(ix0.size());
            pix_tab_off[m][l] = static_cast<int>(hitx.size());
            for (int axis = 0; axis < 2; ++axis) {
                const double theta = axis == 0 ? w.theta_x : w.theta_y;
                const double pb = (theta * hl - s * (ns / 2.0) * dsub) / d + N / 2.0;
                H.pb[axis][m][l] = pb;
                std::vector<int>& i0v = axis == 0 ? ix0 : jy0;
                std::vector<double>& tv = axis == 0 ? txd : tyd;
                const size_t base = i0v.size();
                for (int i = 0; i < nn; ++i) {
                    const double u = std::fma(pa, static_cast<double>(i), pb);
                    if (!(u >= 0.0 && u <= N - 1.0))
                        return fail(WMCAO_ERR_FOOTPRINT, "sensor " + std::to_string(m) +
                                    " leaves layer " + std::to_string(l));
                    int i0 = static_cast<int>(std::floor(u));
                    i0 = std::min(std::max(i0, 0), N - 2);
                    i0v.push_back(i0);
                    tv.push_back(u - i0);
                }
                // pixel rows (columns) that some node's bilinear stencil reaches
                std::vector<char>& hv = axis == 0 ? hitx : hity;
                for (int px = 0; px < N; ++px) hv.push_back(0);
                for (int i = 0; i < nn; ++i) {
                    const int i0 = i0v[base + i];
                    hv[hv.size() - N + i0] = 1;
                    hv[hv.size() - N + i0 + 1] = 1;
                }
            }
        }
    }
    p->n_slopes = soff;
    p->n_nodes = noff;
    for (int l = 0; l < n_layers; ++l) {   // pixels the projection reads
        const int N = layers[l].n;
        std::vector<char> hit(static_cast<size_t>(N) * N, 0);
        for (int m = 0; m < n_wfs; ++m) {
            const int nn = H.wfs[m].nn, no = H.node_tab_off[m][l];
            for (int i = 0; i < nn; ++i)
                for (int j = 0; j < nn; ++j)
                    for (int di = 0; di < 2; ++di)
                        for (int dj = 0; dj < 2; ++dj)
                            hit[static_cast<size_t>(ix0[no + i] + di) * N + jy0[no + j] + dj] = 1;
        }
        for (char c : hit) p->n_fp += c;
    }
    H.n_slopes = soff;
    H.n_nodes = noff;

    // adjoint footprints (Sec. 2.1 read backwards): per (sensor, layer) the
    // pixel rectangle the nodes' bilinear stencils reach, the node range that
    // feeds each of its rows and columns, and the rows per work item that keep
    // the staged node rows and the row-pass buffer within the plan's adjoint LDS
    std::vector<int> fprc;
    for (int m = 0; m < n_wfs; ++m) {
        const int nn = H.wfs[m].nn;
        for (int l = 0; l < n_layers; ++l) {
            const int N = layers[l].n, no = H.node_tab_off[m][l];
            int lo[2], len[2];
            const int tab = static_cast<int>(fprc.size() / 2);
            for (int axis = 0; axis < 2; ++axis) {
                const std::vector<int>& i0v = axis == 0 ? ix0 : jy0;
                std::vector<int> first(N, -1), last(N, -2);
                for (int i = 0; i < nn; ++i)
                    for (int px : {i0v[no + i], i0v[no + i] + 1}) {
                        if (first[px] < 0) first[px] = i;
                        last[px] = i;
                    }
                int a = N, b = -1;
                for (int px = 0; px < N; ++px)
                    if (first[px] >= 0) {
                        a = std::min(a, px);
                        b = std::max(b, px);
                    }
                lo[axis] = b >= a ? a : 0;
                len[axis] = b >= a ? b - a + 1 : 0;
                for (int px = lo[axis]; px < lo[axis] + len[axis]; ++px) {
                    fprc.push_back(first[px] < 0 ? 0 : first[px]);
                    fprc.push_back(first[px] < 0 ? 0 : last[px] - first[px] + 1);
                    // rows or columns fed by more than 4 nodes take the general loop
                    p->adj_taps = std::min(4, std::max(p->adj_taps, fprc.back()));
                }
            }
            H.fp_x0[m][l] = lo[0];
            H.fp_y0[m][l] = lo[1];
            H.fp_h[m][l] = len[0];
            H.fp_w[m][l] = len[1];
            H.fp_tab[m][l] = tab;
            H.fp_off[m][l] = static_cast<int>(p->n_fpimg);
            p->n_fpimg += static_cast<int64_t>(len[0]) * len[1];
            if (p->n_fpimg > (int64_t(1) << 30))
                return fail(WMCAO_ERR_UNSUPPORTED, "adjoint footprint images too large");
            // the level-1 analysis addresses one image with 32-bit byte offsets
            if (static_cast<int64_t>(len[0]) * len[1] * p->osz >= (int64_t(1) << 31))
                return fail(WMCAO_ERR_UNSUPPORTED, "adjoint footprint image too large");
            int br = ADJ_BAND, need = 0;
            for (; br >= 1; br /= 2) {
                need = 0;
                for (int r0 = 0; r0 < len[0]; r0 += br) {
                    int alo = nn, ahi = -1;
                    for (int r = r0; r < std::min(len[0], r0 + br); ++r) {
                        const int f = fprc[2 * (tab + r)], c = fprc[2 * (tab + r) + 1];
                        if (c > 0) {
                            alo = std::min(alo, f);
                            ahi = std::max(ahi, f + c - 1);
                        }
                    }
                    const int rows = std::min(len[0], r0 + br) - r0;
                    // staged node rows and the kernel's zero rows after them
                    // sized for FP64 arithmetic, so one band split serves both
                    const int vbytes = ahi < alo ? 0 : ((ahi - alo + ADJ_TAPS_MAX) * nn * 8 + 15) & ~15;
                    need = std::max(need, vbytes + rows * nn * 8);
                }
                if (need <= p->adj_lds) break;
            }
            if (br < 1)
                return fail(WMCAO_ERR_UNSUPPORTED, "sensor footprint too wide for the adjoint projection");
            H.fp_br[m][l] = br;
            // node rows each band reads: (first, last), after the row and column records
            for (int r0 = 0; r0 < len[0]; r0 += br) {
                int alo = nn, ahi = -1;
                for (int r = r0; r < std::min(len[0], r0 + br); ++r) {
                    const int f = fprc[2 * (tab + r)], c = fprc[2 * (tab + r) + 1];
                    if (c > 0) {
                        alo = std::min(alo, f);
                        ahi = std::max(ahi, f + c - 1);
                    }
                }
                fprc.push_back(alo);
                fprc.push_back(ahi);
            }
            p->lds_adjoint[1] = std::max(p->lds_adjoint[1], need);
            // the same bands with FP32 LDS
            for (int r0 = 0; r0 < len[0]; r0 += br) {
                int alo = nn, ahi = -1;
                for (int r = r0; r < std::min(len[0], r0 + br); ++r) {
                    const int f = fprc[2 * (tab + r)], c = fprc[2 * (tab + r) + 1];
                    if (c > 0) {
                        alo = std::min(alo, f);
                        ahi = std::max(ahi, f + c - 1);
                    }
                }
                const int rows = std::min(len[0], r0 + br) - r0;
                const int vbytes = ahi < alo ? 0 : ((ahi - alo + ADJ_TAPS_MAX) * nn * 4 + 15) & ~15;
                p->lds_adjoint[0] = std::max(p->lds_adjoint[0], vbytes + rows * nn * 4);
            }
        }
    }

    // ---- upload tables --------------------------------------------------
#define UP(vec, dst)                                          \
    do {                                                      \
        rc = upload_vec(p.get(), vec, &dst);                  \
        if (rc) return rc;                                    \
    } while (0)
    for (int m = 0; m < n_wfs; ++m) {
        UP(wh[m].act, H.wfs[m].act);
        UP(wh[m].cell_of, H.wfs[m].cell_of);
        UP(wh[m].cell_count, H.wfs[m].cell_count);
        UP(wh[m].maskmap, H.wfs[m].maskmap);
    }
    UP(ix0, H.ix0);
    UP(jy0, H.jy0);
    UP(fprc, H.fp_rc);
    {
        // adjoint-projection records per (layer, level-1 tile), or per layer at k0 = 0
        std::vector<int> meta;
        const int HT = p->tile / 2, PW = p->tile + 4;
        for (int l = 0; l < n_layers; ++l) {
            const int N = H.layer[l].N;
            H.tmeta_off[l] = static_cast<int>(meta.size());
            const int nt = H.layer[l].k0 >= 1 ? ceil_div(N / 2, HT) : 1;
            for (int t = 0; t < nt * nt; ++t) {
                int x0 = 0, y0 = 0, W0 = N;
                if (H.layer[l].k0 >= 1) {
                    x0 = 2 * (t % nt) * HT;
                    y0 = 2 * (t / nt) * HT;
                    W0 = PW;
                }
                unsigned mask = 0;
                for (int m = 0; m < n_wfs; ++m) {
                    const int po = pix_tab_off[m][l];
                    bool anyr = false, anyc = false;
                    for (int k = 0; k < W0; ++k) {
                        anyr = anyr || hitx[po + (x0 + k) % N];
                        anyc = anyc || hity[po + (y0 + k) % N];
                    }
                    if (anyr && anyc) mask |= 1u << m;
                }
                meta.push_back(static_cast<int>(mask));
            }
        }
        UP(meta, H.tmeta);
    }
    const double* txd_dev = nullptr;
    const double* tyd_dev = nullptr;
    const double* blk_dev_d = nullptr;
    UP(txd, txd_dev);
    UP(tyd, tyd_dev);
    UP(blocksd, blk_dev_d);
    // geometry weights and noise blocks stay FP64 for both dtypes (small tables)
    H.tx = txd_dev;
    H.ty = tyd_dev;
    for (int m = 0; m < n_wfs; ++m) H.wfs[m].blocks = blk_dev_d + H.wfs[m].boff * 3;

    // ---- slots and scratch ------------------------------------------------
    {
        int nf = 0;
        for (int l = 0; l < n_layers; ++l) {
            for (int k = 1; k <= H.layer[l].k0; ++k) {
                const int M = H.layer[l].N >> (k - 1);
                const int nt = ceil_div(M, p->tile);
                nf += nt * nt;
            }
        }
        H.pq_base = nf;   // per-layer totals follow the tile partials
        H.n_fdwt_slots = nf + n_layers;
        H.n_vec_slots = static_cast<int>((p->n + H.vec_chunk - 1) / H.vec_chunk);
        H.slots = std::max(H.n_fdwt_slots, H.n_vec_slots);
    }
    const int B = p->max_batch;
    const size_t ve = static_cast<size_t>(p->n) * B * p->esz;
    if (!(p->vb = p->alloc(ve, &rc))) return rc;
    if (!(p->vr = p->alloc(ve, &rc))) return rc;
    if (!(p->vp = p->alloc(ve, &rc))) return rc;
    if (!(p->vq = p->alloc(ve, &rc))) return rc;
    // operator scratch in the operator type
    if (!(p->vphi = p->alloc(static_cast<size_t>(p->n) * B * p->osz, &rc))) return rc;
    // low-pass bands in the arithmetic type of the stage using them (<= 8 bytes)
    if (!(p->vll = p->alloc(static_cast<size_t>(p->ll_size) * B * 8, &rc))) return rc;
    if (!(p->vnode = p->alloc(static_cast<size_t>(p->n_nodes) * B * p->osz, &rc))) return rc;
    if (!(p->vfp = p->alloc(static_cast<size_t>(p->n_fpimg) * B * p->osz, &rc))) return rc;
    if (!(p->vspart = static_cast<double*>(p->alloc(static_cast<size_t>(p->n_spart) * B * 8, &rc))))
        return rc;
    if (!(p->vu = static_cast<double*>(p->alloc(static_cast<size_t>(p->n_nodes) * B * 8, &rc)))) return rc;
    if (!(p->part = static_cast<double*>(p->alloc(sizeof(double) * NPT * H.slots * B, &rc)))) return rc;
    if (!(p->scal = static_cast<double*>(p->alloc(sizeof(double) * 4 * B, &rc)))) return rc;
    if (!(p->status = static_cast<int*>(p->alloc(sizeof(int) * B, &rc)))) return rc;
    WM_HIP(hipMemset(p->part, 0, sizeof(double) * NPT * H.slots * B));
    WM_HIP(hipMemset(p->scal, 0, sizeof(double) * 4 * B));
    WM_HIP(hipMemset(p->status, 0, sizeof(int) * B));

    // ---- Jacobi diagonal (Sec. 5.1), on the device ----------------------
    void* jac_t = nullptr;
    if (!(p->jac_d = static_cast<double*>(p->alloc(sizeof(double) * p->n, &rc)))) return rc;
    if (p->dtype == WMCAO_F32) {
        if (!(jac_t = p->alloc(sizeof(float) * p->n, &rc))) return rc;
    } else {
        jac_t = p->jac_d;
    }
    H.jac = jac_t;
    void* dev = nullptr;
    rc = upload(p.get(), &H, sizeof(PlanDev), &dev);
    if (rc) return rc;
    p->dev = static_cast<PlanDev*>(dev);
    {
        std::vector<double> protos;
        std::vector<int> poff(WM_MAXL * WM_MAXLEV * 2, 0);
        for (int l = 0; l < n_layers; ++l)
            for (int k = 1; k <= std::max(levels, 1); ++k)
                for (int t = 0; t < 2; ++t) {
                    poff[(l * WM_MAXLEV + (k - 1)) * 2 + t] = static_cast<int>(protos.size());
                    std::vector<double> v(H.layer[l].N, 0.0);
                    if (levels > 0) v = prototype(H.h, H.g, H.layer[l].N, k, t);
                    else v[0] = 1.0;   // no transform: the basis is the unit pixel
                    protos.insert(protos.end(), v.begin(), v.end());
                }
        const double* pr = nullptr;
        const int* po = nullptr;
        UP(protos, pr);
        UP(poff, po);
        launch_jacobi(p->dev, pr, po, txd_dev, tyd_dev, blk_dev_d, p->n, p->jac_d, nullptr);
        rc = check_launch();
        if (rc) return rc;
        if (p->dtype == WMCAO_F32)
            launch_cast<double, float>(p->jac_d, static_cast<float*>(jac_t), p->n, nullptr);
        rc = check_launch();
        if (rc) return rc;
        WM_HIP(hipDeviceSynchronize());
    }
#undef UP
    // the max_batch schedule (its frame prefixes serve the allocation-free
    // solve) and this device's address of the allocation-free scratch
    rc = get_sched(p.get(), p->max_batch, &p->full_sched);
    if (rc) return rc;
    char* nb = nullptr;
    rc = noalloc_base(p->device, &nb);
    if (rc) return rc;
    *out = p.release();
    return WMCAO_OK;
}

int wmcao_sizes(wmcao_plan_t plan, int64_t* n_coeffs, int64_t* n_slopes, int64_t* layer_offsets,
                int64_t* slope_offsets) {
    if (!plan) return fail(WMCAO_ERR_INVALID_ARG, "plan is NULL");
    if (n_coeffs) *n_coeffs = plan->n;
    if (n_slopes) *n_slopes = plan->n_slopes;
    if (layer_offsets)
        for (int l = 0; l <= plan->L; ++l) layer_offsets[l] = plan->layer_off[l];
    if (slope_offsets)
        for (int m = 0; m <= plan->W; ++m) slope_offsets[m] = plan->slope_off[m];
    return WMCAO_OK;
}

static int simple_call(wmcao_plan_t p, const void* in, void* out, int batch, void* stream,
                       int kind) {
    int rc = check_batch(p, batch);
    if (rc) return rc;
    if (!in || !out) return fail(WMCAO_ERR_INVALID_ARG, "NULL buffer");
    std::lock_guard<std::mutex> lk(p->mu);
    DevGuard g(p->device);
    Sched* S = nullptr;
    rc = get_sched(p, batch, &S);
    if (rc) return rc;
    JobArgs a{};
    a.njp = 1;
    a.jp[0] = make_jobplan(p, batch);
    a.jp[0].vec[V_IN] = const_cast<void*>(in);
    a.jp[0].vec[V_OUT] = out;
    hipStream_t s = static_cast<hipStream_t>(stream);
    ProfScope ps(&p->prof);
    // the operator stages read and write pixel fields in the operator type F;
    // when the caller's buffers hold another type (an FP32 plan with FP64
    // operators), pixel fields pass through the plan's pixel scratch
    const bool same = p->esz == p->osz;
    with_types(p, [&]<class T, class Sv>() {
        switch (kind) {
            case 0:   // W^-1
                a.jp[0].stride[V_IN] = a.jp[0].stride[V_OUT] = p->n;
                run_idwt<T, Sv>(a, *S, V_IN, same ? V_OUT : V_PHI, p->c64, s);
                if (!same)
                    launch_cast<Sv, T>(static_cast<const Sv*>(p->vphi), static_cast<T*>(out),
                                       p->n * batch, s);
                break;
            case 1:   // W
                a.jp[0].stride[V_IN] = a.jp[0].stride[V_OUT] = p->n;
                if (!same)
                    launch_cast<T, Sv>(static_cast<const T*>(in), static_cast<Sv*>(p->vphi),
                                       p->n * batch, s);
                run_fdwt<T, Sv>(a, *S, SRC_PIX, same ? V_IN : V_PHI, V_OUT, EPI_NONE, V_OUT, p->c64, s);
                break;
            case 2:   // forward slopes from layers
                a.jp[0].stride[V_IN] = p->n;
                a.jp[0].stride[V_OUT] = p->n_slopes;
                if (!same)
                    launch_cast<T, Sv>(static_cast<const T*>(in), static_cast<Sv*>(p->vphi),
                                       p->n * batch, s);
                launch_project<T, Sv>(a, S->proj, S->n_proj, same ? V_IN : V_PHI, 0, S->lds_project, S->max_layers, s);
                launch_sensor<T, Sv>(a, S->sensor, S->n_sensor, SM_FWD, V_U, V_OUT, S->lds_sensor, s);
                break;
            case 3:   // rhs
                a.jp[0].stride[V_IN] = p->n_slopes;
                a.jp[0].stride[V_OUT] = p->n;
                run_rhs<T, Sv>(a, *S, V_IN, V_OUT, p->c64, s);
                break;
            case 4:   // apply
                a.jp[0].stride[V_IN] = a.jp[0].stride[V_OUT] = p->n;
                run_apply<T, Sv>(a, *S, V_IN, V_OUT, p->c64, s);
                break;
        }
    });
    if (kind < 0 || kind > 4) return fail(WMCAO_ERR_INVALID_ARG, "kind");
    return check_launch();
}

int wmcao_coeffs_to_layers(wmcao_plan_t plan, const void* coeffs, void* layers, int batch,
                           void* hip_stream) {
    return simple_call(plan, coeffs, layers, batch, hip_stream, 0);
}

int wmcao_layers_to_coeffs(wmcao_plan_t plan, const void* layers, void* coeffs, int batch,
                           void* hip_stream) {
    return simple_call(plan, layers, coeffs, batch, hip_stream, 1);
}

int wmcao_forward_layers(wmcao_plan_t plan, const void* layers, void* slopes, int batch,
                         void* hip_stream) {
    return simple_call(plan, layers, slopes, batch, hip_stream, 2);
}

int wmcao_rhs(wmcao_plan_t plan, const void* slopes, void* b, int batch, void* hip_stream) {
    return simple_call(plan, slopes, b, batch, hip_stream, 3);
}

int wmcao_apply_A(wmcao_plan_t plan, const void* x, void* y, int batch, void* hip_stream) {
    if (x == y) return fail(WMCAO_ERR_INVALID_ARG, "x and y must not alias");
    return simple_call(plan, x, y, batch, hip_stream, 4);
}

int wmcao_precond_diag(wmcao_plan_t plan, double* j_dev, void* hip_stream) {
    if (!plan || !j_dev) return fail(WMCAO_ERR_INVALID_ARG, "NULL argument");
    DevGuard g(plan->device);
    WM_HIP(hipMemcpyAsync(j_dev, plan->jac_d, sizeof(double) * plan->n, hipMemcpyDeviceToDevice,
                          static_cast<hipStream_t>(hip_stream)));
    return WMCAO_OK;
}

int wmcao_solve(wmcao_plan_t plan, const void* slopes, void* coeffs, int batch, int n_iter,
                int warm_start, double* resid_dev, int* status_dev, void* hip_stream) {
    int rc = check_batch(plan, batch);
    if (rc) return rc;
    if (!slopes || !coeffs) return fail(WMCAO_ERR_INVALID_ARG, "NULL buffer");
    if (n_iter < 0) return fail(WMCAO_ERR_INVALID_ARG, "n_iter < 0");
    std::lock_guard<std::mutex> lk(plan->mu);
    DevGuard g(plan->device);
    ProfScope ps(&plan->prof);
    return enqueue_solve(plan, slopes, coeffs, batch, n_iter, warm_start, resid_dev, status_dev,
                         static_cast<hipStream_t>(hip_stream));
}

int wmcao_solve_graph(wmcao_plan_t plan, const void* slopes, void* coeffs, int batch, int n_iter,
                      int warm_start, double* resid_dev, int* status_dev, void* hip_stream) {
    int rc = check_batch(plan, batch);
    if (rc) return rc;
    if (!slopes || !coeffs) return fail(WMCAO_ERR_INVALID_ARG, "NULL buffer");
    if (!hip_stream) return fail(WMCAO_ERR_INVALID_ARG, "graph capture needs a non-default stream");
    if (n_iter < 0) return fail(WMCAO_ERR_INVALID_ARG, "n_iter < 0");
    std::lock_guard<std::mutex> lk(plan->mu);
    DevGuard g(plan->device);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    auto key = std::make_tuple(slopes, coeffs, batch, n_iter, warm_start, resid_dev, status_dev,
                               hip_stream);
    if (!plan->gexec || plan->gkey != key) {
        rc = prepare_solve(plan, batch);   // outside the capture (it allocates)
        if (rc) return rc;
        if (plan->gexec) {   // replaced: wait for its last replay before freeing it
            if (plan->gdone) (void)hipEventSynchronize(plan->gdone);
            (void)hipGraphExecDestroy(plan->gexec);
            plan->gexec = nullptr;
        }
        if (!plan->gdone) WM_HIP(hipEventCreateWithFlags(&plan->gdone, hipEventDisableTiming));
        WM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        rc = enqueue_solve(plan, slopes, coeffs, batch, n_iter, warm_start, resid_dev, status_dev, s);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(s, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(WMCAO_ERR_HIP, std::string("capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&plan->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            plan->gexec = nullptr;
            return fail(WMCAO_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(e));
        }
        plan->gkey = key;
    }
    WM_HIP(hipGraphLaunch(plan->gexec, s));
    WM_HIP(hipEventRecord(plan->gdone, s));
    return WMCAO_OK;
}

int wmcao_solve_noalloc(wmcao_plan_t plan, const void* slopes, void* coeffs, int batch, int n_iter,
                        int warm_start, double* resid_dev, int* status_dev, void* hip_stream) {
    int rc = check_batch(plan, batch);
    if (rc) return rc;
    if (!slopes || !coeffs) return fail(WMCAO_ERR_INVALID_ARG, "NULL buffer");
    if (n_iter < 0) return fail(WMCAO_ERR_INVALID_ARG, "n_iter < 0");
    const size_t need = carve_noalloc(plan, batch, nullptr, nullptr);
    if (need > NOALLOC_BYTES)
        return fail(WMCAO_ERR_SIZE, "wmcao_solve_noalloc: " + std::to_string(batch) + " frames need " +
                                        std::to_string(need) + " bytes of scratch, more than its " +
                                        std::to_string(NOALLOC_BYTES) + " bytes");
    std::lock_guard<std::mutex> lk(plan->mu);
    DevGuard g(plan->device);
    char* base = nullptr;
    rc = noalloc_base(plan->device, &base);
    if (rc) return rc;
    const Sched* full = plan->full_sched;
    if (!full || full->frames != plan->max_batch) return fail(WMCAO_ERR_INVALID_ARG, "plan has no schedule");
    // the first `batch` frames of the max_batch schedule: every stage's item
    // list is frame-major, so its prefix is the schedule of those frames
    Sched v = *full;
    const int fb = full->frames;
    auto scale = [&](int cnt) { return cnt / fb * batch; };
    v.n_coarse = scale(full->n_coarse);
    v.n_coarse_syn = scale(full->n_coarse_syn);
    for (int k = 0; k <= WM_MAXLEV; ++k) v.n_tiled[k] = scale(full->n_tiled[k]);
    v.n_sensor = scale(full->n_sensor);
    v.n_proj = scale(full->n_proj);
    v.n_wgt = scale(full->n_wgt);
    v.n_proj_ap = scale(full->n_proj_ap);
    v.n_papply = scale(full->n_papply);
    v.n_adj = scale(full->n_adj);
    v.n_vec = scale(full->n_vec);
    v.frames = batch;
    JobArgs a{};
    a.njp = 1;
    a.jp[0] = make_jobplan(plan, batch);
    carve_noalloc(plan, batch, base, &a.jp[0]);
    a.jp[0].vec[V_X] = coeffs;
    a.jp[0].vec[V_SLOPES] = const_cast<void*>(slopes);
    if (status_dev) a.jp[0].status = status_dev;
    a.jp[0].resid = resid_dev;
    a.jp[0].resid_ld = n_iter + 1;
    ProfScope ps(nullptr);   // no event timing: it would create events
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    with_types(plan, [&]<class T, class Sv>() {
        run_solve<T, Sv>(a, v, n_iter, warm_start, plan->resid_replace, plan->c64, s);
    });
    return check_launch();
}

int wmcao_solve_multi(const wmcao_plan_t* plans, const void* const* slopes, void* const* coeffs,
                      const int* counts, int n_plans, int n_iter, int warm_start,
                      void* hip_stream) {
    std::lock_guard<std::mutex> lk(g_multi_mu);
    return enqueue_multi(plans, slopes, coeffs, counts, n_plans, n_iter, warm_start,
                         static_cast<hipStream_t>(hip_stream));
}

int wmcao_solve_multi_graph(const wmcao_plan_t* plans, const void* const* slopes,
                            void* const* coeffs, const int* counts, int n_plans, int n_iter,
                            int warm_start, void* hip_stream) {
    if (!hip_stream) return fail(WMCAO_ERR_INVALID_ARG, "graph capture needs a non-default stream");
    if (!plans || !slopes || !coeffs || !counts) return fail(WMCAO_ERR_INVALID_ARG, "NULL argument");
    if (n_plans < 1 || n_plans > WM_MAXJP) return fail(WMCAO_ERR_INVALID_ARG, "n_plans out of range");
    std::lock_guard<std::mutex> lk(g_multi_mu);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    MultiGraphKey key;
    for (int i = 0; i < n_plans; ++i)
        key.args.push_back(std::make_tuple(static_cast<const void*>(plans[i]), slopes[i],
                                           static_cast<const void*>(coeffs[i]), counts[i]));
    key.n_iter = n_iter;
    key.warm = warm_start;
    key.stream = hip_stream;
    auto it = g_multi_graphs.find(key);
    if (it == g_multi_graphs.end()) {
        // build the schedule outside the capture (it allocates), then record
        int rc = enqueue_multi(plans, slopes, coeffs, counts, n_plans, n_iter, warm_start, s,
                               /*prepare_only=*/true);
        if (rc) return rc;
        if (g_multi_graphs.size() >= MULTI_GRAPH_CACHE) {   // evict the least recently used
            auto lru = g_multi_graphs.begin();
            for (auto jt = g_multi_graphs.begin(); jt != g_multi_graphs.end(); ++jt)
                if (jt->second.last_use < lru->second.last_use) lru = jt;
            destroy_cached(lru->second);
            g_multi_graphs.erase(lru);
        }
        DevGuard g(plans[0]->device);
        WM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        rc = enqueue_multi(plans, slopes, coeffs, counts, n_plans, n_iter, warm_start, s);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(s, &graph);
        if (rc) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return fail(WMCAO_ERR_HIP, std::string("capture: ") + hipGetErrorString(e));
        CachedGraph cg;
        e = hipGraphInstantiate(&cg.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(WMCAO_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(e));
        e = hipEventCreateWithFlags(&cg.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipGraphExecDestroy(cg.exec);
            return fail(WMCAO_ERR_HIP, std::string("event: ") + hipGetErrorString(e));
        }
        it = g_multi_graphs.emplace(key, cg).first;
    }
    DevGuard g(plans[0]->device);
    it->second.last_use = ++g_graph_clock;
    WM_HIP(hipGraphLaunch(it->second.exec, s));
    WM_HIP(hipEventRecord(it->second.done, s));
    return WMCAO_OK;
}

int wmcao_profile_enable(wmcao_plan_t plan, int enable) {
    if (!plan) return fail(WMCAO_ERR_INVALID_ARG, "plan is NULL");
    std::lock_guard<std::mutex> lk(plan->mu);
    DevGuard g(plan->device);
    if (enable) {
        WM_HIP(hipDeviceSynchronize());
        plan->prof.clear();
    }
    plan->prof.on = enable != 0;
    return WMCAO_OK;
}

int wmcao_profile_read(wmcao_plan_t plan, int kind, double* total_ms, int* launches,
                       double* bytes) {
    if (!plan || !total_ms || !launches || kind < 0 || kind >= WMCAO_K_COUNT)
        return fail(WMCAO_ERR_INVALID_ARG, "bad argument");
    std::lock_guard<std::mutex> lk(plan->mu);
    DevGuard g(plan->device);
    double tot = 0.0, by = 0.0;
    int cnt = 0;
    for (auto& r : plan->prof.rec) {
        if (std::get<0>(r) != kind) continue;
        WM_HIP(hipEventSynchronize(std::get<2>(r)));
        float ms = 0.0f;
        WM_HIP(hipEventElapsedTime(&ms, std::get<1>(r), std::get<2>(r)));
        tot += ms;
        by += std::get<3>(r);
        ++cnt;
    }
    *total_ms = tot;
    *launches = cnt;
    if (bytes) *bytes = by;
    return WMCAO_OK;
}

int wmcao_serve_launch(wmcao_plan_t plan, void* stage_slopes, void* stage_coeffs, int count,
                       const void* const* slopes, const void* const* warm, int n_out,
                       const int* out_rows, void* const* out_ptrs, int n_iter, void* hip_stream) {
    if (!plan || !stage_slopes || !stage_coeffs || !slopes || !warm || (n_out > 0 && (!out_rows || !out_ptrs)))
        return fail(WMCAO_ERR_INVALID_ARG, "NULL argument");
    if (!hip_stream) return fail(WMCAO_ERR_INVALID_ARG, "a served launch needs a non-default stream");
    if (count < 1 || count > plan->max_batch || 2 * count > SERVE_ROWS)
        return fail(WMCAO_ERR_INVALID_ARG, "count must be 1 .. min(max_batch, " +
                                               std::to_string(SERVE_ROWS / 2) + ")");
    if (n_out < 0 || n_out > SERVE_ROWS)
        return fail(WMCAO_ERR_INVALID_ARG, "n_out must be 0 .. " + std::to_string(SERVE_ROWS));
    for (int i = 0; i < count; ++i)
        if (!slopes[i] || !warm[i]) return fail(WMCAO_ERR_INVALID_ARG, "NULL frame pointer");
    for (int i = 0; i < n_out; ++i)
        if (!out_ptrs[i] || out_rows[i] < 0 || out_rows[i] >= count)
            return fail(WMCAO_ERR_INVALID_ARG, "out row out of range");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int64_t wn = plan->n * static_cast<int64_t>(plan->esz) / 4;
    const int64_t ws = plan->n_slopes * static_cast<int64_t>(plan->esz) / 4;
    char* sb = static_cast<char*>(stage_slopes);
    char* xb = static_cast<char*>(stage_coeffs);
    DevGuard g(plan->device);
    CopyRows in{};
    for (int i = 0; i < count; ++i) {
        in.src[i] = slopes[i];
        in.dst[i] = sb + i * ws * 4;
        in.len[i] = ws;
        in.src[count + i] = warm[i];
        in.dst[count + i] = xb + i * wn * 4;
        in.len[count + i] = wn;
    }
    launch_copy_rows(in, 2 * count, std::max(wn, ws), s);
    int rc = check_launch();
    if (rc) return rc;
    const void* sbc = stage_slopes;
    rc = wmcao_solve_multi_graph(&plan, &sbc, &stage_coeffs, &count, 1, n_iter, 1, hip_stream);
    if (rc) return rc;
    CopyRows out{};
    for (int i = 0; i < n_out; ++i) {
        out.src[i] = xb + out_rows[i] * wn * 4;
        out.dst[i] = out_ptrs[i];
        out.len[i] = wn;
    }
    launch_copy_rows(out, n_out, wn, s);
    return check_launch();
}

int wmcao_axpby(wmcao_dtype dtype, int64_t n, double a, const void* x, double b, const void* y,
                void* out, void* hip_stream) {
    if (n < 0 || (n > 0 && (!x || !y || !out))) return fail(WMCAO_ERR_INVALID_ARG, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (dtype == WMCAO_F32)
        launch_axpby<float>(n, a, static_cast<const float*>(x), b, static_cast<const float*>(y),
                            static_cast<float*>(out), s);
    else if (dtype == WMCAO_F64)
        launch_axpby<double>(n, a, static_cast<const double*>(x), b, static_cast<const double*>(y),
                             static_cast<double*>(out), s);
    else
        return fail(WMCAO_ERR_INVALID_ARG, "dtype");
    return check_launch();
}

void wmcao_plan_destroy(wmcao_plan_t plan) {
    if (!plan) return;
    DevGuard g(plan->device);
    (void)hipDeviceSynchronize();
    {
        std::lock_guard<std::mutex> lk(g_multi_mu);
        for (auto it = g_multi_cache.begin(); it != g_multi_cache.end();) {
            bool uses = false;
            for (auto& kv : it->first) uses = uses || std::get<0>(kv) == plan;
            if (uses) it = g_multi_cache.erase(it); else ++it;
        }
        for (auto it = g_multi_graphs.begin(); it != g_multi_graphs.end();) {
            bool uses = false;
            for (auto& t : it->first.args) uses = uses || std::get<0>(t) == plan;
            if (uses) {
                destroy_cached(it->second);
                it = g_multi_graphs.erase(it);
            } else {
                ++it;
            }
        }
    }
    if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
    if (plan->gdone) (void)hipEventDestroy(plan->gdone);
    if (plan->ev_fork) (void)hipEventDestroy(plan->ev_fork);
    for (int i = 0; i < 3; ++i) {
        if (plan->ev_join[i]) (void)hipEventDestroy(plan->ev_join[i]);
        if (plan->side[i]) (void)hipStreamDestroy(plan->side[i]);
    }
    delete plan;
}

}  // extern "C"
