// C ABI of libp2m (declared in include/p2m.h): argument validation, workspace
// carving and the launch sequence of every entry point.  No device memory is
// allocated here; every launch goes on the caller's stream.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "p2m_internal.hpp"

using namespace p2m;

namespace {

// The graph of the last batch submitted on a context, relaunched as long as the
// batch (instance table, field count, options, workspace, reports) is unchanged.
struct BatchCache {
    std::vector<unsigned char> key;
    std::vector<unsigned char> upload;   // instance table and tile maps (host copy)
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        key.clear();
    }
    ~BatchCache() {
        release();
        if (capture) (void)hipStreamDestroy(capture);
    }
};

// Tuned plans by shape class (see shape_key).
struct PlanCache {
    std::map<std::string, p2m_plan, std::less<>> plans;   // transparent: found by char key
};

struct Context {
    int device;
    int cg_blocks_f32;
    int cg_blocks_f64;
    int solver_mode;        // P2M_SOLVER_*: AUTO or a forced solve kernel
    int use_plans;          // 1: apply tuned plans of the problem's shape class
    long scan_spin;         // bound of the binning scan's look-back wait (< 0: test hook)
    long solve_spin;        // bound of a solve's grid-barrier wait (< 0: test hook)
    int fft;                // 1: circulant mesh systems by the 2D FFT where the sides allow
    BatchCache* batch;      // created on the first batched call
    const float* learned;   // parameters of the learned start (device), or null
    PlanCache* plans;       // created on the first tuned or loaded plan
    const p2m_plan* forced; // the candidate being timed by p2m_tune
    void* scratch;          // device address of this device's static scratch, or null
};

// Makes the context's device current for the duration of a call and restores
// the caller's device afterwards.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ---------------------------------------------------------------------------
// Static scratch of p2m_mass_assign_noalloc: the workspace of that entry point is
// this file-scope device array (one copy per device, held by the loaded code
// object until the process ends).  Host code never uses the array's name as an
// address: p2m_create looks the device address up once per device with
// hipGetSymbolAddress, and every use goes through that pointer.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)P2M_SCRATCH_BYTES;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_dev[kScratchDevices];   // device address per device (null: not looked up)

// The device address of `scratch` on `device`, which must be current; null when
// the lookup fails (the no-allocation entry point then reports P2M_ERR_HIP).
void* scratch_address(int device) {
    if (device < 0 || device >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p) g_scratch_dev[device] = p;
        else (void)hipGetLastError();   // leave no sticky error for the caller's next call
    }
    return g_scratch_dev[device];
}

// Workspace carve-up.  Offsets are fixed functions of (problem, F, cg blocks).
struct Layout {
    size_t key, counts, cell_start, perm, scan, b, w, coef, r, p0, p1, q, dinv, x64, partials,
        resident, tiles, learned, report, total;
};

Layout make_layout(const Mesh& m, int F, size_t tsize, int cg_blocks) {
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t np = (size_t)m.np, nn = (size_t)m.nn;
    const size_t cm = (m.dim == 2) ? 4 : 2;
    L.key = take(2 * np * sizeof(int32_t));      // cell keys, then in-cell ranks
    L.counts = take(nn * sizeof(int32_t));
    L.scan = take(scan_workspace_bytes((int)nn));   // right after counts: one fill clears both
    L.cell_start = take((nn + 1) * sizeof(int32_t));
    L.perm = take(np * sizeof(int32_t));
    L.b = take((size_t)F * nn * tsize);
    L.w = take(nn * tsize);
    L.coef = take(cm * nn * tsize);
    L.r = take((size_t)F * nn * tsize);
    L.p0 = take((size_t)F * nn * tsize);
    L.p1 = take((size_t)F * nn * tsize);
    L.q = take((size_t)F * nn * tsize);
    L.dinv = take(nn * tsize);
    L.x64 = take((size_t)2 * F * nn * sizeof(double));
    L.partials = take(cg_partials_bytes(cg_blocks));
    L.resident = take((m.dim == 2 && F <= kResidentMaxFields && tsize == 4)
                          ? cgr_workspace_bytes(m, F, cgr_tiles(m)) : 0);
    L.tiles = take((m.dim == 2 && F <= kResidentMaxFields && tsize == 4) ? cgt_workspace_bytes(m, F)
                                                                         : 0);
    L.learned = take((m.dim == 2 && tsize == 4) ? learned_start_workspace_bytes(m, F) : 0);
    L.report = take(sizeof(p2m_report));
    L.total = off;
    return L;
}

inline size_t tsize_of(const p2m_problem* p) { return p->dtype == P2M_F64 ? 8 : 4; }

int cg_blocks_for(const Context* c, const Mesh& m, int dtype) {
    int maxb = dtype == P2M_F64 ? c->cg_blocks_f64 : c->cg_blocks_f32;
    int need = (m.nn + 255) / 256;
    int b = need < maxb ? need : maxb;
    return b < 1 ? 1 : b;
}

template <typename T>
Particles<T> particles_of(const p2m_problem* p) {
    Particles<T> P;
    P.x = (const T*)p->x;
    P.y = (const T*)p->y;
    P.vol = (const T*)p->vol;
    return P;
}

// Shape class of a batch for tuned plans: field count, and the instance count, total
// nodes and total particles, each rounded to a power of two.
// A shape-class key in a fixed buffer (looking a plan up allocates nothing).
struct Key {
    char s[96];
};

Key batch_key(int F, int nprob, int64_t nn, int64_t np) {
    auto lg = [](double v) { return (int)floor(log2(v > 1.0 ? v : 1.0) + 0.5); };
    Key k;
    snprintf(k.s, sizeof k.s, "batch-f32-F%d-n%d-nodes%d-parts%d", F, lg(nprob), lg((double)nn),
             lg((double)np));
    return k;
}

// Shape class of a problem for tuned plans: dimension, dtype, field count, the
// mesh sides and the particles per cell, each rounded to a power of two.
Key shape_key(const Mesh& m, int dtype, int F) {
    auto lg = [](double v) { return (int)floor(log2(v) + 0.5); };
    const double ppc = m.np > 0 ? (double)m.np / (double)m.nn : 0.125;
    Key k;
    snprintf(k.s, sizeof k.s, "%dd-%s-F%d-nx%d-ny%d-ppc%d", m.dim, dtype == P2M_F64 ? "f64" : "f32", F,
             lg(m.nx), lg(m.ny), lg(ppc < 0.125 ? 0.125 : ppc));
    return k;
}

struct Choice {
    int solver = P2M_SOLVER_AUTO;
    int groups = 0;
    int tile = 0;
    double inner_rtol = -1.0;   // < 0: the caller's
};

Choice choose(const Context* c, const Mesh& m, int dtype, int F) {
    Choice ch;
    if (c->forced) {
        ch.solver = c->forced->solver;
        ch.groups = c->forced->groups;
        ch.tile = c->forced->scatter_tile;
        ch.inner_rtol = c->forced->inner_rtol;
        return ch;
    }
    if (c->use_plans && c->plans) {
        auto it = c->plans->plans.find(shape_key(m, dtype, F).s);
        if (it != c->plans->plans.end()) {
            ch.solver = it->second.solver;
            ch.groups = it->second.groups;
            ch.tile = it->second.scatter_tile;
            ch.inner_rtol = it->second.inner_rtol;
        }
    }
    if (c->solver_mode != P2M_SOLVER_AUTO) ch.solver = c->solver_mode;
    return ch;
}

inline p2m_status st(hipError_t e) { return e == hipSuccess ? P2M_OK : P2M_ERR_HIP; }
#define P2M_TRY(expr)                               \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) return P2M_ERR_HIP;   \
    } while (0)

struct Prepared {
    Mesh m;
    Layout L;
    char* ws;
    hipStream_t stream;
    p2m_report* rep;
    long scan_spin;
    long solve_spin;
    // the report still has to be zeroed: the first launch of the call does it
    // together with its own clearing work (one launch fewer per call)
    mutable bool clear_rep = false;
};

p2m_status prepare(void* ctx, const p2m_problem* prob, int F, void* ws, size_t ws_bytes,
                   void* stream, p2m_report* rep, Prepared& out) {
    if (!ctx) return P2M_ERR_INVALID_ARG;
    if (F < 1 || F > kMaxFields) return P2M_ERR_INVALID_ARG;
    p2m_status s = check_problem(prob, out.m);
    if (s != P2M_OK) return s;
    const Context* c = (const Context*)ctx;
    out.L = make_layout(out.m, F, tsize_of(prob), cg_blocks_for(c, out.m, prob->dtype));
    if (!ws || ws_bytes < out.L.total) return P2M_ERR_WORKSPACE;
    if (((uintptr_t)ws) % kAlign) return P2M_ERR_WORKSPACE;
    out.ws = (char*)ws;
    out.stream = (hipStream_t)stream;
    out.rep = rep ? rep : (p2m_report*)(out.ws + out.L.report);
    out.scan_spin = c->scan_spin;
    out.solve_spin = c->solve_spin;
    return P2M_OK;
}

template <typename T>
p2m_status run_bin(const Prepared& pp, const p2m_problem* prob, int32_t* perm, int32_t* cs) {
    const Mesh& m = pp.m;
    int32_t* key = (int32_t*)(pp.ws + pp.L.key);
    int32_t* counts = (int32_t*)(pp.ws + pp.L.counts);
    int32_t* rank = key + m.np;
    void* scan_ws = pp.ws + pp.L.scan;
    const size_t clear = (pp.L.scan + scan_workspace_bytes(m.nn) - pp.L.counts) / sizeof(int32_t);
    // counts and the scan's words (and the report, when the call has not cleared it)
    P2M_TRY(launch_fill_i32(counts, 0, clear, pp.stream, pp.clear_rep ? pp.rep : nullptr));
    pp.clear_rep = false;
    P2M_TRY(launch_locate_count<T>(m, particles_of<T>(prob), key, rank, counts, pp.rep,
                                   pp.stream));
    P2M_TRY(launch_exclusive_scan(counts, cs, m.nn, scan_ws, pp.scan_spin, pp.rep, 1, pp.stream));
    P2M_TRY(launch_place(m, key, rank, cs, perm, scan_ws, pp.stream));
    P2M_TRY(launch_segment_sort(m, cs, perm, pp.stream));
    return P2M_OK;
}

template <typename T>
p2m_status run_assign(const Prepared& pp, const p2m_problem* prob, p2m_assign_kind kind,
                      const void* values, int F, void* nodal_out) {
    int32_t* perm = (int32_t*)(pp.ws + pp.L.perm);
    int32_t* cs = (int32_t*)(pp.ws + pp.L.cell_start);
    p2m_status s = run_bin<T>(pp, prob, perm, cs);
    if (s != P2M_OK) return s;
    if (kind == P2M_DELTA) {
        P2M_TRY(launch_delta1d<T>(pp.m, particles_of<T>(prob), (const T*)values, F, perm, cs,
                                  (T*)nodal_out, pp.stream));
        return P2M_OK;
    }
    T* b = (T*)(pp.ws + pp.L.b);
    T* w = (T*)(pp.ws + pp.L.w);
    P2M_TRY(launch_assemble<T>(pp.m, particles_of<T>(prob), (const T*)values, F, perm, cs, b, w,
                               nullptr, pp.stream));
    P2M_TRY(launch_finalize<T>(pp.m, F, b, w, kind == P2M_PIC ? 1 : 0, (T*)nodal_out, pp.rep,
                               pp.stream));
    return P2M_OK;
}

template <typename T>
p2m_status run_assemble(const Prepared& pp, const p2m_problem* prob, const void* values, int F,
                        void* b, void* w, void* coef, const Choice& ch) {
    int32_t* perm = (int32_t*)(pp.ws + pp.L.perm);
    int32_t* cs = (int32_t*)(pp.ws + pp.L.cell_start);
    p2m_status s = run_bin<T>(pp, prob, perm, cs);
    if (s != P2M_OK) return s;
    P2M_TRY(launch_assemble<T>(pp.m, particles_of<T>(prob), (const T*)values, F, perm, cs, (T*)b,
                               (T*)w, (T*)coef, pp.stream, ch.tile));
    return P2M_OK;
}

// Solve kernel: the choice's kernel where it applies; AUTO and RESIDENT take the
// register-resident kernel where the mesh fits, else the tile-streaming one, else
// the grid-synchronised streaming kernel (1D, FP64, F > 3).
template <typename T>
p2m_status run_solve(const Context* c, const Prepared& pp, int F, T* b, const T* w, T* coef,
                     int start, const p2m_solve_opts& caller_opts, void* x, const Choice& ch) {
    p2m_solve_opts opts = caller_opts;
    if (ch.inner_rtol >= 0.0 && ch.inner_rtol < 1.0) opts.inner_rtol = ch.inner_rtol;
    const bool tiled = sizeof(T) == 4 && pp.m.dim == 2 && F <= kResidentMaxFields;
    const int kind = ch.solver;
    if (tiled && kind == P2M_SOLVER_RESIDENT_CHEB && cgrc_supported(pp.m, F, c->device)) {
        P2M_TRY(launch_cg_resident_cheb(pp.m, F, (float*)coef, (float*)b, (const float*)w,
                                        (float*)x, start, pp.ws + pp.L.resident, opts, pp.rep,
                                        pp.clear_rep, pp.solve_spin, pp.stream));
        pp.clear_rep = false;
        return P2M_OK;
    }
    if (tiled && (kind == P2M_SOLVER_AUTO || kind == P2M_SOLVER_RESIDENT ||
                  kind == P2M_SOLVER_RESIDENT_CHEB) &&
        cgr_supported(pp.m, F, c->device)) {
        P2M_TRY(launch_cg_resident(pp.m, F, (float*)coef, (float*)b, (const float*)w, (float*)x,
                                   start, pp.ws + pp.L.resident, opts, pp.rep, pp.clear_rep,
                                   pp.solve_spin, pp.stream));
        pp.clear_rep = false;
        return P2M_OK;
    }
    if (pp.clear_rep) {
        P2M_TRY(launch_report_clear(pp.rep, pp.stream));
        pp.clear_rep = false;
    }
    if (tiled && kind != P2M_SOLVER_STREAMING && cgt_grid(pp.m, F, ch.groups, c->device) > 0) {
        P2M_TRY(launch_cg_tiles(pp.m, F, (float*)coef, (float*)b, (const float*)w, (float*)x, start,
                                pp.ws + pp.L.tiles, opts, pp.rep, ch.groups, c->device,
                                pp.solve_spin, pp.stream));
        return P2M_OK;
    }
    CgWorkspace cw;
    cw.r = pp.ws + pp.L.r;
    cw.p0 = pp.ws + pp.L.p0;
    cw.p1 = pp.ws + pp.L.p1;
    cw.q = pp.ws + pp.L.q;
    cw.x64 = (double*)(pp.ws + pp.L.x64);
    cw.partials = (double*)(pp.ws + pp.L.partials);
    cw.dinv = pp.ws + pp.L.dinv;
    cw.blocks = cg_blocks_for(c, pp.m, sizeof(T) == 8 ? P2M_F64 : P2M_F32);
    cw.spin = pp.solve_spin;
    P2M_TRY(launch_cg<T>(pp.m, F, coef, b, w, (T*)x, start, cw, opts, pp.rep, pp.stream));
    return P2M_OK;
}

template <typename T>
p2m_status run_mass(const Context* c, const Prepared& pp, const p2m_problem* prob,
                    const void* values, int F, const p2m_solve_opts& opts, void* x,
                    const Choice& ch) {
    int32_t* perm = (int32_t*)(pp.ws + pp.L.perm);
    int32_t* cs = (int32_t*)(pp.ws + pp.L.cell_start);
    p2m_status s = run_bin<T>(pp, prob, perm, cs);
    if (s != P2M_OK) return s;
    T* b = (T*)(pp.ws + pp.L.b);
    T* w = (T*)(pp.ws + pp.L.w);
    T* coef = (T*)(pp.ws + pp.L.coef);
    P2M_TRY(launch_assemble<T>(pp.m, particles_of<T>(prob), (const T*)values, F, perm, cs, b, w,
                               coef, pp.stream, ch.tile));
    int start = opts.start;
    if (start == P2M_START_LEARNED) {
        if (sizeof(T) != 4) return P2M_ERR_UNSUPPORTED;
        P2M_TRY(launch_learned_start(pp.m, particles_of<float>(prob), (const float*)values, F, perm,
                                     cs, (const float*)b, (const float*)w, (const float*)coef,
                                     c->learned, (float*)x, pp.ws + pp.L.learned, pp.rep,
                                     pp.stream));
        start = P2M_START_USER;
    }
    if (start == P2M_START_DELTA1D) {
        P2M_TRY(launch_delta1d<T>(pp.m, particles_of<T>(prob), (const T*)values, F, perm, cs,
                                  (T*)x, pp.stream));
        start = P2M_START_USER;
    }
    return run_solve<T>(c, pp, F, b, w, coef, start, opts, x, ch);
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
struct BatchPlan {
    int nprob = 0, F = 0;
    int64_t np = 0, nn = 0;              // particles and nodes of the whole batch
    int nlb = 0, nat = 0, nrt = 0;       // locate blocks, scatter tiles, solver tiles
    int grid = 0;                        // workgroups of the batched solve
    std::vector<BatchInst> inst;
    std::vector<int32_t> lmap, amap, rmap, omap;
    size_t inst_b = 0, lmap_b = 0, amap_b = 0, rmap_b = 0, omap_b = 0;   // upload sections
    size_t o_key = 0, o_counts = 0, o_cs = 0, o_perm = 0, o_scan = 0, o_b = 0, o_w = 0,
           o_coef = 0, o_solve = 0, total = 0;
};

// Validates the batch and lays out its workspace.  values / outs / reps may be
// null for a size query.
p2m_status plan_batch(const Context* c, const p2m_problem* probs, int nprob, int F,
                      const void* const* values, void* const* outs, p2m_report* reps,
                      BatchPlan& P) {
    if (!probs || nprob < 1 || F < 1 || F > kMaxFields) return P2M_ERR_INVALID_ARG;
    if (F > kResidentMaxFields || nprob > kBatchMaxInstances || nprob * F > kBatchMaxPairs)
        return P2M_ERR_UNSUPPORTED;
    P.nprob = nprob;
    P.F = F;
    P.inst.resize(nprob);
    const int ts = assemble_tile(F, 4);
    int64_t np = 0, nn = 0, nlb = 0, nat = 0, nrt = 0;
    for (int k = 0; k < nprob; ++k) {
        Mesh m;
        p2m_status s = check_problem(&probs[k], m);
        if (s != P2M_OK) return s;
        if (m.dim != 2 || probs[k].dtype != P2M_F32) return P2M_ERR_UNSUPPORTED;
        BatchInst& I = P.inst[k];
        memset(&I, 0, sizeof(I));
        I.m = m;
        I.P = particles_of<float>(&probs[k]);
        if (values) {
            if (m.np > 0 && !values[k]) return P2M_ERR_INVALID_ARG;
            I.values = (const float*)values[k];
        }
        if (outs) {
            if (!outs[k]) return P2M_ERR_INVALID_ARG;
            I.out = (float*)outs[k];
        }
        I.rep = reps ? reps + k : nullptr;
        const int atx = (m.nx + ts - 1) / ts, aty = (m.ny + ts - 1) / ts;
        const int rtx = (m.nx + kSolveTileX - 1) / kSolveTileX;
        const int rty = (m.ny + kSolveTileY - 1) / kSolveTileY;
        const int lbk = (m.np + kBinBlock - 1) / kBinBlock;
        I.po = (int32_t)np;
        I.no = (int32_t)nn;
        I.lb = (int32_t)nlb;
        I.at = (int32_t)nat;
        I.atx = atx;
        I.rt = (int32_t)nrt;
        I.rtx = rtx;
        I.nrt = rtx * rty;
        np += m.np;
        nn += m.nn;
        nlb += lbk;
        nat += (int64_t)atx * aty;
        nrt += (int64_t)rtx * rty;
        if (np >= ((int64_t)1 << 31) - 1 || nn >= ((int64_t)1 << 31) - 1 ||
            nat >= ((int64_t)1 << 31) - 1)
            return P2M_ERR_UNSUPPORTED;
    }
    P.np = np;
    P.nn = nn;
    P.nlb = (int)nlb;
    P.nat = (int)nat;
    P.nrt = (int)nrt;
    P.lmap.resize(P.nlb);
    P.amap.resize(P.nat);
    P.rmap.resize(P.nrt);
    for (int k = 0; k < nprob; ++k) {
        const BatchInst& I = P.inst[k];
        const int lbk = (I.m.np + kBinBlock - 1) / kBinBlock;
        const int ts2 = (I.m.ny + ts - 1) / ts;
        for (int b = 0; b < lbk; ++b) P.lmap[I.lb + b] = k;
        for (int t = 0; t < I.atx * ts2; ++t) P.amap[I.at + t] = k;
        for (int t = 0; t < I.nrt; ++t) P.rmap[I.rt + t] = k;
    }
    // Dealing order of the solver tiles (workgroup g owns the tiles at positions
    // g, g + grid, ...): instances with fewer particles per node first (they need
    // the most CG iterations, so their tiles should sit on distinct workgroups), then
    // instances with more tiles, then by index.  Ownership changes no arithmetic.
    {
        std::vector<int> ord(nprob);
        for (int k = 0; k < nprob; ++k) ord[k] = k;
        auto before = [&](int x, int y) {
            const BatchInst& X = P.inst[x];
            const BatchInst& Y = P.inst[y];
            const long long lx = (long long)X.m.np * Y.m.nn, ly = (long long)Y.m.np * X.m.nn;
            if (lx != ly) return lx < ly;
            if (X.nrt != Y.nrt) return X.nrt > Y.nrt;
            return x < y;
        };
        for (int i = 1; i < nprob; ++i)   // insertion sort: nprob <= 128, stable
            for (int j = i; j > 0 && before(ord[j], ord[j - 1]); --j) {
                const int t = ord[j];
                ord[j] = ord[j - 1];
                ord[j - 1] = t;
            }
        P.omap.clear();
        P.omap.reserve(P.nrt);
        for (int k : ord)
            for (int t = 0; t < P.inst[k].nrt; ++t) P.omap.push_back(P.inst[k].rt + t);
    }
    P.grid = cgb_grid(F, P.nrt, c->device);
    if (P.grid < 1) return P2M_ERR_UNSUPPORTED;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    P.inst_b = align_up(sizeof(BatchInst) * nprob);
    P.lmap_b = align_up(sizeof(int32_t) * P.nlb);
    P.amap_b = align_up(sizeof(int32_t) * P.nat);
    P.rmap_b = align_up(sizeof(int32_t) * P.nrt);
    P.omap_b = align_up(sizeof(int32_t) * P.nrt);
    take(P.inst_b + P.lmap_b + P.amap_b + P.rmap_b + P.omap_b);
    P.o_key = take(sizeof(int32_t) * 2 * (size_t)np);      // keys, then in-cell ranks
    P.o_counts = take(sizeof(int32_t) * (size_t)nn);
    P.o_scan = take(scan_workspace_bytes((int)nn));   // right after counts: one fill clears both
    P.o_cs = take(sizeof(int32_t) * ((size_t)nn + 1));
    P.o_perm = take(sizeof(int32_t) * (size_t)np);
    P.o_b = take(sizeof(float) * (size_t)F * nn);
    P.o_w = take(sizeof(float) * (size_t)nn);
    P.o_coef = take(sizeof(float) * (size_t)4 * nn);
    P.o_solve = take(cgb_workspace_bytes(F, nprob, P.nrt, (size_t)nn));
    P.total = off;
    return P2M_OK;
}

// The launch sequence of a batch on `stream` (captured into the batch graph).
hipError_t enqueue_batch(const BatchPlan& P, char* ws, p2m_report* reps, const p2m_solve_opts& opts,
                         long scan_spin, long solve_spin, hipStream_t stream) {
    const BatchInst* inst = (const BatchInst*)ws;
    const int32_t* lmap = (const int32_t*)(ws + P.inst_b);
    const int32_t* amap = (const int32_t*)(ws + P.inst_b + P.lmap_b);
    const int32_t* rmap = (const int32_t*)(ws + P.inst_b + P.lmap_b + P.amap_b);
    const int32_t* omap = (const int32_t*)(ws + P.inst_b + P.lmap_b + P.amap_b + P.rmap_b);
    int32_t* key = (int32_t*)(ws + P.o_key);
    int32_t* counts = (int32_t*)(ws + P.o_counts);
    int32_t* cs = (int32_t*)(ws + P.o_cs);
    int32_t* perm = (int32_t*)(ws + P.o_perm);
    void* scan_ws = ws + P.o_scan;
    const size_t clear = (P.o_scan + scan_workspace_bytes((int)P.nn) - P.o_counts) / sizeof(int32_t);
    float* b = (float*)(ws + P.o_b);
    float* w = (float*)(ws + P.o_w);
    float* coef = (float*)(ws + P.o_coef);
    hipError_t e;
    if ((e = launch_report_clear_n(reps, P.nprob, stream)) != hipSuccess) return e;
    if ((e = launch_fill_i32(counts, 0, clear, stream)) != hipSuccess) return e;
    if ((e = launch_locate_count_batch(inst, lmap, P.nlb, key, key + P.np, counts, stream)) !=
        hipSuccess)
        return e;
    if ((e = launch_exclusive_scan(counts, cs, (int)P.nn, scan_ws, scan_spin, reps, P.nprob,
                                   stream)) != hipSuccess)
        return e;
    if ((e = launch_place_flat((int)P.np, (int)P.nn, key, key + P.np, cs, perm, scan_ws, stream)) !=
        hipSuccess)
        return e;
    if ((e = launch_segment_sort_flat((int)P.nn, cs, perm, stream)) != hipSuccess) return e;
    if ((e = launch_assemble_batch(P.F, inst, amap, P.nat, perm, cs, b, w, coef, stream)) !=
        hipSuccess)
        return e;
    BatchSolveBufs bb;
    bb.inst = inst;
    bb.nprob = P.nprob;
    bb.rmap = rmap;
    bb.order = omap;
    bb.ntiles = P.nrt;
    bb.coef = coef;
    bb.b = b;
    bb.w = w;
    bb.ws = ws + P.o_solve;
    bb.spin = solve_spin;
    return launch_cg_batch(P.F, bb, (size_t)P.nn, P.grid, opts.start, opts, stream);
}

// ---------------------------------------------------------------------------
// paper-exact 1D (k_exact1d.hip)
// ---------------------------------------------------------------------------
struct X1DLayout {
    size_t key, counts, scan, cell_start, perm;          // binning (as in Layout)
    size_t skey, sidx, gap, vols, volc, As, fa, fb, tlo, thi, c, coef, w, x, b, bw;
    size_t r, p0, p1, q, x64, dinv, part, report, total;
    int blocks;
};

X1DLayout make_x1d_layout(const Context* c, const Mesh& m, int F) {
    X1DLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t np = (size_t)m.np, n = (size_t)m.nn, K = np > n ? np : n, d8 = sizeof(double);
    Mesh mk = m;
    mk.nn = (int)K;
    L.blocks = cg_blocks_for(c, mk, P2M_F64);
    L.key = take(2 * np * sizeof(int32_t));
    L.counts = take(n * sizeof(int32_t));
    L.scan = take(scan_workspace_bytes((int)n));   // right after counts: one fill clears both
    L.cell_start = take((n + 1) * sizeof(int32_t));
    L.perm = take(np * sizeof(int32_t));
    L.skey = take(np * d8);
    L.sidx = take(np * sizeof(int32_t));
    L.gap = take(np * d8);
    L.vols = take(np * d8);
    L.volc = take(np * d8);
    L.As = take((size_t)F * np * d8);
    L.fa = take((size_t)F * K * d8);
    L.fb = take((size_t)F * K * d8);
    L.tlo = take((size_t)F * K * d8);
    L.thi = take((size_t)F * K * d8);
    L.c = take((size_t)F * K * d8);
    L.coef = take(2 * K * d8);
    L.w = take(K * d8);
    L.x = take((size_t)F * K * d8);
    L.b = take((size_t)F * n * d8);
    L.bw = take(n * d8);
    L.r = take((size_t)F * K * d8);
    L.p0 = take((size_t)F * K * d8);
    L.p1 = take((size_t)F * K * d8);
    L.q = take((size_t)F * K * d8);
    L.x64 = take((size_t)2 * F * K * d8);
    L.dinv = take(K * d8);
    L.part = take(cg_partials_bytes(L.blocks));
    L.report = take(sizeof(p2m_report));
    L.total = off;
    return L;
}

// Validation, layout, binning and the located count N (one stream synchronisation).
p2m_status x1d_begin(void* ctx, const p2m_problem* prob, int F, void* ws, size_t ws_bytes,
                     void* stream, p2m_report* rep, Prepared& pp, X1DLayout& X, int& N) {
    if (!ctx || F < 1 || F > kMaxFields) return P2M_ERR_INVALID_ARG;
    Mesh m;
    p2m_status s = check_problem(prob, m);
    if (s != P2M_OK) return s;
    if (m.dim != 1 || prob->dtype != P2M_F64) return P2M_ERR_UNSUPPORTED;
    const Context* c = (const Context*)ctx;
    X = make_x1d_layout(c, m, F);
    if (!ws || ws_bytes < X.total || ((uintptr_t)ws) % kAlign) return P2M_ERR_WORKSPACE;
    pp.m = m;
    memset(&pp.L, 0, sizeof(pp.L));
    pp.L.key = X.key;
    pp.L.counts = X.counts;
    pp.L.scan = X.scan;
    pp.L.cell_start = X.cell_start;
    pp.L.perm = X.perm;
    pp.ws = (char*)ws;
    pp.stream = (hipStream_t)stream;
    pp.rep = rep ? rep : (p2m_report*)(pp.ws + X.report);
    pp.scan_spin = c->scan_spin;
    pp.solve_spin = c->solve_spin;
    pp.clear_rep = true;
    int32_t* perm = (int32_t*)(pp.ws + X.perm);
    int32_t* cs = (int32_t*)(pp.ws + X.cell_start);
    s = run_bin<double>(pp, prob, perm, cs);
    if (s != P2M_OK) return s;
    int32_t located = 0;
    P2M_TRY(hipMemcpyAsync(&located, cs + m.nn, sizeof(int32_t), hipMemcpyDeviceToHost, pp.stream));
    P2M_TRY(hipStreamSynchronize(pp.stream));
    N = located;
    P2M_TRY(x1d_sort(m, N, (const double*)prob->x, perm, cs, (double*)(pp.ws + X.skey),
                     (int32_t*)(pp.ws + X.sidx), pp.stream));
    return P2M_OK;
}

CgWorkspace x1d_cg_ws(const Prepared& pp, const X1DLayout& X, const Context* c, const Mesh& ms) {
    CgWorkspace cw;
    cw.r = pp.ws + X.r;
    cw.p0 = pp.ws + X.p0;
    cw.p1 = pp.ws + X.p1;
    cw.q = pp.ws + X.q;
    cw.x64 = (double*)(pp.ws + X.x64);
    cw.partials = (double*)(pp.ws + X.part);
    cw.dinv = pp.ws + X.dinv;
    cw.blocks = cg_blocks_for(c, ms, P2M_F64);
    cw.spin = pp.solve_spin;
    return cw;
}

p2m_solve_opts x1d_opts(const p2m_solve_opts* o, int n) {
    p2m_solve_opts r;
    if (o) {
        r = *o;
    } else {
        r.tol = 1e-14;
        r.maxit = 20 * n + 200;
        r.max_refine = 20;
    }
    r.inner_rtol = 0.0;
    r.start = P2M_START_FLIP;
    r.reserved = 0;
    return r;
}

// ---------------------------------------------------------------------------
// paper-exact 2D (k_x2d.hip)
// ---------------------------------------------------------------------------
struct X2DLayout {
    size_t key, counts, scan, cell_start, perm;          // binning (as in Layout)
    size_t xs, ys, cell, As, deg, nbr, nsh, vol, volc, H, b, bw, coef, ecol, w, x, fft;
    size_t r, p0, p1, q, x64, dinv, part, report, total;
    int blocks;
};

X2DLayout make_x2d_layout(const Context* c, const Mesh& m, int F) {
    X2DLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t np = (size_t)m.np, n = (size_t)m.nn, K = np > n ? np : n, d8 = sizeof(double);
    const size_t cap = P2M_X2D_MAXDEG, i4 = sizeof(int32_t);
    Mesh mk = m;
    mk.nn = (int)K;
    L.blocks = cg_blocks_for(c, mk, P2M_F64);
    L.key = take(2 * np * i4);
    L.counts = take(n * i4);
    L.scan = take(scan_workspace_bytes((int)n));   // right after counts: one fill clears both
    L.cell_start = take((n + 1) * i4);
    L.perm = take(np * i4);
    L.xs = take(np * d8);
    L.ys = take(np * d8);
    L.cell = take(np * i4);
    L.As = take((size_t)F * np * d8);
    L.deg = take(np * i4);
    L.nbr = take(np * cap * i4);
    L.nsh = take(np * cap * i4);
    L.vol = take(np * d8);
    L.volc = take(np * d8);
    L.H = take((size_t)F * 4 * n * d8);
    L.b = take((size_t)F * K * d8);
    L.bw = take(n * d8);
    const size_t cm = 4 * n > (1 + cap) * np ? 4 * n : (1 + cap) * np;
    L.coef = take(cm * d8);
    L.ecol = take(cap * np * i4);
    L.w = take(K * d8);
    L.x = take((size_t)F * K * d8);
    L.fft = take(fft_supported(m) ? fft_workspace_bytes(m, F) : 0);
    L.r = take((size_t)F * K * d8);
    L.p0 = take((size_t)F * K * d8);
    L.p1 = take((size_t)F * K * d8);
    L.q = take((size_t)F * K * d8);
    L.x64 = take((size_t)2 * F * K * d8);
    L.dinv = take(K * d8);
    L.part = take(cg_partials_bytes(L.blocks));
    L.report = take(sizeof(p2m_report));
    L.total = off;
    return L;
}

p2m_status x2d_check(void* ctx, const p2m_problem* prob, int F, Mesh& m) {
    if (!ctx || F < 1 || F > kMaxFields) return P2M_ERR_INVALID_ARG;
    p2m_status s = check_problem(prob, m);
    if (s != P2M_OK) return s;
    if (m.dim != 2 || prob->dtype != P2M_F64) return P2M_ERR_UNSUPPORTED;
    return P2M_OK;
}

// Validation, layout, binning, the located count N (one stream synchronisation)
// and the triangulation; values (may be null) are gathered into binned order.
p2m_status x2d_begin(void* ctx, const p2m_problem* prob, int F, const void* values, void* ws,
                     size_t ws_bytes, void* stream, p2m_report* rep, Prepared& pp, X2DLayout& X,
                     X2dArgs& A) {
    Mesh m;
    p2m_status s = x2d_check(ctx, prob, F, m);
    if (s != P2M_OK) return s;
    const Context* c = (const Context*)ctx;
    X = make_x2d_layout(c, m, F);
    if (!ws || ws_bytes < X.total || ((uintptr_t)ws) % kAlign) return P2M_ERR_WORKSPACE;
    pp.m = m;
    memset(&pp.L, 0, sizeof(pp.L));
    pp.L.key = X.key;
    pp.L.counts = X.counts;
    pp.L.scan = X.scan;
    pp.L.cell_start = X.cell_start;
    pp.L.perm = X.perm;
    pp.ws = (char*)ws;
    pp.stream = (hipStream_t)stream;
    pp.rep = rep ? rep : (p2m_report*)(pp.ws + X.report);
    pp.scan_spin = c->scan_spin;
    pp.solve_spin = c->solve_spin;
    pp.clear_rep = true;
    int32_t* perm = (int32_t*)(pp.ws + X.perm);
    int32_t* cs = (int32_t*)(pp.ws + X.cell_start);
    s = run_bin<double>(pp, prob, perm, cs);
    if (s != P2M_OK) return s;
    int32_t located = 0;
    P2M_TRY(hipMemcpyAsync(&located, cs + m.nn, sizeof(int32_t), hipMemcpyDeviceToHost, pp.stream));
    P2M_TRY(hipStreamSynchronize(pp.stream));
    char* w8 = pp.ws;
    A.m = m;
    A.N = located;
    A.F = F;
    A.lx = prob->lx;
    A.ly = prob->ly;
    A.perm = perm;
    A.cs = cs;
    A.x = (const double*)prob->x;
    A.y = (const double*)prob->y;
    A.values = (const double*)values;
    A.xs = (double*)(w8 + X.xs);
    A.ys = (double*)(w8 + X.ys);
    A.cell = (int32_t*)(w8 + X.cell);
    A.As = (double*)(w8 + X.As);
    A.deg = (int32_t*)(w8 + X.deg);
    A.nbr = (int32_t*)(w8 + X.nbr);
    A.nsh = (int32_t*)(w8 + X.nsh);
    A.vol = (double*)(w8 + X.vol);
    A.rep = pp.rep;
    P2M_TRY(x2d_triangulate(A, pp.stream));
    return P2M_OK;
}

CgWorkspace x2d_cg_ws(const Prepared& pp, const X2DLayout& X, const Context* c, const Mesh& ms) {
    CgWorkspace cw;
    cw.r = pp.ws + X.r;
    cw.p0 = pp.ws + X.p0;
    cw.p1 = pp.ws + X.p1;
    cw.q = pp.ws + X.q;
    cw.x64 = (double*)(pp.ws + X.x64);
    cw.partials = (double*)(pp.ws + X.part);
    cw.dinv = pp.ws + X.dinv;
    cw.blocks = cg_blocks_for(c, ms, P2M_F64);
    cw.spin = pp.solve_spin;
    return cw;
}

p2m_status x2d_check_p2m(const p2m_problem* prob, int32_t kind, const void* values,
                         const p2m_solve_opts* opts) {
    if (kind < P2M_X1D_DELTA || kind > P2M_X1D_LUMPED) return P2M_ERR_INVALID_ARG;
    if (opts && kind == P2M_X1D_MASS) {
        p2m_status so = check_opts(opts);
        if (so != P2M_OK) return so;
    }
    if (!prob || (prob->np > 0 && !values)) return P2M_ERR_INVALID_ARG;
    return P2M_OK;
}

p2m_status x2d_check_m2p(int32_t kind, const p2m_solve_opts* opts) {
    if (kind != P2M_X1D_DELTA && kind != P2M_X1D_MASS && kind != P2M_X1D_LUMPED)
        return P2M_ERR_INVALID_ARG;
    if (opts && kind == P2M_X1D_MASS) {
        p2m_status so = check_opts(opts);
        if (so != P2M_OK) return so;
    }
    return P2M_OK;
}

// P2M of one kind after x2d_begin; the mass solve reports to rep
p2m_status x2d_run_p2m(const Context* c, const Prepared& pp, const X2DLayout& X, const X2dArgs& A,
                       const p2m_problem* prob, int32_t kind, const void* values,
                       const p2m_solve_opts* opts, double* out, p2m_report* rep) {
    const Mesh& m = pp.m;
    const int F = A.F;
    char* w8 = pp.ws;
    if (kind == P2M_X1D_FLIP || kind == P2M_X1D_PIC) {
        double* volc = (double*)(w8 + X.volc);
        P2M_TRY(x1d_scatter(A.N, 1, m.np, A.perm, A.vol, volc, pp.stream));
        Particles<double> P = particles_of<double>(prob);
        P.vol = volc;
        double* b = (double*)(w8 + X.b);
        double* bw = (double*)(w8 + X.bw);
        P2M_TRY(launch_assemble<double>(m, P, (const double*)values, F, A.perm, A.cs, b, bw,
                                        nullptr, pp.stream));
        P2M_TRY(launch_finalize<double>(m, F, b, bw, kind == P2M_X1D_PIC ? 1 : 0, out, rep,
                                        pp.stream));
        return P2M_OK;
    }
    if (kind == P2M_X1D_DELTA) {
        P2M_TRY(x2d_locate(A, false, out, pp.stream));
        return P2M_OK;
    }
    double* H = (double*)(w8 + X.H);
    double* b = (double*)(w8 + X.b);
    P2M_TRY(x2d_locate(A, true, H, pp.stream));
    P2M_TRY(x2d_rhs_mesh(A, H, b, pp.stream));
    if (kind == P2M_X1D_LUMPED) {
        P2M_TRY(x1d_div(m.nn, F, b, nullptr, m.cell_measure, out, pp.stream));
        return P2M_OK;
    }
    if (c->fft && fft_supported(m)) {   // circulant: a direct FP64 solve by the 2D DFT
        P2M_TRY(launch_fft_solve<double>(m, F, m.cell_measure, kFftMass, b, out, w8 + X.fft,
                                         pp.stream));
        return P2M_OK;
    }
    double* coef = (double*)(w8 + X.coef);
    double* wv = (double*)(w8 + X.w);
    P2M_TRY(x2d_mass_mesh(A, coef, wv, pp.stream));
    const p2m_solve_opts o = x1d_opts(opts, m.nn);
    P2M_TRY(launch_cg<double>(m, F, coef, b, wv, out, P2M_START_FLIP, x2d_cg_ws(pp, X, c, m), o,
                              rep, pp.stream));
    return P2M_OK;
}

// M2P of kind MASS or LUMPED after x2d_begin; the mass solve reports to rep
p2m_status x2d_run_m2p(const Context* c, const Prepared& pp, const X2DLayout& X, const X2dArgs& A,
                       int32_t kind, const double* nodal, const p2m_solve_opts* opts,
                       double* values_out, p2m_report* rep) {
    const Mesh& m = pp.m;
    const int F = A.F, N = A.N;
    char* w8 = pp.ws;
    double* cvec = (double*)(w8 + X.b);
    double* xs = (double*)(w8 + X.x);
    P2M_TRY(x2d_rhs_part(A, nodal, cvec, pp.stream));
    if (kind == P2M_X1D_LUMPED) {
        P2M_TRY(x1d_div(N, F, cvec, A.vol, 0.0, xs, pp.stream));
    } else if (N > 0) {
        double* coef = (double*)(w8 + X.coef);
        int32_t* ecol = (int32_t*)(w8 + X.ecol);
        P2M_TRY(x2d_mass_part(A, coef, ecol, pp.stream));
        Mesh mp;
        memset(&mp, 0, sizeof(mp));
        mp.dim = 3;
        mp.nx = N;
        mp.ny = 1;
        mp.nn = N;
        mp.inv_hx = mp.inv_hy = 1.0;
        mp.cell_measure = 1.0;
        CgWorkspace cw = x2d_cg_ws(pp, X, c, mp);
        cw.ell_col = ecol;
        cw.ell_w = P2M_X2D_MAXDEG;
        const p2m_solve_opts o = x1d_opts(opts, N);
        P2M_TRY(launch_cg<double>(mp, F, coef, cvec, A.vol, xs, P2M_START_FLIP, cw, o, rep,
                                  pp.stream));
    }
    P2M_TRY(x1d_scatter(N, F, m.np, A.perm, xs, values_out, pp.stream));
    return P2M_OK;
}


}  // namespace

extern "C" {

const char* p2m_status_string(p2m_status s) {
    switch (s) {
        case P2M_OK: return "P2M_OK";
        case P2M_ERR_INVALID_ARG: return "P2M_ERR_INVALID_ARG";
        case P2M_ERR_UNSUPPORTED: return "P2M_ERR_UNSUPPORTED";
        case P2M_ERR_WORKSPACE: return "P2M_ERR_WORKSPACE";
        case P2M_ERR_RANGE: return "P2M_ERR_RANGE";
        case P2M_ERR_NONFINITE: return "P2M_ERR_NONFINITE";
        case P2M_ERR_HIP: return "P2M_ERR_HIP";
        case P2M_ERR_SCRATCH: return "P2M_ERR_SCRATCH";
    }
    return "P2M_UNKNOWN_STATUS";
}

p2m_status p2m_create(void** ctx, int device) {
    if (!ctx) return P2M_ERR_INVALID_ARG;
    *ctx = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) return P2M_ERR_HIP;
    if (device < 0 || device >= count) return P2M_ERR_INVALID_ARG;
    DeviceGuard g(device);
    if (!g.ok) return P2M_ERR_HIP;
    Context* c = (Context*)calloc(1, sizeof(Context));
    if (!c) return P2M_ERR_HIP;
    c->device = device;
    c->cg_blocks_f32 = cg_max_blocks<float>(device);
    c->cg_blocks_f64 = cg_max_blocks<double>(device);
    c->solver_mode = P2M_SOLVER_AUTO;
    c->use_plans = 1;
    c->scan_spin = kScanSpinDefault;
    c->solve_spin = kSolveSpinDefault;
    c->fft = 1;
    c->scratch = scratch_address(device);
    if (c->cg_blocks_f32 <= 0 || c->cg_blocks_f64 <= 0) {
        free(c);
        return P2M_ERR_HIP;
    }
    *ctx = c;
    return P2M_OK;
}

p2m_status p2m_set_option(void* ctx, int32_t option, int32_t value) {
    if (!ctx) return P2M_ERR_INVALID_ARG;
    Context* c = (Context*)ctx;
    if (option == P2M_OPT_SOLVER) {
        if (value < P2M_SOLVER_AUTO || value > P2M_SOLVER_RESIDENT_CHEB) return P2M_ERR_INVALID_ARG;
        c->solver_mode = value;
        return P2M_OK;
    }
    if (option == P2M_OPT_PLANS) {
        if (value != 0 && value != 1) return P2M_ERR_INVALID_ARG;
        c->use_plans = value;
        return P2M_OK;
    }
    if (option == P2M_OPT_SCAN_SPIN) {
        c->scan_spin = value == 0 ? kScanSpinDefault : (long)value;
        return P2M_OK;
    }
    if (option == P2M_OPT_SOLVE_SPIN) {
        c->solve_spin = value == 0 ? kSolveSpinDefault : (long)value;
        return P2M_OK;
    }
    if (option == P2M_OPT_FFT) {
        if (value != 0 && value != 1) return P2M_ERR_INVALID_ARG;
        c->fft = value;
        return P2M_OK;
    }
    return P2M_ERR_INVALID_ARG;
}

p2m_status p2m_destroy(void* ctx) {
    if (ctx) {
        Context* c = (Context*)ctx;
        if (c->batch) {
            DeviceGuard g(c->device);
            delete c->batch;
        }
        delete c->plans;
    }
    free(ctx);
    return P2M_OK;
}

p2m_status p2m_workspace_size(void* ctx, const p2m_problem* prob, int32_t nfields, size_t* bytes) {
    if (!ctx || !bytes) return P2M_ERR_INVALID_ARG;
    if (nfields < 1 || nfields > kMaxFields) return P2M_ERR_INVALID_ARG;
    Mesh m;
    p2m_status s = check_problem(prob, m);
    if (s != P2M_OK) return s;
    const Context* c = (const Context*)ctx;
    *bytes = make_layout(m, nfields, tsize_of(prob), cg_blocks_for(c, m, prob->dtype)).total;
    return P2M_OK;
}

p2m_status p2m_bin(void* ctx, const p2m_problem* prob, int32_t* perm, int32_t* cell_start,
                   p2m_report* rep, void* ws, size_t ws_bytes, void* stream) {
    Prepared pp;
    p2m_status s = prepare(ctx, prob, 1, ws, ws_bytes, stream, rep, pp);
    if (s != P2M_OK) return s;
    if ((pp.m.np > 0 && !perm) || !cell_start) return P2M_ERR_INVALID_ARG;
    DeviceGuard g(((Context*)ctx)->device);
    if (!g.ok) return P2M_ERR_HIP;
    pp.clear_rep = true;   // zeroed by the call's first launch
    return prob->dtype == P2M_F64 ? run_bin<double>(pp, prob, perm, cell_start)
                                  : run_bin<float>(pp, prob, perm, cell_start);
}

p2m_status p2m_assemble(void* ctx, const p2m_problem* prob, const void* values, int32_t nfields,
                        void* b, void* w, void* coef, p2m_report* rep, void* ws, size_t ws_bytes,
                        void* stream) {
    Prepared pp;
    p2m_status s = prepare(ctx, prob, nfields, ws, ws_bytes, stream, rep, pp);
    if (s != P2M_OK) return s;
    if ((pp.m.np > 0 && !values) || !b || !w) return P2M_ERR_INVALID_ARG;
    DeviceGuard g(((Context*)ctx)->device);
    if (!g.ok) return P2M_ERR_HIP;
    pp.clear_rep = true;   // zeroed by the call's first launch
    const Choice ch = choose((const Context*)ctx, pp.m, prob->dtype, nfields);
    return prob->dtype == P2M_F64 ? run_assemble<double>(pp, prob, values, nfields, b, w, coef, ch)
                                  : run_assemble<float>(pp, prob, values, nfields, b, w, coef, ch);
}

p2m_status p2m_assign(void* ctx, const p2m_problem* prob, p2m_assign_kind kind, const void* values,
                      int32_t nfields, void* nodal_out, p2m_report* rep, void* ws, size_t ws_bytes,
                      void* stream) {
    if (kind != P2M_DELTA && kind != P2M_FLIP && kind != P2M_PIC) return P2M_ERR_INVALID_ARG;
    Prepared pp;
    p2m_status s = prepare(ctx, prob, nfields, ws, ws_bytes, stream, rep, pp);
    if (s != P2M_OK) return s;
    if (kind == P2M_DELTA && pp.m.dim != 1) return P2M_ERR_UNSUPPORTED;
    if ((pp.m.np > 0 && !values) || !nodal_out) return P2M_ERR_INVALID_ARG;
    DeviceGuard g(((Context*)ctx)->device);
    if (!g.ok) return P2M_ERR_HIP;
    pp.clear_rep = true;   // zeroed by the call's first launch
    return prob->dtype == P2M_F64 ? run_assign<double>(pp, prob, kind, values, nfields, nodal_out)
                                  : run_assign<float>(pp, prob, kind, values, nfields, nodal_out);
}

p2m_status p2m_interpolate(void* ctx, const p2m_problem* prob, const void* nodal, int32_t nfields,
                           void* values_out, p2m_report* rep, void* ws, size_t ws_bytes,
                           void* stream) {
    if (!ctx) return P2M_ERR_INVALID_ARG;
    if (nfields < 1 || nfields > kMaxFields) return P2M_ERR_INVALID_ARG;
    Mesh m;
    p2m_status s = check_problem(prob, m);
    if (s != P2M_OK) return s;
    if (!nodal || (m.np > 0 && !values_out)) return P2M_ERR_INVALID_ARG;
    DeviceGuard g(((Context*)ctx)->device);
    if (!g.ok) return P2M_ERR_HIP;
    hipStream_t strm = (hipStream_t)stream;
    P2M_TRY(launch_report_clear(rep, strm));
    if (prob->dtype == P2M_F64)
        return st(launch_gather<double>(m, particles_of<double>(prob), (const double*)nodal, nfields,
                                        (double*)values_out, rep, strm, ws, ws ? ws_bytes : 0));
    return st(launch_gather<float>(m, particles_of<float>(prob), (const float*)nodal, nfields,
                                   (float*)values_out, rep, strm, ws, ws ? ws_bytes : 0));
}

p2m_status p2m_mass_assign(void* ctx, const p2m_problem* prob, const void* values, int32_t nfields,
                           const p2m_solve_opts* opts, void* nodal_inout, p2m_report* rep,
                           void* ws, size_t ws_bytes, void* stream) {
    if (!rep) return P2M_ERR_INVALID_ARG;
    p2m_status s = check_opts(opts);
    if (s != P2M_OK) return s;
    Prepared pp;
    s = prepare(ctx, prob, nfields, ws, ws_bytes, stream, rep, pp);
    if (s != P2M_OK) return s;
    if (opts->start == P2M_START_DELTA1D && pp.m.dim != 1) return P2M_ERR_UNSUPPORTED;
    if (opts->start == P2M_START_LEARNED &&
        (pp.m.dim != 2 || prob->dtype != P2M_F32 || !((const Context*)ctx)->learned))
        return P2M_ERR_UNSUPPORTED;
    if ((pp.m.np > 0 && !values) || !nodal_inout) return P2M_ERR_INVALID_ARG;
    DeviceGuard g(((Context*)ctx)->device);
    if (!g.ok) return P2M_ERR_HIP;
    pp.clear_rep = true;   // zeroed by the call's first launch
    const Context* c = (const Context*)ctx;
    const Choice ch = choose(c, pp.m, prob->dtype, nfields);
    return prob->dtype == P2M_F64
               ? run_mass<double>(c, pp, prob, values, nfields, *opts, nodal_inout, ch)
               : run_mass<float>(c, pp, prob, values, nfields, *opts, nodal_inout, ch);
}

p2m_status p2m_mass_assign_noalloc(void* ctx, const p2m_problem* prob, const void* values,
                                   int32_t nfields, const p2m_solve_opts* opts, void* nodal_inout,
                                   p2m_report* rep, void* stream) {
    if (!ctx) return P2M_ERR_INVALID_ARG;
    size_t need = 0;
    p2m_status s = p2m_workspace_size(ctx, prob, nfields, &need);
    if (s != P2M_OK) return s;
    if (need > kScratchBytes) return P2M_ERR_SCRATCH;
    void* ws = ((const Context*)ctx)->scratch;
    if (!ws) return P2M_ERR_HIP;
    return p2m_mass_assign(ctx, prob, values, nfields, opts, nodal_inout, rep, ws, kScratchBytes,
                           stream);
}

// ---------------------------------------------------------------------------
// particle fluid solver (Sec. 3.3): one time step
// ---------------------------------------------------------------------------
// The step's arrays after the F = 2 layout of the problem: Ubar, U*, U^{n+1} [2][nn],
// the viscous and pressure stencils [4][nn] with their diagonals [nn], the pressure
// right-hand side and the pressure [nn], and (power-of-two sides) the transform
// buffers of the direct solves.
struct NsLayout {
    size_t ubar, ustar, unew, cv, wv, cp, wp, rhs, p, fft, total;
};

NsLayout make_ns_layout(size_t base, const Mesh& m) {
    NsLayout N;
    size_t off = base;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    const size_t nn = (size_t)m.nn;
    N.ubar = take(2 * nn * sizeof(float));
    N.ustar = take(2 * nn * sizeof(float));
    N.unew = take(2 * nn * sizeof(float));
    N.cv = take(4 * nn * sizeof(float));
    N.wv = take(nn * sizeof(float));
    N.cp = take(4 * nn * sizeof(float));
    N.wp = take(nn * sizeof(float));
    N.rhs = take(nn * sizeof(float));
    N.p = take(nn * sizeof(float));
    N.fft = take(fft_supported(m) ? fft_workspace_bytes(m, 2) : 0);
    N.total = off;
    return N;
}

p2m_status check_ns_problem(const p2m_problem* prob, Mesh& m) {
    p2m_status s = check_problem(prob, m);
    if (s != P2M_OK) return s;
    if (m.dim != 2 || prob->dtype != P2M_F32) return P2M_ERR_UNSUPPORTED;
    const double hx = prob->lx / prob->nx, hy = prob->ly / prob->ny;
    if (fabs(hx - hy) > 1e-12 * hx) return P2M_ERR_UNSUPPORTED;   // square cells only
    return P2M_OK;
}

p2m_status p2m_ns_workspace_size(void* ctx, const p2m_problem* prob, size_t* bytes) {
    if (!ctx || !bytes) return P2M_ERR_INVALID_ARG;
    Mesh m;
    p2m_status s = check_ns_problem(prob, m);
    if (s != P2M_OK) return s;
    const Context* c = (const Context*)ctx;
    const Layout L = make_layout(m, 2, sizeof(float), cg_blocks_for(c, m, P2M_F32));
    *bytes = make_ns_layout(L.total, m).total;
    return P2M_OK;
}

p2m_status p2m_ns_step(void* ctx, const p2m_problem* prob, int32_t assign, double dt, double nu,
                       const p2m_solve_opts* opts, void* vel, void* x_out, void* y_out,
                       void* mesh_vel, p2m_report* reps, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || !reps) return P2M_ERR_INVALID_ARG;
    if (assign != P2M_NS_FLIP && assign != P2M_NS_MASS) return P2M_ERR_INVALID_ARG;
    if (!isfinite(dt) || !isfinite(nu)) return P2M_ERR_NONFINITE;
    if (!(dt > 0.0) || !(nu >= 0.0)) return P2M_ERR_RANGE;
    p2m_status s = check_opts(opts);
    if (s != P2M_OK) return s;
    if (opts->start != P2M_START_FLIP && opts->start != P2M_START_ZERO) return P2M_ERR_UNSUPPORTED;
    Mesh m;
    s = check_ns_problem(prob, m);
    if (s != P2M_OK) return s;
    if (m.np > 0 && (!vel || !x_out || !y_out)) return P2M_ERR_INVALID_ARG;
    size_t need = 0;
    s = p2m_ns_workspace_size(ctx, prob, &need);
    if (s != P2M_OK) return s;
    if (!ws || ws_bytes < need) return P2M_ERR_WORKSPACE;
    Prepared pp;
    s = prepare(ctx, prob, 2, ws, ws_bytes, stream, &reps[0], pp);
    if (s != P2M_OK) return s;
    const NsLayout N = make_ns_layout(pp.L.total, m);
    DeviceGuard g(((Context*)ctx)->device);
    if (!g.ok) return P2M_ERR_HIP;
    const Context* c = (const Context*)ctx;
    char* w = pp.ws;
    float* ubar = (float*)(w + N.ubar);
    float* ustar = (float*)(w + N.ustar);
    float* unew = mesh_vel ? (float*)mesh_vel : (float*)(w + N.unew);
    float* cv = (float*)(w + N.cv);
    float* wv = (float*)(w + N.wv);
    float* cpr = (float*)(w + N.cp);
    float* wpr = (float*)(w + N.wp);
    float* rhs = (float*)(w + N.rhs);
    float* pr = (float*)(w + N.p);
    const double h = prob->lx / prob->nx;
    // 1. P2M of the particle velocities (report 0: binning, assignment and its solve)
    pp.clear_rep = true;
    if (assign == P2M_NS_FLIP) {
        s = run_assign<float>(pp, prob, P2M_FLIP, vel, 2, ubar);
    } else {
        p2m_solve_opts o = *opts;
        s = run_mass<float>(c, pp, prob, vel, 2, o, ubar, choose(c, m, P2M_F32, 2));
    }
    if (s != P2M_OK) return s;
    // 2. viscous step (I + s K) U* = Ubar (report 1); 3. pressure K p = -(1/dt) D U*
    //    (report 2).  Sides the FFT takes (P2M_OPT_FFT on): both by 2D FFT, exactly
    //    (zero-mean pressure; the reports show no iteration).  Otherwise by the
    //    mass-matrix solver, node 0 holding the pressure at 0; a Poisson system needs
    //    O(n) CG iterations, so the pressure solve's cap is at least 64 per mesh side.
    const double sv = dt * nu / (h * h);
    if (c->fft && fft_supported(m)) {
        P2M_TRY(launch_report_clear(&reps[1], pp.stream));
        P2M_TRY(launch_report_clear(&reps[2], pp.stream));
        P2M_TRY(launch_ns_fft_solve(m, 2, sv, 0, ubar, ustar, w + N.fft, pp.stream));
        P2M_TRY(launch_ns_div(m, -(h / 6.0) / dt, 0, ustar, rhs, pp.stream));
        P2M_TRY(launch_ns_fft_solve(m, 1, 0.0, 1, rhs, pr, w + N.fft, pp.stream));
    } else {
        P2M_TRY(launch_ns_coef(m, (float)sv, cv, wv, cpr, wpr, pp.stream));
        Prepared pv = pp;
        pv.rep = &reps[1];
        pv.clear_rep = true;
        p2m_solve_opts ov = *opts;
        ov.start = P2M_START_FLIP;
        s = run_solve<float>(c, pv, 2, ubar, wv, cv, P2M_START_FLIP, ov, ustar,
                             choose(c, m, P2M_F32, 2));
        if (s != P2M_OK) return s;
        P2M_TRY(launch_ns_div(m, -(h / 6.0) / dt, 1, ustar, rhs, pp.stream));
        Prepared pq = pp;
        pq.rep = &reps[2];
        pq.clear_rep = true;
        p2m_solve_opts op = *opts;
        op.start = P2M_START_FLIP;
        const int64_t cap = 64 * (int64_t)(m.nx > m.ny ? m.nx : m.ny);
        if (op.maxit < cap) op.maxit = (int32_t)(cap < INT32_MAX ? cap : INT32_MAX);
        s = run_solve<float>(c, pq, 1, rhs, wpr, cpr, P2M_START_FLIP, op, pr,
                             choose(c, m, P2M_F32, 1));
        if (s != P2M_OK) return s;
    }
    // 4. projection U^{n+1} = U* - dt M_L^-1 G p
    P2M_TRY(launch_ns_correct(m, dt / (6.0 * h), ustar, pr, unew, pp.stream));
    // 5. M2P: the particles' new velocities (invalid particles flagged in report 0)
    P2M_TRY(launch_gather<float>(m, particles_of<float>(prob), unew, 2, (float*)vel, &reps[0],
                                 pp.stream, nullptr, 0));
    // 6. mid-point advection
    P2M_TRY(launch_ns_advect(m, prob->lx, prob->ly, dt, (const float*)prob->x,
                             (const float*)prob->y, (const float*)vel, unew, (float*)x_out,
                             (float*)y_out, &reps[0], pp.stream));
    return P2M_OK;
}

p2m_status p2m_x1d_workspace_size(void* ctx, const p2m_problem* prob, int32_t nfields,
                                  size_t* bytes) {
    if (!ctx || !bytes || nfields < 1 || nfields > kMaxFields) return P2M_ERR_INVALID_ARG;
    Mesh m;
    p2m_status s = check_problem(prob, m);
    if (s != P2M_OK) return s;
    if (m.dim != 1 || prob->dtype != P2M_F64) return P2M_ERR_UNSUPPORTED;
    *bytes = make_x1d_layout((const Context*)ctx, m, nfields).total;
    return P2M_OK;
}

p2m_status p2m_x1d_assign(void* ctx, const p2m_problem* prob, int32_t kind, int32_t quad,
                          const void* values, int32_t nfields, const p2m_solve_opts* opts,
                          void* nodal_out, p2m_report* rep, void* ws, size_t ws_bytes,
                          void* stream) {
    if (!rep || !nodal_out) return P2M_ERR_INVALID_ARG;
    if (kind < P2M_X1D_DELTA || kind > P2M_X1D_LUMPED) return P2M_ERR_INVALID_ARG;
    if (quad != P2M_QUAD_EXACT && quad != P2M_QUAD_APPB) return P2M_ERR_INVALID_ARG;
    if (opts && kind == P2M_X1D_MASS) {
        p2m_status so = check_opts(opts);
        if (so != P2M_OK) return so;
    }
    if (!prob || (prob->np > 0 && !values)) return P2M_ERR_INVALID_ARG;
    if (!ctx) return P2M_ERR_INVALID_ARG;
    const Context* c = (const Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return P2M_ERR_HIP;
    Prepared pp;
    X1DLayout X;
    int N = 0;
    p2m_status s = x1d_begin(ctx, prob, nfields, ws, ws_bytes, stream, rep, pp, X, N);
    if (s != P2M_OK) return s;
    const Mesh& m = pp.m;
    const int F = nfields, n = m.nx;
    const double h = m.cell_measure, L = h * n;
    char* w8 = pp.ws;
    double* out = (double*)nodal_out;
    const double* key = (const double*)(w8 + X.skey);
    const int32_t* idx = (const int32_t*)(w8 + X.sidx);
    double* volc = (double*)(w8 + X.volc);
    P2M_TRY(x1d_setup(N, L, key, idx, (const double*)values, F, m.np, (double*)(w8 + X.gap),
                      (double*)(w8 + X.vols), volc, (double*)(w8 + X.As), pp.stream));
    if (kind == P2M_X1D_FLIP || kind == P2M_X1D_PIC) {
        Particles<double> P = particles_of<double>(prob);
        P.vol = volc;
        double* b = (double*)(w8 + X.b);
        double* bw = (double*)(w8 + X.bw);
        P2M_TRY(launch_assemble<double>(m, P, (const double*)values, F,
                                        (const int32_t*)(w8 + X.perm),
                                        (const int32_t*)(w8 + X.cell_start), b, bw, nullptr,
                                        pp.stream));
        P2M_TRY(launch_finalize<double>(m, F, b, bw, kind == P2M_X1D_PIC ? 1 : 0, out, pp.rep,
                                        pp.stream));
        return P2M_OK;
    }
    const double* As = (const double*)(w8 + X.As);
    double* cvec = (double*)(w8 + X.c);
    // the particle interpolant at the nodes (the delta P2M) goes to nodal_out or fa
    double* fn = kind == P2M_X1D_DELTA ? out : (double*)(w8 + X.fa);
    P2M_TRY(x1d_p2m_overlap(m, N, key, As, F, kind == P2M_X1D_DELTA ? P2M_QUAD_APPB : quad, fn,
                            (double*)(w8 + X.fb), (double*)(w8 + X.tlo), (double*)(w8 + X.thi),
                            cvec, pp.stream));
    if (kind == P2M_X1D_DELTA) return P2M_OK;
    if (kind == P2M_X1D_LUMPED) {
        P2M_TRY(x1d_div(n, F, cvec, nullptr, h, out, pp.stream));
        return P2M_OK;
    }
    double* coef = (double*)(w8 + X.coef);
    double* wv = (double*)(w8 + X.w);
    P2M_TRY(x1d_mass_mesh(n, L, coef, wv, pp.stream));
    const p2m_solve_opts o = x1d_opts(opts, n);
    P2M_TRY(launch_cg<double>(m, F, coef, cvec, wv, out, P2M_START_FLIP, x1d_cg_ws(pp, X, c, m), o,
                              pp.rep, pp.stream));
    return P2M_OK;
}

p2m_status p2m_x1d_interpolate(void* ctx, const p2m_problem* prob, int32_t kind, int32_t quad,
                               const void* nodal, int32_t nfields, const p2m_solve_opts* opts,
                               void* values_out, p2m_report* rep, void* ws, size_t ws_bytes,
                               void* stream) {
    if (!rep || !nodal || !values_out || !ctx) return P2M_ERR_INVALID_ARG;
    if (kind != P2M_X1D_DELTA && kind != P2M_X1D_MASS && kind != P2M_X1D_LUMPED)
        return P2M_ERR_INVALID_ARG;
    if (quad != P2M_QUAD_EXACT && quad != P2M_QUAD_APPB) return P2M_ERR_INVALID_ARG;
    if (opts && kind == P2M_X1D_MASS) {
        p2m_status so = check_opts(opts);
        if (so != P2M_OK) return so;
    }
    const Context* c = (const Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return P2M_ERR_HIP;
    if (kind == P2M_X1D_DELTA) {
        Prepared pp;
        p2m_status s = prepare(ctx, prob, nfields, ws, ws_bytes, stream, rep, pp);
        if (s != P2M_OK && s != P2M_ERR_WORKSPACE) return s;
        if (s == P2M_ERR_WORKSPACE) {   // the gather needs none
            s = check_problem(prob, pp.m);
            if (s != P2M_OK) return s;
        }
        if (pp.m.dim != 1 || prob->dtype != P2M_F64) return P2M_ERR_UNSUPPORTED;
        P2M_TRY(launch_report_clear(rep, (hipStream_t)stream));
        P2M_TRY(launch_gather<double>(pp.m, particles_of<double>(prob), (const double*)nodal,
                                      nfields, (double*)values_out, rep, (hipStream_t)stream));
        return P2M_OK;
    }
    Prepared pp;
    X1DLayout X;
    int N = 0;
    p2m_status s = x1d_begin(ctx, prob, nfields, ws, ws_bytes, stream, rep, pp, X, N);
    if (s != P2M_OK) return s;
    const Mesh& m = pp.m;
    const int F = nfields, n = m.nx;
    const double h = m.cell_measure, L = h * n;
    char* w8 = pp.ws;
    const double* key = (const double*)(w8 + X.skey);
    const int32_t* idx = (const int32_t*)(w8 + X.sidx);
    const double* gap = (const double*)(w8 + X.gap);
    double* vols = (double*)(w8 + X.vols);
    P2M_TRY(x1d_setup(N, L, key, idx, nullptr, 0, m.np, (double*)gap, vols, (double*)(w8 + X.volc),
                      nullptr, pp.stream));
    double* cvec = (double*)(w8 + X.c);
    double* xs = (double*)(w8 + X.x);
    P2M_TRY(x1d_m2p_overlap(m, N, key, gap, (const double*)nodal, F, quad, (double*)(w8 + X.fa),
                            (double*)(w8 + X.fb), (double*)(w8 + X.tlo), (double*)(w8 + X.thi),
                            cvec, pp.stream));
    if (kind == P2M_X1D_LUMPED) {
        P2M_TRY(x1d_div(N, F, cvec, vols, 0.0, xs, pp.stream));
    } else if (N > 0) {
        double* coef = (double*)(w8 + X.coef);
        P2M_TRY(x1d_mass_part(N, gap, coef, pp.stream));
        Mesh mp;
        memset(&mp, 0, sizeof(mp));
        mp.dim = 1;
        mp.nx = N;
        mp.ny = 1;
        mp.nn = N;
        mp.inv_hx = mp.inv_hy = 1.0;
        mp.cell_measure = 1.0;
        const p2m_solve_opts o = x1d_opts(opts, N);
        P2M_TRY(launch_cg<double>(mp, F, coef, cvec, vols, xs, P2M_START_FLIP,
                                  x1d_cg_ws(pp, X, c, mp), o, pp.rep, pp.stream));
    }
    P2M_TRY(x1d_scatter(N, F, m.np, idx, xs, (double*)values_out, pp.stream));
    return P2M_OK;
}

p2m_status p2m_x1d_volumes(void* ctx, const p2m_problem* prob, void* vol_out, p2m_report* rep,
                           void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || !vol_out) return P2M_ERR_INVALID_ARG;
    const Context* c = (const Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return P2M_ERR_HIP;
    Prepared pp;
    X1DLayout X;
    int N = 0;
    p2m_status s = x1d_begin(ctx, prob, 1, ws, ws_bytes, stream, rep, pp, X, N);
    if (s != P2M_OK) return s;
    const double L = pp.m.cell_measure * pp.m.nx;
    char* w8 = pp.ws;
    P2M_TRY(x1d_scatter(0, 1, pp.m.np, nullptr, nullptr, (double*)vol_out, pp.stream));   // NaN
    P2M_TRY(x1d_setup(N, L, (const double*)(w8 + X.skey), (const int32_t*)(w8 + X.sidx), nullptr, 0,
                      pp.m.np, (double*)(w8 + X.gap), (double*)(w8 + X.vols), (double*)vol_out,
                      nullptr, pp.stream));
    return P2M_OK;
}

p2m_status p2m_x2d_workspace_size(void* ctx, const p2m_problem* prob, int32_t nfields,
                                  size_t* bytes) {
    if (!bytes) return P2M_ERR_INVALID_ARG;
    Mesh m;
    p2m_status s = x2d_check(ctx, prob, nfields, m);
    if (s != P2M_OK) return s;
    *bytes = make_x2d_layout((const Context*)ctx, m, nfields).total;
    return P2M_OK;
}

p2m_status p2m_x2d_triangulation(void* ctx, const p2m_problem* prob, int32_t* deg_out,
                                 int32_t* nbr_out, int32_t* shift_out, p2m_report* rep, void* ws,
                                 size_t ws_bytes, void* stream) {
    if (!ctx || !rep || !deg_out || !nbr_out || !shift_out) return P2M_ERR_INVALID_ARG;
    const Context* c = (const Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return P2M_ERR_HIP;
    Prepared pp;
    X2DLayout X;
    X2dArgs A;
    p2m_status s = x2d_begin(ctx, prob, 1, nullptr, ws, ws_bytes, stream, rep, pp, X, A);
    if (s != P2M_OK) return s;
    P2M_TRY(x2d_export(A, deg_out, nbr_out, shift_out, pp.stream));
    return P2M_OK;
}

p2m_status p2m_x2d_volumes(void* ctx, const p2m_problem* prob, void* vol_out, p2m_report* rep,
                           void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || !rep || !vol_out) return P2M_ERR_INVALID_ARG;
    const Context* c = (const Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return P2M_ERR_HIP;
    Prepared pp;
    X2DLayout X;
    X2dArgs A;
    p2m_status s = x2d_begin(ctx, prob, 1, nullptr, ws, ws_bytes, stream, rep, pp, X, A);
    if (s != P2M_OK) return s;
    P2M_TRY(x1d_scatter(A.N, 1, pp.m.np, A.perm, A.vol, (double*)vol_out, pp.stream));
    return P2M_OK;
}

p2m_status p2m_x2d_assign(void* ctx, const p2m_problem* prob, int32_t kind, const void* values,
                          int32_t nfields, const p2m_solve_opts* opts, void* nodal_out,
                          p2m_report* rep, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || !rep || !nodal_out) return P2M_ERR_INVALID_ARG;
    p2m_status s = x2d_check_p2m(prob, kind, values, opts);
    if (s != P2M_OK) return s;
    const Context* c = (const Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return P2M_ERR_HIP;
    Prepared pp;
    X2DLayout X;
    X2dArgs A;
    s = x2d_begin(ctx, prob, nfields, values, ws, ws_bytes, stream, rep, pp, X, A);
    if (s != P2M_OK) return s;
    return x2d_run_p2m(c, pp, X, A, prob, kind, values, opts, (double*)nodal_out, pp.rep);
}

p2m_status p2m_x2d_interpolate(void* ctx, const p2m_problem* prob, int32_t kind,
                               const void* nodal, int32_t nfields, const p2m_solve_opts* opts,
                               void* values_out, p2m_report* rep, void* ws, size_t ws_bytes,
                               void* stream) {
    if (!ctx || !rep || !nodal || !values_out) return P2M_ERR_INVALID_ARG;
    p2m_status s = x2d_check_m2p(kind, opts);
    if (s != P2M_OK) return s;
    const Context* c = (const Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return P2M_ERR_HIP;
    if (kind == P2M_X1D_DELTA) {   // the mesh interpolant at the particles: no triangulation
        Mesh m;
        s = x2d_check(ctx, prob, nfields, m);
        if (s != P2M_OK) return s;
        P2M_TRY(launch_report_clear(rep, (hipStream_t)stream));
        P2M_TRY(launch_gather<double>(m, particles_of<double>(prob), (const double*)nodal,
                                      nfields, (double*)values_out, rep, (hipStream_t)stream));
        return P2M_OK;
    }
    Prepared pp;
    X2DLayout X;
    X2dArgs A;
    s = x2d_begin(ctx, prob, nfields, nullptr, ws, ws_bytes, stream, rep, pp, X, A);
    if (s != P2M_OK) return s;
    return x2d_run_m2p(c, pp, X, A, kind, (const double*)nodal, opts, (double*)values_out,
                       pp.rep);
}

p2m_status p2m_x2d_round_trip(void* ctx, const p2m_problem* prob, int32_t kind_p2m,
                              int32_t kind_m2p, const void* values, int32_t nfields,
                              const p2m_solve_opts* opts, void* nodal_out, void* values_out,
                              p2m_report* reps, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || !reps || !nodal_out || !values_out) return P2M_ERR_INVALID_ARG;
    p2m_status s = x2d_check_p2m(prob, kind_p2m, values, opts);
    if (s != P2M_OK) return s;
    s = x2d_check_m2p(kind_m2p, opts);
    if (s != P2M_OK) return s;
    const Context* c = (const Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return P2M_ERR_HIP;
    Prepared pp;
    X2DLayout X;
    X2dArgs A;
    s = x2d_begin(ctx, prob, nfields, values, ws, ws_bytes, stream, reps, pp, X, A);
    if (s != P2M_OK) return s;
    s = x2d_run_p2m(c, pp, X, A, prob, kind_p2m, values, opts, (double*)nodal_out, reps);
    if (s != P2M_OK) return s;
    P2M_TRY(launch_report_clear(reps + 1, pp.stream));
    if (kind_m2p == P2M_X1D_DELTA) {
        P2M_TRY(launch_gather<double>(pp.m, particles_of<double>(prob), (const double*)nodal_out,
                                      nfields, (double*)values_out, reps + 1, pp.stream));
        return P2M_OK;
    }
    return x2d_run_m2p(c, pp, X, A, kind_m2p, (const double*)nodal_out, opts,
                       (double*)values_out, reps + 1);
}

p2m_status p2m_mass_solve(void* ctx, const p2m_problem* prob, int32_t nfields, void* b, const void* w,
                          void* coef, const p2m_solve_opts* opts, void* nodal_inout, p2m_report* rep,
                          void* ws, size_t ws_bytes, void* stream) {
    if (!rep) return P2M_ERR_INVALID_ARG;
    p2m_status s = check_opts(opts);
    if (s != P2M_OK) return s;
    if (opts->start == P2M_START_DELTA1D || opts->start == P2M_START_LEARNED)
        return P2M_ERR_UNSUPPORTED;
    Prepared pp;
    s = prepare(ctx, prob, nfields, ws, ws_bytes, stream, rep, pp);
    if (s != P2M_OK) return s;
    if (!b || !w || !coef || !nodal_inout) return P2M_ERR_INVALID_ARG;
    DeviceGuard g(((Context*)ctx)->device);
    if (!g.ok) return P2M_ERR_HIP;
    pp.clear_rep = true;   // zeroed by the call's first launch
    const Context* c = (const Context*)ctx;
    const Choice ch = choose(c, pp.m, prob->dtype, nfields);
    if (prob->dtype == P2M_F64)
        return run_solve<double>(c, pp, nfields, (double*)b, (const double*)w, (double*)coef,
                                 opts->start, *opts, nodal_inout, ch);
    return run_solve<float>(c, pp, nfields, (float*)b, (const float*)w, (float*)coef, opts->start,
                            *opts, nodal_inout, ch);
}

p2m_status p2m_batch_workspace_size(void* ctx, const p2m_problem* probs, int32_t nprob,
                                    int32_t nfields, size_t* bytes) {
    if (!ctx || !bytes) return P2M_ERR_INVALID_ARG;
    DeviceGuard g(((const Context*)ctx)->device);
    if (!g.ok) return P2M_ERR_HIP;
    BatchPlan P;
    p2m_status s = plan_batch((const Context*)ctx, probs, nprob, nfields, nullptr, nullptr,
                              nullptr, P);
    if (s != P2M_OK) return s;
    *bytes = P.total;
    return P2M_OK;
}

p2m_status p2m_mass_assign_batched(void* ctx, const p2m_problem* probs, int32_t nprob,
                                   const void* const* values, int32_t nfields,
                                   const p2m_solve_opts* opts, void* const* nodal_inout,
                                   p2m_report* reps, void* ws, size_t ws_bytes, void* stream) {
    if (!ctx || !values || !nodal_inout || !reps) return P2M_ERR_INVALID_ARG;
    p2m_status s = check_opts(opts);
    if (s != P2M_OK) return s;
    if (opts->start == P2M_START_DELTA1D || opts->start == P2M_START_LEARNED)
        return P2M_ERR_UNSUPPORTED;
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return P2M_ERR_HIP;
    BatchPlan P;
    s = plan_batch(c, probs, nprob, nfields, values, nodal_inout, reps, P);
    if (s != P2M_OK) return s;
    if (!ws || ws_bytes < P.total || ((uintptr_t)ws) % kAlign) return P2M_ERR_WORKSPACE;
    hipStream_t strm = (hipStream_t)stream;
    // the batch's plan (the tuner's candidate, else a stored plan of its shape class)
    // sets the inner/outer CG schedule
    p2m_solve_opts o = *opts;
    {
        const p2m_plan* plan = c->forced;
        if (!plan && c->use_plans && c->plans) {
            auto it = c->plans->plans.find(batch_key(P.F, P.nprob, P.nn, P.np).s);
            if (it != c->plans->plans.end()) plan = &it->second;
        }
        if (plan && plan->inner_rtol >= 0.0 && plan->inner_rtol < 1.0) o.inner_rtol = plan->inner_rtol;
    }
    opts = &o;
    if (!c->batch) {
        c->batch = new (std::nothrow) BatchCache();
        if (!c->batch) return P2M_ERR_HIP;
        if (hipStreamCreateWithFlags(&c->batch->capture, hipStreamNonBlocking) != hipSuccess) {
            c->batch->capture = nullptr;
            return P2M_ERR_HIP;
        }
    }
    BatchCache& bc = *c->batch;
    // the graph is a function of the instance table, the field count, the options,
    // the workspace and the reports
    std::vector<unsigned char> key;
    auto put = [&](const void* p, size_t n) {
        key.insert(key.end(), (const unsigned char*)p, (const unsigned char*)p + n);
    };
    put(P.inst.data(), sizeof(BatchInst) * P.inst.size());
    put(&P.F, sizeof(P.F));
    put(opts, sizeof(*opts));
    put(&ws, sizeof(ws));
    put(&reps, sizeof(reps));
    put(&c->scan_spin, sizeof(c->scan_spin));
    put(&c->solve_spin, sizeof(c->solve_spin));
    if (!bc.exec || key != bc.key) {
        bc.release();
        // the instance table and tile maps go to the head of the workspace
        bc.upload.assign(P.inst_b + P.lmap_b + P.amap_b + P.rmap_b + P.omap_b, 0);
        unsigned char* u = bc.upload.data();
        memcpy(u, P.inst.data(), sizeof(BatchInst) * P.nprob);
        memcpy(u + P.inst_b, P.lmap.data(), sizeof(int32_t) * P.nlb);
        memcpy(u + P.inst_b + P.lmap_b, P.amap.data(), sizeof(int32_t) * P.nat);
        memcpy(u + P.inst_b + P.lmap_b + P.amap_b, P.rmap.data(), sizeof(int32_t) * P.nrt);
        memcpy(u + P.inst_b + P.lmap_b + P.amap_b + P.rmap_b, P.omap.data(),
               sizeof(int32_t) * P.nrt);
        P2M_TRY(hipMemcpyAsync(ws, u, bc.upload.size(), hipMemcpyHostToDevice, strm));
        P2M_TRY(hipStreamSynchronize(strm));
        P2M_TRY(hipStreamBeginCapture(bc.capture, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_batch(P, (char*)ws, reps, *opts, c->scan_spin, c->solve_spin,
                                     bc.capture);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(bc.capture, &graph);
        if (e != hipSuccess || e2 != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            return P2M_ERR_HIP;
        }
        bc.graph = graph;
        if (hipGraphInstantiate(&bc.exec, bc.graph, nullptr, nullptr, 0) != hipSuccess) {
            bc.exec = nullptr;
            bc.release();
            return P2M_ERR_HIP;
        }
        bc.key.swap(key);
    }
    P2M_TRY(hipGraphLaunch(bc.exec, strm));
    return P2M_OK;
}

p2m_status p2m_set_learned(void* ctx, const float* params) {
    if (!ctx) return P2M_ERR_INVALID_ARG;
    ((Context*)ctx)->learned = params;
    return P2M_OK;
}

p2m_status p2m_learned_features(void* ctx, const p2m_problem* prob, const void* values,
                                int32_t nfields, const int32_t* nodes, int32_t nrows, void* x_out,
                                float* base_out, float* scale_out, p2m_report* rep, void* ws,
                                size_t ws_bytes, void* stream) {
    Prepared pp;
    p2m_status s = prepare(ctx, prob, nfields, ws, ws_bytes, stream, rep, pp);
    if (s != P2M_OK) return s;
    if (pp.m.dim != 2 || prob->dtype != P2M_F32) return P2M_ERR_UNSUPPORTED;
    if (nrows < 0 || (!nodes && nrows != pp.m.nn)) return P2M_ERR_INVALID_ARG;
    if ((pp.m.np > 0 && !values) || (nrows > 0 && (!x_out || !base_out || !scale_out)))
        return P2M_ERR_INVALID_ARG;
    if ((size_t)nrows * nfields * P2M_LEARNED_NIN >= ((size_t)1 << 40)) return P2M_ERR_UNSUPPORTED;
    DeviceGuard g(((Context*)ctx)->device);
    if (!g.ok) return P2M_ERR_HIP;
    pp.clear_rep = true;   // zeroed by the call's first launch
    int32_t* perm = (int32_t*)(pp.ws + pp.L.perm);
    int32_t* cs = (int32_t*)(pp.ws + pp.L.cell_start);
    s = run_bin<float>(pp, prob, perm, cs);
    if (s != P2M_OK) return s;
    float* b = (float*)(pp.ws + pp.L.b);
    float* w = (float*)(pp.ws + pp.L.w);
    P2M_TRY(launch_assemble<float>(pp.m, particles_of<float>(prob), (const float*)values, nfields,
                                   perm, cs, b, w, nullptr, pp.stream));
    P2M_TRY(launch_learn_features(pp.m, particles_of<float>(prob), (const float*)values, nfields,
                                  perm, cs, b, w, nodes, nrows, x_out, base_out, scale_out,
                                  pp.stream));
    return P2M_OK;
}

p2m_status p2m_learned_forward(void* ctx, const float* params, const void* x, int32_t nrows,
                               float* y_out, void* stream) {
    if (!ctx || !params || nrows < 0 || (nrows > 0 && (!x || !y_out))) return P2M_ERR_INVALID_ARG;
    DeviceGuard g(((Context*)ctx)->device);
    if (!g.ok) return P2M_ERR_HIP;
    return st(launch_learn_forward(params, x, nrows, y_out, (hipStream_t)stream));
}

p2m_status p2m_learned_workspace_size(void* ctx, int32_t batch, size_t* bytes) {
    if (!ctx || !bytes || batch < 1) return P2M_ERR_INVALID_ARG;
    *bytes = learn_workspace_bytes(batch);
    return P2M_OK;
}

p2m_status p2m_learned_train_step(void* ctx, float* params, float* adam_m, float* adam_v,
                                  int32_t step, float lr, const void* x, const float* target,
                                  const int32_t* rows, int32_t batch, float* loss_out,
                                  float* grad_out, int32_t apply, void* ws, size_t ws_bytes,
                                  void* stream) {
    if (!ctx || !params || !x || !target || !rows || batch < 1) return P2M_ERR_INVALID_ARG;
    if (apply && (!adam_m || !adam_v || step < 1 || !(lr >= 0.f) || !isfinite(lr)))
        return P2M_ERR_INVALID_ARG;
    if (!ws || ws_bytes < learn_workspace_bytes(batch) || ((uintptr_t)ws) % kAlign)
        return P2M_ERR_WORKSPACE;
    DeviceGuard g(((Context*)ctx)->device);
    if (!g.ok) return P2M_ERR_HIP;
    return st(launch_learn_train(params, adam_m, adam_v, step, lr, x, target, rows, batch,
                                 loss_out, grad_out, apply, ws, (hipStream_t)stream));
}

p2m_status p2m_tune(void* ctx, const p2m_problem* prob, const void* values, int32_t nfields,
                    const p2m_solve_opts* opts, void* nodal_out, p2m_report* rep, void* ws,
                    size_t ws_bytes, void* stream, p2m_plan* best) {
    if (!ctx || !best || !rep) return P2M_ERR_INVALID_ARG;
    p2m_status s = check_opts(opts);
    if (s != P2M_OK) return s;
    if (opts->start != P2M_START_FLIP && opts->start != P2M_START_ZERO) return P2M_ERR_UNSUPPORTED;
    Context* c = (Context*)ctx;
    Prepared pp;
    s = prepare(ctx, prob, nfields, ws, ws_bytes, stream, rep, pp);
    if (s != P2M_OK) return s;
    if ((pp.m.np > 0 && !values) || !nodal_out) return P2M_ERR_INVALID_ARG;
    DeviceGuard g(c->device);
    if (!g.ok) return P2M_ERR_HIP;
    // candidates: every solve kernel that applies, with the default and the 8 x 8
    // scatter tile; the tile-streaming solve with one and with half a workgroup per CU
    std::vector<p2m_plan> cand;
    const double rtols[5] = {-1.0, 3e-5, 1e-5, 1e-6, 0.0};
    auto add = [&](int solver, int groups, int tile) {
        for (double rt : rtols) {
            if (rt >= 0.0 && rt == opts->inner_rtol) continue;
            p2m_plan p;
            memset(&p, 0, sizeof(p));
            p.solver = solver;
            p.groups = groups;
            p.scatter_tile = tile;
            p.inner_rtol = rt;
            cand.push_back(p);
        }
    };
    const bool tiled = prob->dtype == P2M_F32 && pp.m.dim == 2 && nfields <= kResidentMaxFields;
    const int tiles[2] = {0, 8};
    for (int ti = 0; ti < (pp.m.dim == 2 ? 2 : 1); ++ti) {
        const int tile = tiles[ti];
        if (tiled && cgr_supported(pp.m, nfields, c->device)) add(P2M_SOLVER_RESIDENT, 0, tile);
        if (tiled && cgrc_supported(pp.m, nfields, c->device))
            add(P2M_SOLVER_RESIDENT_CHEB, 0, tile);
        if (tiled) {
            const int cap = cgt_grid(pp.m, nfields, 0, c->device);
            if (cap > 0) add(P2M_SOLVER_TILES, cap, tile);
            const int half = cgt_grid(pp.m, nfields, cap / 2, c->device);
            if (half > 0 && half < cap) add(P2M_SOLVER_TILES, half, tile);
        }
        add(P2M_SOLVER_STREAMING, 0, tile);
    }
    hipStream_t strm = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return P2M_ERR_HIP;
    }
    p2m_status result = P2M_OK;
    int best_i = -1;
    p2m_report host_rep;
    for (size_t i = 0; i < cand.size() && result == P2M_OK; ++i) {
        c->forced = &cand[i];
        float ms = 0.f;
        const int reps = 3;
        for (int r = 0; r <= reps && result == P2M_OK; ++r) {
            if (r == 1 && hipEventRecord(e0, strm) != hipSuccess) result = P2M_ERR_HIP;
            if (result == P2M_OK)
                result = p2m_mass_assign(ctx, prob, values, nfields, opts, nodal_out, rep, ws,
                                         ws_bytes, stream);
        }
        if (result == P2M_OK && (hipEventRecord(e1, strm) != hipSuccess ||
                                 hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
                                 hipMemcpy(&host_rep, rep, sizeof(host_rep), hipMemcpyDeviceToHost) !=
                                     hipSuccess))
            result = P2M_ERR_HIP;
        if (result != P2M_OK) break;
        cand[i].time_ms = ms / reps;
        const bool ok = !(host_rep.flags & (P2M_FLAG_NOT_CONVERGED | P2M_FLAG_BREAKDOWN));
        if (ok && (best_i < 0 || cand[i].time_ms < cand[best_i].time_ms)) best_i = (int)i;
    }
    c->forced = nullptr;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != P2M_OK) return result;
    if (best_i < 0) return P2M_ERR_UNSUPPORTED;   // no candidate converged
    if (!c->plans) {
        c->plans = new (std::nothrow) PlanCache();
        if (!c->plans) return P2M_ERR_HIP;
    }
    *best = cand[best_i];
    c->plans->plans[std::string(shape_key(pp.m, prob->dtype, nfields).s)] = *best;
    // leave the chosen plan's result in nodal_out and rep
    c->forced = best;
    result = p2m_mass_assign(ctx, prob, values, nfields, opts, nodal_out, rep, ws, ws_bytes, stream);
    c->forced = nullptr;
    return result;
}

p2m_status p2m_tune_batched(void* ctx, const p2m_problem* probs, int32_t nprob,
                            const void* const* values, int32_t nfields, const p2m_solve_opts* opts,
                            void* const* nodal_inout, p2m_report* reps, void* ws, size_t ws_bytes,
                            void* stream, p2m_plan* best) {
    if (!ctx || !best || !reps || nprob < 1) return P2M_ERR_INVALID_ARG;
    p2m_status s = check_opts(opts);
    if (s != P2M_OK) return s;
    if (opts->start != P2M_START_FLIP && opts->start != P2M_START_ZERO) return P2M_ERR_UNSUPPORTED;
    Context* c = (Context*)ctx;
    DeviceGuard g(c->device);
    if (!g.ok) return P2M_ERR_HIP;
    BatchPlan P;
    s = plan_batch(c, probs, nprob, nfields, values, nodal_inout, reps, P);
    if (s != P2M_OK) return s;
    // candidates: the inner/outer CG schedule of the batched solve
    std::vector<p2m_plan> cand;
    const double rtols[5] = {-1.0, 3e-5, 1e-5, 1e-6, 0.0};
    for (double rt : rtols) {
        if (rt >= 0.0 && rt == opts->inner_rtol) continue;
        p2m_plan p;
        memset(&p, 0, sizeof(p));
        p.solver = P2M_SOLVER_TILES;
        p.inner_rtol = rt;
        cand.push_back(p);
    }
    hipStream_t strm = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return P2M_ERR_HIP;
    }
    std::vector<p2m_report> host(nprob);
    p2m_status result = P2M_OK;
    int best_i = -1;
    for (size_t i = 0; i < cand.size() && result == P2M_OK; ++i) {
        c->forced = &cand[i];
        float ms = 0.f;
        const int runs = 3;
        for (int r = 0; r <= runs && result == P2M_OK; ++r) {  // run 0 captures the graph
            if (r == 1 && hipEventRecord(e0, strm) != hipSuccess) result = P2M_ERR_HIP;
            if (result == P2M_OK)
                result = p2m_mass_assign_batched(ctx, probs, nprob, values, nfields, opts,
                                                 nodal_inout, reps, ws, ws_bytes, stream);
        }
        if (result == P2M_OK &&
            (hipEventRecord(e1, strm) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
             hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
             hipMemcpy(host.data(), reps, sizeof(p2m_report) * nprob, hipMemcpyDeviceToHost) !=
                 hipSuccess))
            result = P2M_ERR_HIP;
        if (result != P2M_OK) break;
        cand[i].time_ms = ms / runs;
        bool ok = true;
        for (const p2m_report& r : host)
            ok = ok && !(r.flags & (P2M_FLAG_NOT_CONVERGED | P2M_FLAG_BREAKDOWN));
        if (ok && (best_i < 0 || cand[i].time_ms < cand[best_i].time_ms)) best_i = (int)i;
    }
    c->forced = nullptr;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != P2M_OK) return result;
    if (best_i < 0) return P2M_ERR_UNSUPPORTED;   // no candidate converged
    if (!c->plans) {
        c->plans = new (std::nothrow) PlanCache();
        if (!c->plans) return P2M_ERR_HIP;
    }
    *best = cand[best_i];
    c->plans->plans[std::string(batch_key(P.F, P.nprob, P.nn, P.np).s)] = *best;
    // leave the chosen plan's results in nodal_inout and reps
    c->forced = best;
    result = p2m_mass_assign_batched(ctx, probs, nprob, values, nfields, opts, nodal_inout, reps, ws,
                                     ws_bytes, stream);
    c->forced = nullptr;
    return result;
}

p2m_status p2m_plan_get_batched(void* ctx, const p2m_problem* probs, int32_t nprob,
                                int32_t nfields, p2m_plan* plan) {
    if (!ctx || !plan) return P2M_ERR_INVALID_ARG;
    Context* c = (Context*)ctx;
    BatchPlan P;
    p2m_status s = plan_batch(c, probs, nprob, nfields, nullptr, nullptr, nullptr, P);
    if (s != P2M_OK) return s;
    if (!c->plans) return P2M_ERR_UNSUPPORTED;
    auto it = c->plans->plans.find(batch_key(P.F, P.nprob, P.nn, P.np).s);
    if (it == c->plans->plans.end()) return P2M_ERR_UNSUPPORTED;
    *plan = it->second;
    return P2M_OK;
}

p2m_status p2m_plan_get(void* ctx, const p2m_problem* prob, int32_t nfields, p2m_plan* plan) {
    if (!ctx || !plan || nfields < 1 || nfields > kMaxFields) return P2M_ERR_INVALID_ARG;
    Mesh m;
    p2m_status s = check_problem(prob, m);
    if (s != P2M_OK) return s;
    const Context* c = (const Context*)ctx;
    if (!c->plans) return P2M_ERR_UNSUPPORTED;
    auto it = c->plans->plans.find(shape_key(m, prob->dtype, nfields).s);
    if (it == c->plans->plans.end()) return P2M_ERR_UNSUPPORTED;
    *plan = it->second;
    return P2M_OK;
}

p2m_status p2m_plan_save(void* ctx, const char* path) {
    if (!ctx || !path) return P2M_ERR_INVALID_ARG;
    const Context* c = (const Context*)ctx;
    FILE* f = fopen(path, "w");
    if (!f) return P2M_ERR_INVALID_ARG;
    bool ok = fputs("{\n", f) >= 0;
    size_t i = 0, n = c->plans ? c->plans->plans.size() : 0;
    if (c->plans)
        for (const auto& kv : c->plans->plans) {
            char line[512];
            const int len = format_plan_line(line, sizeof line, kv.first, kv.second, ++i == n);
            ok = ok && len > 0 && fputs(line, f) >= 0;
        }
    ok = ok && fputs("}\n", f) >= 0;
    return (fclose(f) == 0 && ok) ? P2M_OK : P2M_ERR_INVALID_ARG;
}

p2m_status p2m_plan_load(void* ctx, const char* path) {
    if (!ctx || !path) return P2M_ERR_INVALID_ARG;
    Context* c = (Context*)ctx;
    FILE* f = fopen(path, "r");
    if (!f) return P2M_ERR_INVALID_ARG;
    std::map<std::string, p2m_plan> got;
    char line[512];
    p2m_status s = P2M_OK;
    while (fgets(line, sizeof line, f)) {
        std::string key;
        p2m_plan p;
        const PlanLine r = parse_plan_line(line, key, p);
        if (r == kPlanSkip) continue;   // braces
        if (r == kPlanBad) {
            s = P2M_ERR_INVALID_ARG;
            break;
        }
        got[key] = p;
    }
    fclose(f);
    if (s != P2M_OK) return s;
    if (!c->plans) {
        c->plans = new (std::nothrow) PlanCache();
        if (!c->plans) return P2M_ERR_HIP;
    }
    for (const auto& kv : got) c->plans->plans[kv.first] = kv.second;
    return P2M_OK;
}

p2m_status p2m_plan_clear(void* ctx) {
    if (!ctx) return P2M_ERR_INVALID_ARG;
    Context* c = (Context*)ctx;
    if (c->plans) c->plans->plans.clear();
    return P2M_OK;
}

}  // extern "C"
