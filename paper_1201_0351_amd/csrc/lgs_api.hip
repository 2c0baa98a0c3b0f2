// lgs_api.hip -- host side of the C ABI declared in include/lgs_lbm.h.
//
// A context owns n instances laid out back to back in one device workspace
// (caller-provided, e.g. a torch tensor, or allocated here).  Kernels receive
// an Inst descriptor by value.  Steps alternate between two population
// lattices ("parity"); per-step counters and force accumulators are kept per
// parity so that no memset is ever needed inside a step.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "lgs_internal.h"

using namespace lgs;

// Scratch memory of lbm_mass_total_noalloc: the chunk partials of the mass
// total (MASS_PARTS_MAX) and its result, one copy per GPU, held until the
// process ends.  Host code never uses this name as an address: it uses the
// device's copy looked up by scratch_setup.
static __device__ __align__(256) double scratch[MASS_PARTS_MAX + 1];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_OK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(LBM_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Address of `scratch` on each device (null until looked up).
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES];

// Look up device dev's copy of `scratch` once; dev must be the current device.
int scratch_setup(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return fail(LBM_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return LBM_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(LBM_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = (double*)p;
    return LBM_OK;
}

double* scratch_of(int dev) {
    if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[dev];
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t storage_bytes(int storage) { return storage == LBM_FP32 ? 4 : 2; }

// Elements between two population planes: N plus a pad, so that the planes a
// wavefront streams do not all start at the same offset modulo a large power
// of two (LGS_PLANE_PAD_BYTES, a multiple of 256; 17 x 256 bytes measured
// 7% faster for FP16 storage on the 512x256x256 lattice, whose planes are
// 2^27 bytes apart without it, and no slower elsewhere).
#ifndef LGS_PLANE_PAD_BYTES
#define LGS_PLANE_PAD_BYTES 4352
#endif
// Uniform factors of the bulk collision (k_sweep.hip), from omega, the
// acceleration and the storage scale, rounded once to FP32.
static void collide_constants(Inst& I) {
    CollideConst& K = I.cc;
    const double om = (double)I.omega;
    const double a[3] = {(double)I.ax, (double)I.ay, (double)I.az};
    const double sc = (double)I.scale;
    K.om1 = (float)(1.0 - om);
    K.om15 = (float)(1.5 * om);
    K.om45 = (float)(4.5 * om);
    K.om3 = (float)(3.0 * om);
    for (int c = 0; c < 3; ++c) K.a3[c] = (float)(3.0 * a[c]);
    for (int k = 0; k < 9; ++k) {
        const int p = pair_p(k);
        const double ca = cx(p) * a[0] + cy(p) * a[1] + cz(p) * a[2];
        K.ca9[k] = (float)(9.0 * ca);
        K.ca3[k] = (float)(3.0 * ca);
    }
    const int rep[3] = {0, 1, 7};  // a link of each weight class
    for (int c = 0; c < 3; ++c) {
        K.omw[c] = (float)(om * wgtd(rep[c]));
        K.sw[c] = (float)(sc * wgtd(rep[c]));
    }
    K.inv = (float)(1.0 / sc);
}

size_t plane_stride(const lbm_config& c) {
    const size_t N = (size_t)c.nx * c.ny * c.nz;
    const size_t sb = storage_bytes(c.storage);
    const size_t bytes = (N * sb + 255) / 256 * 256 + LGS_PLANE_PAD_BYTES;
    return bytes / sb;
}

struct InstHost {
    lbm_config cfg;
    Inst dev;
    DevBody bodies[MAXB];  // host copy, refreshed from the device before use
    lbm_body desc[MAXB];   // caller's description (shape, density, mode)
    bool need_remap;       // a body was set since the last remap
    bool any_free;         // some body is integrated on the device
    int remap_blocks;      // workgroups per body of the remap kernels
    size_t offset, bytes;
    // The bulk sweep's layer bound.  The commit launch of full step m
    // reports (m << 32) | v into zpin_host, with v at least the highest layer
    // that may hold fluid after step m - 1.  A step raises that layer by at
    // most two (its remap refills cells next to fluid, its conversions give
    // gas cells next to filling cells interface), so the bulk sweep of step
    // s needs layers 0 .. v + 2 (s - m) + 1 only.  steps counts every step
    // that advanced the instance.
    unsigned long long* zpin_host;
    long long steps;
    // pinned landing place of a step's force sums and body records for the
    // host body update (null: pageable copies)
    unsigned char* cpl_host;
};
constexpr size_t CPL_BYTES = sizeof(double) * MAXB * 6 + sizeof(DevBody) * MAXB;

// Byte layout of one instance inside the workspace.
size_t layout(const lbm_config& c, Inst* I, char* base) {
    const size_t N = (size_t)c.nx * c.ny * c.nz;
    const size_t sb = storage_bytes(c.storage);
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const size_t ps = plane_stride(c);
    char* p0 = take(Q * ps * sb);
    char* p1 = take(Q * ps * sb);
    char* fl = take(N);
    char* ph0 = take(4 * N);
    char* ph1 = take(4 * N);
    char* mh = take(4 * N);
    char* ml = take(4 * N);
    char* sh = take(4 * N);
    char* ax = take(4 * N);
    char* ru = take(N);
    char* no = take(N);
    char* lb = take(N);
    char* kp = take(c.surface_tension != 0.0 ? 4 * N : 0);
    char* cl = take(4 * (N / 32 + 1));
    char* cm = take(4 * N);
    char* l0 = take(4 * N);
    char* l1 = take(4 * N);
    char* l2 = take(4 * N);
    char* l3 = take(4 * N);
    char* l4 = take(4 * N);
    char* fb = take(sizeof(uint32_t) * BND_BLOCKS_MAX);
    char* fv = take(sizeof(long long) * FXW * MAXB * BND_BLOCKS_MAX);
    char* mp = take(sizeof(double) * mass_parts((int)N));
    char* ct = take(sizeof(Ctl));
    char* bd = take(sizeof(DevBody) * MAXB);
    if (I) {
        I->pop[0] = p0;
        I->pop[1] = p1;
        I->flags = (uint8_t*)fl;
        I->phi[0] = (float*)ph0;
        I->phi[1] = (float*)ph1;
        I->m_hi = (float*)mh;
        I->m_lo = (float*)ml;
        I->share = (float*)sh;
        I->aux = (float*)ax;
        I->rule = (uint8_t*)ru;
        I->nearo = (uint8_t*)no;
        I->lnb = (uint8_t*)lb;
        I->kap = c.surface_tension != 0.0 ? (float*)kp : nullptr;
        I->claim = (uint32_t*)cl;
        I->cmask = (uint32_t*)cm;
        I->cand = (int*)l0;
        I->newg = (int*)l1;
        I->newl = (int*)l2;
        I->recv = (int*)l3;
        I->bnd = (int*)l4;
        I->frec_mask = (uint32_t*)fb;
        I->frec_v = (long long*)fv;
        I->mass_part = (double*)mp;
        I->ctl = (Ctl*)ct;
        I->bodies = (DevBody*)bd;
        I->list_cap = (int)N;
    }
    return off;
}

int validate(const lbm_config& c, int k) {
    char buf[256];
    auto bad = [&](const char* what) {
        snprintf(buf, sizeof buf, "instance %d: %s", k, what);
        return fail(LBM_ERR_INVALID, buf);
    };
    if (c.nx <= 0 || c.ny <= 0 || c.nz <= 0) return bad("lattice sizes must be positive");
    if ((double)c.nx * c.ny * c.nz > 2.0e9 / Q) return bad("lattice too large for 32-bit indexing");
    if (!(c.tau > 0.5)) return bad("tau must exceed 1/2 (positive viscosity)");
    if (c.storage != LBM_FP32 && c.storage != LBM_FP16_DEV && c.storage != LBM_BF16_DEV) return bad("unknown storage");
    if (!(c.rho_gas > 0.0)) return bad("rho_gas must be positive");
    if (!(c.eps >= 0.0)) return bad("eps must be >= 0");
    if (c.recon_mode < 0 || c.recon_mode > 2) return bad("unknown recon_mode");
    if (c.max_bodies < 0 || c.max_bodies > MAXB) return bad("max_bodies out of range");
    if (c.host_body_update != 0 && c.host_body_update != 1) return bad("host_body_update must be 0 or 1");
    for (int a = 0; a < 3; ++a)
        if (!(std::fabs(c.wall_vel[a]) < 0.1)) return bad("wall_vel must be well below the lattice speed of sound");
    if (!(c.surface_tension >= 0.0 && c.surface_tension < 0.1)) return bad("surface_tension must be in [0, 0.1)");
    const double n[3] = {(double)c.nx, (double)c.ny, (double)c.nz};
    for (int a = 0; a < 3; ++a)
        if (!(n[a] * std::fabs(c.accel[a]) < 0.1 / 3.0))
            return bad("acceleration too large for the lattice (l_k |a_k| must be << c_s^2)");
    if (c.storage == LBM_FP16_DEV) {
        double s = c.fp16_scale == 0.0 ? 4096.0 : c.fp16_scale;
        int e;
        if (!(s > 0.0) || std::frexp(s, &e) != 0.5) return bad("fp16_scale must be a power of two");
    }
    return LBM_OK;
}

}  // namespace

struct lbm_ctx {
    int n_inst = 0;
    int device = 0;  // the device current at creation
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    int parity = 0;
    int last_parity = 0;
    bool have_forces = false;
    std::vector<InstHost> inst;
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;  // start/stop events of timed sweeps
    size_t ev_used = 0;
    int tile_x = 0;   // bulk-sweep tile width (cells along x; 0: 256 consecutive cells of a layer)
    bool nt_store = false;  // non-temporal population stores in the bulk sweep
    int bnd_layout = 0;     // boundary sweep: 0 = 8 lanes per cell, 1 = one thread per cell
    // batches: all instances of the context step with one launch per kernel
    // (instance table and workgroup offsets at the head of the workspace)
    bool batched = false;
    Inst* d_tab = nullptr;
    int* d_bulk_off = nullptr;
    int* d_bnd_off = nullptr;
    int bulk_total = 0, bnd_total = 0;
    bool bnd_fits = false;  // every instance addressable with 32-bit offsets
    // graph replay of two full steps (captured on a private stream)
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    int gparity = 0;
    std::vector<unsigned char> gremap;  // need_remap of every instance at the start of the graph
    bool capturing = false;             // run_step launches into a graph capture
    unsigned max_lag = 8;               // steps the host may run ahead of the layer reports
};

// Steps a report may lag behind the host before the host waits for the GPU:
// enough to keep about LAG_BYTES of bulk-sweep traffic queued, 2 to
// LAYER_LAG.  Each step of lag widens the bound by two layers, which cost
// their early-exit tiles (a third of the liquid tiles of a batch of small
// lattices at 8 steps).
constexpr unsigned LAYER_LAG = 8;
constexpr double LAG_BYTES = 4e9;
static unsigned lag_limit(double moved_bytes) {
    const double n = moved_bytes > 0.0 ? std::ceil(LAG_BYTES / moved_bytes) : (double)LAYER_LAG;
    return (unsigned)std::min((double)LAYER_LAG, std::max(2.0, n));
}

// Layers the bulk sweep of the instance's next step must cover (0: all).
static int layer_bound(lbm_ctx* c, const InstHost& h) {
    if (!h.zpin_host) return 0;
    for (;;) {
        const unsigned long long w = *(volatile unsigned long long*)h.zpin_host;
        const unsigned lag = (unsigned)h.steps - (unsigned)(w >> 32);
        // one launch per instance of a batch: the host's launches bound the
        // step, so it keeps the deepest queue
        const unsigned lim = c->n_inst > 1 && !c->batched ? LAYER_LAG : c->max_lag;
        if (lag <= lim) {
            const long long top = (long long)(unsigned)w + 2ll * lag + 1;
            return top + 1 >= h.dev.nz ? 0 : (int)(top + 1);
        }
        // the host is ahead: wait for a newer report, unless nothing is queued
        // (or the stream failed, which the next sync reports)
        if (hipStreamQuery(c->stream) != hipErrorNotReady) return 0;
        std::this_thread::yield();
    }
}

// Population bytes the bulk sweeps of a step move: 2 Q values per cell of
// the layers up to each instance's bound.  Streaming stores pass the caches,
// which is faster once these exceed the 256 MiB cache in front of HBM and
// slower below it (the next step's source then stays cached).
constexpr double CACHE_BYTES = 256.0 * (1 << 20);
static double moved_bytes(lbm_ctx* c) {
    double b = 0.0;
    for (const InstHost& h : c->inst) {
        const int L = layer_bound(c, h);
        const double layers = L > 0 ? L : h.dev.nz;
        b += 2.0 * Q * (double)h.dev.nx * (double)h.dev.ny * layers * (double)storage_bytes(h.cfg.storage);
    }
    return b;
}

// Workspace head of a context: the instance table and two offset arrays.
size_t ctx_head_bytes(int n) { return align256(sizeof(Inst) * n) + 2 * align256(sizeof(int) * (n + 1)); }

static hipEvent_t next_event(lbm_ctx* c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        // timing only: no system-scope fence when the event completes, so the
        // brackets add as little as possible to the measured kernels
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

extern "C" {

static void drop_graph(lbm_ctx* c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
}

// Instance table and workgroup offsets of a batched context (synchronous;
// called at creation and whenever a descriptor or the tile width changes).
static int upload_batch(lbm_ctx* c) {
    if (!c->batched) return LBM_OK;
    const int n = c->n_inst;
    std::vector<Inst> tab(n);
    std::vector<int> bo(n + 1), bb(n + 1);
    bo[0] = bb[0] = 0;
    for (int k = 0; k < n; ++k) {
        tab[k] = c->inst[k].dev;
        bo[k + 1] = bo[k] + bulk_blocks(tab[k], c->tile_x);
        bb[k + 1] = bb[k] + (boundary_blocks(tab[k]) + 7) / 8 * 8;
    }
    c->bulk_total = bo[n];
    c->bnd_total = bb[n];
    c->bnd_fits = true;
    for (int k = 0; k < n; ++k)
        c->bnd_fits = c->bnd_fits && bnd_buf_fits(tab[k], storage_bytes(c->inst[k].cfg.storage));
    HIP_OK(hipStreamSynchronize(c->stream));
    HIP_OK(hipMemcpy(c->d_tab, tab.data(), sizeof(Inst) * n, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->d_bulk_off, bo.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->d_bnd_off, bb.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
    return LBM_OK;
}

const char* lbm_last_error(void) { return g_err.c_str(); }

int32_t lbm_workspace_size(const lbm_config* cfgs, int32_t n_inst, size_t* bytes) {
    if (!cfgs || n_inst <= 0 || !bytes) return fail(LBM_ERR_INVALID, "workspace_size: bad arguments");
    size_t tot = ctx_head_bytes(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        int rc = validate(cfgs[k], k);
        if (rc) return rc;
        tot += layout(cfgs[k], nullptr, nullptr);
    }
    *bytes = tot;
    return LBM_OK;
}

int32_t lbm_create(const lbm_config* cfgs, int32_t n_inst, void* d_workspace, size_t ws_bytes, void* hip_stream,
                   lbm_ctx** out) {
    if (!out) return fail(LBM_ERR_INVALID, "create: out is NULL");
    size_t need = 0;
    int rc = lbm_workspace_size(cfgs, n_inst, &need);
    if (rc) return rc;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    rc = scratch_setup(dev);
    if (rc) return rc;
    lbm_ctx* c = new lbm_ctx();
    c->n_inst = n_inst;
    c->device = dev;
    c->stream = (hipStream_t)hip_stream;
    if (d_workspace) {
        if (ws_bytes < need) {
            delete c;
            return fail(LBM_ERR_NOMEM, "create: workspace smaller than lbm_workspace_size");
        }
        if (((uintptr_t)d_workspace) & 255) {
            delete c;
            return fail(LBM_ERR_INVALID, "create: workspace must be 256-byte aligned");
        }
        c->ws = (char*)d_workspace;
        c->ws_bytes = ws_bytes;
    } else {
        void* p = nullptr;
        if (hipMalloc(&p, need) != hipSuccess) {
            delete c;
            return fail(LBM_ERR_NOMEM, "create: hipMalloc of the workspace failed");
        }
        c->ws = (char*)p;
        c->ws_bytes = need;
        c->own_ws = true;
    }
    c->inst.resize(n_inst);
    c->d_tab = (Inst*)c->ws;
    c->d_bulk_off = (int*)(c->ws + align256(sizeof(Inst) * n_inst));
    c->d_bnd_off = (int*)(c->ws + align256(sizeof(Inst) * n_inst) + align256(sizeof(int) * (n_inst + 1)));
    size_t off = ctx_head_bytes(n_inst);
    for (int k = 0; k < n_inst; ++k) {
        InstHost& h = c->inst[k];
        memset(&h, 0, sizeof(InstHost));
        h.cfg = cfgs[k];
        if (h.cfg.storage == LBM_FP16_DEV && h.cfg.fp16_scale == 0.0) h.cfg.fp16_scale = 4096.0;
        Inst& I = h.dev;
        h.offset = off;
        h.bytes = layout(h.cfg, &I, c->ws + off);
        off += h.bytes;
        I.nx = h.cfg.nx;
        I.ny = h.cfg.ny;
        I.nz = h.cfg.nz;
        I.N = h.cfg.nx * h.cfg.ny * h.cfg.nz;
        I.ps = plane_stride(h.cfg);
        I.periodic = h.cfg.periodic & 7;
        I.recon_mode = h.cfg.recon_mode;
        I.storage = h.cfg.storage;
        I.nbodies = 0;
        I.omega = (float)(1.0 / h.cfg.tau);
        I.ax = (float)h.cfg.accel[0];
        I.ay = (float)h.cfg.accel[1];
        I.az = (float)h.cfg.accel[2];
        I.rho_g = (float)h.cfg.rho_gas;
        for (int a = 0; a < 3; ++a) I.wall_u[a] = (float)h.cfg.wall_vel[a];
        I.wall_moving = h.cfg.wall_vel[0] != 0.0 || h.cfg.wall_vel[1] != 0.0 || h.cfg.wall_vel[2] != 0.0;
        I.lap = (float)(6.0 * h.cfg.surface_tension);
        I.scale = h.cfg.storage == LBM_FP16_DEV ? (float)h.cfg.fp16_scale : 1.f;
        I.inv_scale = 1.f / I.scale;
        collide_constants(I);
        I.eps = h.cfg.eps;
        const size_t N = (size_t)I.N;
        HIP_OK(hipMemsetAsync(I.ctl, 0, sizeof(Ctl), c->stream));
        HIP_OK(hipMemsetAsync(I.bodies, 0, sizeof(DevBody) * MAXB, c->stream));
        HIP_OK(hipMemsetAsync(I.claim, 0, 4 * (N / 32 + 1), c->stream));
        HIP_OK(hipMemsetAsync(I.cmask, 0, 4 * N, c->stream));
        HIP_OK(hipMemsetAsync(I.rule, 0, N, c->stream));
        HIP_OK(hipMemsetAsync(I.nearo, 0, N, c->stream));  // no bodies and a closed layer
        launch_init(I, h.cfg, c->stream);
        launch_ztop(I, c->stream);
        HIP_OK(hipGetLastError());
    }
    // Bulk-sweep tiles of 256 consecutive cells of a layer: no idle lanes for
    // widths that are no multiple of a tile width, rows as long as the
    // lattice's (measured at least as fast as the rectangular tiles on every
    // workload here, 9-21% faster on the batch of uneven lattices).
    c->tile_x = 0;
    c->nt_store = false;  // set from the layer bounds below
    c->batched = n_inst > 1;
    for (int k = 1; k < n_inst; ++k)
        if (c->inst[k].cfg.storage != c->inst[0].cfg.storage) c->batched = false;
    // the layer bounds' pinned words, starting from the scanned ztop
    HIP_OK(hipStreamSynchronize(c->stream));
    for (int k = 0; k < n_inst; ++k) {
        InstHost& h = c->inst[k];
        if (h.cfg.host_body_update) {
            void* cp = nullptr;
            if (hipHostMalloc(&cp, CPL_BYTES, hipHostMallocDefault) == hipSuccess) h.cpl_host = (unsigned char*)cp;
            else (void)hipGetLastError();  // pageable copies instead
        }
        void* hp = nullptr;
        void* dp = nullptr;
        if (hipHostMalloc(&hp, sizeof(unsigned long long), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
            hipHostGetDevicePointer(&dp, hp, 0) != hipSuccess) {
            if (hp) (void)hipHostFree(hp);
            (void)hipGetLastError();
            continue;  // no bound: the bulk sweep covers all layers
        }
        int zt = 0;
        HIP_OK(hipMemcpy(&zt, &h.dev.ctl->ztop, sizeof(int), hipMemcpyDeviceToHost));
        h.zpin_host = (unsigned long long*)hp;
        *(volatile unsigned long long*)h.zpin_host = (unsigned long long)(unsigned)zt;
        h.dev.zpin = (unsigned long long*)dp;
    }
    const double moved = moved_bytes(c);
    c->nt_store = moved > CACHE_BYTES;
    c->max_lag = lag_limit(moved);
    rc = upload_batch(c);
    if (rc) return rc;
    *out = c;
    return LBM_OK;
}

int32_t lbm_destroy(lbm_ctx* c) {
    if (!c) return LBM_OK;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->own_ws) (void)hipFree(c->ws);
    for (InstHost& h : c->inst) {
        if (h.zpin_host) (void)hipHostFree(h.zpin_host);
        if (h.cpl_host) (void)hipHostFree(h.cpl_host);
    }
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return LBM_OK;
}

static int check_inst(lbm_ctx* c, int inst) {
    if (!c) return fail(LBM_ERR_INVALID, "context is NULL");
    if (inst < 0 || inst >= c->n_inst) return fail(LBM_ERR_INVALID, "instance index out of range");
    return LBM_OK;
}

// Copy the device body records into the host copy (the device owns the
// state of free bodies and the mapping bookkeeping).
static int pull_bodies(lbm_ctx* c, InstHost& h) {
    HIP_OK(hipStreamSynchronize(c->stream));
    HIP_OK(hipMemcpy(h.bodies, h.dev.bodies, sizeof(DevBody) * MAXB, hipMemcpyDeviceToHost));
    return LBM_OK;
}

static void refresh_instance_flags(InstHost& h) {
    h.any_free = false;
    h.remap_blocks = 0;
    for (int k = 0; k < h.dev.nbodies; ++k) {
        const DevBody& d = h.bodies[k];
        if (!d.active) continue;
        if (d.free_body && d.dof) h.any_free = true;
        // the remap box is at most 2 Rc + 9 cells wide on each axis (old and
        // new bounding boxes within a cell of each other, two cells margin)
        const double Rc = std::sqrt(d.half[0] * d.half[0] + d.half[1] * d.half[1] + d.half[2] * d.half[2]);
        const double w = std::ceil(2.0 * Rc) + 9.0;
        const double cells = w * w * w;
        const int blocks = (int)std::min(512.0, std::ceil(cells / 256.0));
        h.remap_blocks = std::max(h.remap_blocks, blocks);
    }
}

// The lbm_set_body checks of a new pose d of body k (h.bodies holds the
// device's current records).
static int check_pose(const InstHost& h, int k, const DevBody& d, bool was_mapped, const char* who) {
    const double n[3] = {(double)h.cfg.nx, (double)h.cfg.ny, (double)h.cfg.nz};
    const double Rc = std::sqrt(d.half[0] * d.half[0] + d.half[1] * d.half[1] + d.half[2] * d.half[2]);
    // inside the non-periodic extent with a free cell of margin
    for (int a = 0; a < 3; ++a) {
        if (h.cfg.periodic & (1 << a)) {
            if (2.0 * d.ext[a] >= n[a] && !(d.half[a] >= 0.5 * n[a] && d.ext[a] == d.half[a]))
                return fail(LBM_ERR_INVALID, std::string(who) + ": body wider than a periodic axis");
            continue;
        }
        if (d.pos[a] - d.ext[a] < 1.0 || d.pos[a] + d.ext[a] > n[a] - 1.0)
            return fail(LBM_ERR_INVALID, std::string(who) + ": body must stay one cell inside the walls");
    }
    const double speed = std::sqrt(d.vel[0] * d.vel[0] + d.vel[1] * d.vel[1] + d.vel[2] * d.vel[2]) +
                         std::sqrt(d.omega[0] * d.omega[0] + d.omega[1] * d.omega[1] + d.omega[2] * d.omega[2]) * Rc;
    if (!(speed < 1.0))
        return fail(LBM_ERR_INVALID, std::string(who) + ": surface speed must be below one cell per step");
    if (was_mapped) {
        for (int a = 0; a < 3; ++a) {
            const double dd = wrap_rel(d.pos[a] - h.bodies[k].prev_pos[a], n[a], h.cfg.periodic & (1 << a));
            if (!(std::fabs(dd) < 1.0))
                return fail(LBM_ERR_INVALID, std::string(who) + ": body moved a cell or more since its last mapping");
        }
    }
    for (int j = 0; j < h.dev.nbodies; ++j) {
        if (j == k || !h.bodies[j].active) continue;
        bool sep = false;
        for (int a = 0; a < 3; ++a) {
            const double dd = wrap_rel(d.pos[a] - h.bodies[j].pos[a], n[a], h.cfg.periodic & (1 << a));
            if (std::fabs(dd) >= d.ext[a] + h.bodies[j].ext[a] + 3.0) sep = true;
        }
        if (!sep) return fail(LBM_ERR_INVALID, std::string(who) + ": bodies must stay three cells apart");
    }
    return LBM_OK;
}

int32_t lbm_set_body(lbm_ctx* c, int32_t inst, int32_t k, const lbm_body* b) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    InstHost& h = c->inst[inst];
    if (!b || k < 0 || k >= MAXB || k >= std::max(1, h.cfg.max_bodies))
        return fail(LBM_ERR_INVALID, "set_body: body index out of range (raise max_bodies)");
    rc = pull_bodies(c, h);
    if (rc) return rc;
    drop_graph(c);
    const double n[3] = {(double)h.cfg.nx, (double)h.cfg.ny, (double)h.cfg.nz};
    const DevBody& old = h.bodies[k];
    const bool was_mapped = old.active && old.mapped;
    DevBody d;
    memset(&d, 0, sizeof d);
    if (b->shape != LBM_SHAPE_CUBOID && b->shape != LBM_SHAPE_SPHERE)
        return fail(LBM_ERR_INVALID, "set_body: unknown shape");
    d.shape = (int)b->shape;
    for (int a = 0; a < 3; ++a) {
        // a sphere keeps its radius on every axis
        const double hk = d.shape == LBM_SHAPE_SPHERE ? b->half_ext[0] : b->half_ext[a];
        if (!(hk > 0.0)) return fail(LBM_ERR_INVALID, "set_body: half extents must be positive");
        double p = b->pos[a];
        if (h.cfg.periodic & (1 << a)) p = p - n[a] * std::floor(p / n[a]);
        d.pos[a] = p;
        d.half[a] = hk;
        d.vel[a] = b->vel[a];
        d.omega[a] = b->omega[a];
    }
    const double qn = std::sqrt(b->quat[0] * b->quat[0] + b->quat[1] * b->quat[1] + b->quat[2] * b->quat[2] +
                                b->quat[3] * b->quat[3]);
    if (!(std::fabs(qn - 1.0) < 1e-6)) return fail(LBM_ERR_INVALID, "set_body: quaternion must be unit");
    for (int a = 0; a < 4; ++a) d.quat[a] = b->quat[a];
    quat_to_R(b->quat, d.R);
    box_extent(d.shape, d.R, d.half, d.ext);
    rc = check_pose(h, k, d, was_mapped, "set_body");
    if (rc) return rc;
    if (b->fixed == 0 && (b->dof_mask & ~0x3Fu)) return fail(LBM_ERR_INVALID, "set_body: dof_mask has unknown bits");
    if (b->fixed == 0 && !(b->density > 0.0)) return fail(LBM_ERR_INVALID, "set_body: free body needs a density > 0");
    d.density = b->density;
    d.free_body = b->fixed == 0 ? 1 : 0;
    d.dof = b->fixed == 0 ? b->dof_mask : 0u;
    d.active = 1;
    d.moved = 1;
    d.mapped = was_mapped ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        d.prev_pos[a] = was_mapped ? old.prev_pos[a] : d.pos[a];
        d.prev_ext[a] = was_mapped ? old.prev_ext[a] : d.ext[a];
    }
    h.desc[k] = *b;
    for (int a = 0; a < 3; ++a) h.desc[k].pos[a] = d.pos[a];
    h.bodies[k] = d;
    const bool grown = k + 1 > h.dev.nbodies;
    if (grown) h.dev.nbodies = k + 1;
    h.need_remap = true;
    refresh_instance_flags(h);
    launch_set_body(h.dev, k, h.bodies[k], c->stream);
    HIP_OK(hipGetLastError());
    if (grown) return upload_batch(c);  // the descriptor changed
    return LBM_OK;
}

int32_t lbm_get_body(lbm_ctx* c, int32_t inst, int32_t k, lbm_body* b) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    InstHost& h = c->inst[inst];
    if (!b || k < 0 || k >= h.dev.nbodies || !h.bodies[k].active) return fail(LBM_ERR_INVALID, "get_body: no such body");
    rc = pull_bodies(c, h);
    if (rc) return rc;
    const DevBody& d = h.bodies[k];
    *b = h.desc[k];
    for (int a = 0; a < 3; ++a) {
        b->pos[a] = d.pos[a];
        b->vel[a] = d.vel[a];
        b->omega[a] = d.omega[a];
    }
    for (int a = 0; a < 4; ++a) b->quat[a] = d.quat[a];
    return LBM_OK;
}

__global__ void k_copy_state(Inst I, int from);

// Host update of the free bodies of an instance configured for it, after a
// full step of parity p: wait for the step, read the reduced forces and the
// body records, apply lbm_integrate_body fed with the mean of this and the
// previous step's force and torque, check the new pose as lbm_set_body does
// and upload it; the next step maps it.
static int couple_on_host(lbm_ctx* c, InstHost& h, int p) {
    double acc[MAXB][6];
    int rc = LBM_OK;
    if (h.cpl_host) {
        // both copies queued behind the step, one wait for the stream
        unsigned char* pa = h.cpl_host;
        unsigned char* pb = h.cpl_host + sizeof acc;
        HIP_OK(hipMemcpyAsync(pa, &h.dev.ctl->cnt[p].acc[0][0], sizeof acc, hipMemcpyDeviceToHost, c->stream));
        HIP_OK(hipMemcpyAsync(pb, h.dev.bodies, sizeof(DevBody) * MAXB, hipMemcpyDeviceToHost, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
        std::memcpy(acc, pa, sizeof acc);
        std::memcpy(h.bodies, pb, sizeof(DevBody) * MAXB);
    } else {
        HIP_OK(hipStreamSynchronize(c->stream));
        HIP_OK(hipMemcpy(acc, &h.dev.ctl->cnt[p].acc[0][0], sizeof acc, hipMemcpyDeviceToHost));
        rc = pull_bodies(c, h);
        if (rc) return rc;
    }
    for (int b = 0; b < h.dev.nbodies; ++b) {
        DevBody d = h.bodies[b];
        if (!d.active || !d.free_body || !d.dof) continue;
        double F[3], T[3];
        for (int a = 0; a < 3; ++a) {
            F[a] = d.have_prev ? 0.5 * (acc[b][a] + d.fprev[a]) : acc[b][a];
            T[a] = d.have_prev ? 0.5 * (acc[b][3 + a] + d.fprev[3 + a]) : acc[b][3 + a];
        }
        for (int a = 0; a < 6; ++a) d.fprev[a] = acc[b][a];
        d.have_prev = 1;
        lbm_body in = h.desc[b], out;
        for (int a = 0; a < 3; ++a) {
            in.pos[a] = d.pos[a];
            in.vel[a] = d.vel[a];
            in.omega[a] = d.omega[a];
        }
        for (int a = 0; a < 4; ++a) in.quat[a] = d.quat[a];
        rc = lbm_integrate_body(&in, F, T, h.cfg.accel, d.dof, &out);
        if (rc) return rc;
        const double n[3] = {(double)h.cfg.nx, (double)h.cfg.ny, (double)h.cfg.nz};
        for (int a = 0; a < 3; ++a) {
            double q = out.pos[a];
            if (h.cfg.periodic & (1 << a)) q = q - n[a] * std::floor(q / n[a]);
            d.pos[a] = q;
            d.vel[a] = out.vel[a];
            d.omega[a] = out.omega[a];
        }
        for (int a = 0; a < 4; ++a) d.quat[a] = out.quat[a];
        quat_to_R(d.quat, d.R);
        box_extent(d.shape, d.R, d.half, d.ext);
        rc = check_pose(h, b, d, d.mapped != 0, "free-body update (host)");
        if (rc) return fail(LBM_ERR_UNSTABLE, lbm_last_error());
        d.moved = 1;
        h.bodies[b] = d;
        launch_set_body(h.dev, b, d, c->stream);
    }
    HIP_OK(hipGetLastError());
    h.need_remap = true;
    return LBM_OK;
}

static int timing_events(lbm_ctx* c, hipEvent_t e[4]) {
    for (int q = 0; q < 4; ++q) e[q] = nullptr;
    if (!c->timing) return LBM_OK;
    for (int q = 0; q < 4; ++q) {
        e[q] = next_event(c);
        if (!e[q]) return fail(LBM_ERR_DEVICE, "kernel timing: event creation failed");
    }
    return LBM_OK;
}

// Each instance's bulk grid cut to its layer bound: the offsets to pass by
// value and the layer counts.  False (all layers) in a capture, beyond
// BATCH_OFF_MAX instances, or if the instances' step counts differ.
static bool batch_cut(lbm_ctx* c, BatchOff& hoff, std::vector<int>& layers) {
    const int n = c->n_inst;
    bool cut = !c->capturing && n <= BATCH_OFF_MAX;
    for (int k = 1; k < n && cut; ++k) cut = c->inst[k].steps == c->inst[0].steps;
    if (!cut) return false;
    hoff.off[0] = 0;
    for (int k = 0; k < n; ++k) {
        layers[k] = layer_bound(c, c->inst[k]);
        hoff.off[k + 1] = hoff.off[k] + bulk_blocks(c->inst[k].dev, c->tile_x, layers[k]);
    }
    return true;
}

// A full step of a batched context: every kernel runs once for all
// instances (remap and conversions in groups of 64 instances).
static int run_step_batched(lbm_ctx* c) {
    const int p = c->parity;
    const int n = c->n_inst;
    const int storage = c->inst[0].cfg.storage;
    std::vector<unsigned char> remapped(n, 0), integrate(n, 0);
    for (int g = 0; g < n; g += 64) {
        const int ng = std::min(64, n - g);
        int bpb = 0, maxb = 0;
        bool any = false;
        for (int k = g; k < g + ng; ++k) {
            InstHost& h = c->inst[k];
            if (!h.need_remap) continue;
            any = true;
            bpb = std::max(bpb, h.remap_blocks);
            maxb = std::max(maxb, h.dev.nbodies);
            remapped[k] = 1;
            h.need_remap = false;
        }
        if (any) launch_remap_batch(c->d_tab + g, ng, maxb, storage, p, bpb, c->stream);
    }
    hipEvent_t e[4];
    int rc = timing_events(c, e);
    if (rc) return rc;
    std::vector<int> layers(n, 0);
    BatchOff hoff;
    const bool cut = batch_cut(c, hoff, layers);
    BatchGrid bulk{c->d_tab, c->d_bulk_off, n, c->bulk_total};
    if (cut) bulk.hoff = &hoff;
    launch_sweep_bulk_batch(bulk, storage, c->tile_x, c->nt_store, p, c->stream, e[0], e[1]);
    bool tension = false;
    for (int k = 0; k < n; ++k) tension |= c->inst[k].dev.lap != 0.f;
    if (tension) launch_curvature_batch(BatchGrid{c->d_tab, c->d_bnd_off, n, c->bnd_total}, p, c->stream);
    launch_sweep_boundary_batch(BatchGrid{c->d_tab, c->d_bnd_off, n, c->bnd_total, c->bnd_fits}, storage, p, c->bnd_layout,
                                c->stream, e[2], e[3]);
    for (int g = 0; g < n; g += 64) {
        const int ng = std::min(64, n - g);
        unsigned long long rm = 0, im = 0;
        int blocks = 0;
        for (int k = g; k < g + ng; ++k) {
            InstHost& h = c->inst[k];
            integrate[k] = h.any_free && h.cfg.host_body_update == 0;
            if (remapped[k]) rm |= 1ull << (k - g);
            if (integrate[k]) im |= 1ull << (k - g);
            blocks = std::max(blocks, conv_blocks(h.dev));
        }
        launch_convert_batch(c->d_tab + g, ng, blocks, storage, p, rm, im, c->stream,
                             cut ? (unsigned)c->inst[0].steps : NO_STEP_TAG, cut ? layers.data() + g : nullptr);
    }
    for (int k = 0; k < n; ++k)
        if (integrate[k]) c->inst[k].need_remap = true;  // the device moved free bodies
    HIP_OK(hipGetLastError());
    c->last_parity = p;
    c->have_forces = true;
    c->parity ^= 1;
    for (InstHost& h : c->inst) ++h.steps;
    for (int k = 0; k < n; ++k) {
        InstHost& h = c->inst[k];
        if (!h.any_free || h.cfg.host_body_update == 0) continue;
        rc = couple_on_host(c, h, p);
        if (rc) return rc;
    }
    return LBM_OK;
}

static int run_step(lbm_ctx* c, int mask) {
    if (c->batched && mask == LBM_PHASE_ALL) return run_step_batched(c);
    const int p = c->parity;
    const bool advances = (mask & (LBM_PHASE_SWEEP | LBM_PHASE_CONVERT)) != 0;
    for (int k = 0; k < c->n_inst; ++k) {
        InstHost& h = c->inst[k];
        bool remapped = false;
        int layers = 0;  // of the bulk grid (0: all)
        if ((mask & LBM_PHASE_REMAP) && h.need_remap) {
            launch_remap(h.dev, p, h.remap_blocks, c->stream);
            h.need_remap = false;
            remapped = true;
        }
        if (mask & LBM_PHASE_SWEEP) {
            hipEvent_t e[4];
            int rc = timing_events(c, e);
            if (rc) return rc;
            // a full step outside a capture launches the layers its bound needs
            layers = mask == LBM_PHASE_ALL && !c->capturing ? layer_bound(c, h) : 0;
            launch_sweep_bulk(h.dev, p, c->tile_x, c->nt_store, c->stream, e[0], e[1], layers);
            if (h.dev.lap != 0.f) launch_curvature(h.dev, p, c->stream);
            launch_sweep_boundary(h.dev, p, c->bnd_layout, c->stream, e[2], e[3]);
        } else if (mask & LBM_PHASE_CONVERT) {
            hipLaunchKernelGGL(k_copy_state, dim3((h.dev.N + 255) / 256), dim3(256), 0, c->stream, h.dev, p);
            launch_mark(h.dev, p, c->stream);
        }
        const bool integrate = mask == LBM_PHASE_ALL && h.any_free && h.cfg.host_body_update == 0;
        if (mask & LBM_PHASE_CONVERT)
            launch_convert(h.dev, p, remapped, integrate, c->stream,
                           mask == LBM_PHASE_ALL && !c->capturing ? (unsigned)h.steps : NO_STEP_TAG, layers);
        else if (advances || remapped)
            launch_finish(h.dev, p, (mask & LBM_PHASE_SWEEP) != 0, advances, remapped, c->stream);
        // free bodies moved on the device: the next step maps them
        if (integrate) h.need_remap = true;
    }
    HIP_OK(hipGetLastError());
    if (advances) {
        c->last_parity = p;
        c->have_forces = (mask & LBM_PHASE_SWEEP) != 0;
        c->parity ^= 1;
        for (InstHost& h : c->inst) ++h.steps;
    }
    if (mask == LBM_PHASE_ALL)
        for (int k = 0; k < c->n_inst; ++k) {
            InstHost& h = c->inst[k];
            if (!h.any_free || h.cfg.host_body_update == 0) continue;
            int rc = couple_on_host(c, h, p);
            if (rc) return rc;
        }
    return LBM_OK;
}

// Two full steps can be replayed from a graph when no instance needs the
// host between steps and the host-side state the launches depend on (parity
// and which instances remap) repeats after two steps: free bodies remap
// every step, held ones never after their first.
static bool graph_replayable(lbm_ctx* c) {
    if (!c->use_graph || c->timing) return false;
    for (const InstHost& h : c->inst) {
        if (h.any_free && h.cfg.host_body_update != 0) return false;
        if (h.need_remap != (h.any_free && h.cfg.host_body_update == 0)) return false;
    }
    return true;
}

static int graph_two_steps(lbm_ctx* c) {
    std::vector<unsigned char> rm(c->n_inst);
    for (int k = 0; k < c->n_inst; ++k) rm[k] = c->inst[k].need_remap;
    if (!c->gexec || c->gparity != c->parity || c->gremap != rm) {
        drop_graph(c);
        if (!c->cap_stream) HIP_OK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        // the two steps are launched into the capture; the host-side state
        // advances as if they ran, and the graph launch below runs them
        const int p0 = c->parity;
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        c->capturing = true;  // all layers, no bound reports: the graph replays with any state
        int rc = e == hipSuccess ? run_step(c, LBM_PHASE_ALL) : LBM_OK;
        if (e == hipSuccess && rc == LBM_OK) rc = run_step(c, LBM_PHASE_ALL);
        c->capturing = false;
        hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(c->cap_stream, &g) : e;
        c->stream = user;
        if (e != hipSuccess || e2 != hipSuccess)
            return fail(LBM_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
        if (rc) {
            (void)hipGraphDestroy(g);
            return rc;
        }
        e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->gexec = nullptr;
            return fail(LBM_ERR_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        c->gparity = p0;
        c->gremap = rm;
    } else {
        // replay: the host-side state after two steps
        c->last_parity = c->parity ^ 1;
        c->have_forces = true;
        for (InstHost& h : c->inst) h.steps += 2;
    }
    HIP_OK(hipGraphLaunch(c->gexec, c->stream));
    return LBM_OK;
}

int32_t lbm_step(lbm_ctx* c, int32_t nsteps) {
    if (!c) return fail(LBM_ERR_INVALID, "context is NULL");
    if (nsteps < 0) return fail(LBM_ERR_INVALID, "step: nsteps < 0");
    int s = 0;
    while (s < nsteps) {
        int rc;
        if (nsteps - s >= 2 && graph_replayable(c)) {
            rc = graph_two_steps(c);
            s += 2;
        } else {
            rc = run_step(c, LBM_PHASE_ALL);
            s += 1;
        }
        if (rc) return rc;
    }
    return LBM_OK;
}

// zero the boundary-list count (and overflow flag) of the current parity
__global__ void k_reset_bnd(Ctl* ctl, int parity) {
    if (threadIdx.x == 0) {
        ctl->cnt[parity].n_bnd = 0;
        ctl->cnt[parity].overflow = 0;
    }
}

int32_t lbm_set_tuning(lbm_ctx* c, int32_t tile_x, int32_t batched, int32_t use_graph, int32_t stream_store,
                       int32_t boundary_layout) {
    if (!c) return fail(LBM_ERR_INVALID, "context is NULL");
    if (tile_x != 0 && tile_x != 32 && tile_x != 64 && tile_x != 128)
        return fail(LBM_ERR_INVALID, "set_tuning: tile_x must be 0, 32, 64 or 128");
    if (stream_store != 0 && stream_store != 1) return fail(LBM_ERR_INVALID, "set_tuning: stream_store must be 0 or 1");
    if (boundary_layout != 0 && boundary_layout != 1)
        return fail(LBM_ERR_INVALID, "set_tuning: boundary_layout must be 0 or 1");
    if (batched) {
        for (int k = 1; k < c->n_inst; ++k)
            if (c->inst[k].cfg.storage != c->inst[0].cfg.storage)
                return fail(LBM_ERR_INVALID, "set_tuning: a batch needs one storage type");
    }
    HIP_OK(hipStreamSynchronize(c->stream));
    drop_graph(c);
    c->tile_x = tile_x;
    c->nt_store = stream_store != 0;
    c->bnd_layout = boundary_layout;
    c->batched = batched != 0 && c->n_inst > 1;
    c->use_graph = use_graph != 0;
    return upload_batch(c);
}

int32_t lbm_get_tuning(lbm_ctx* c, int32_t* tile_x, int32_t* batched, int32_t* use_graph, int32_t* stream_store,
                       int32_t* boundary_layout) {
    if (!c) return fail(LBM_ERR_INVALID, "context is NULL");
    if (tile_x) *tile_x = c->tile_x;
    if (batched) *batched = c->batched ? 1 : 0;
    if (use_graph) *use_graph = c->use_graph ? 1 : 0;
    if (stream_store) *stream_store = c->nt_store ? 1 : 0;
    if (boundary_layout) *boundary_layout = c->bnd_layout;
    return LBM_OK;
}

// Times the boundary sweep of the current state with both work layouts and
// keeps the faster.  The sweep updates the interface cells' mass and marks in
// place and appends to the step counters, so those are saved after one bulk
// sweep (which lists the cells) and restored after every launch.  Without
// room for the copies the layout stays as it is (out_ms < 0).
static int tune_boundary(lbm_ctx* c, int reps, hipEvent_t e0, hipEvent_t e1, double* out_ms) {
    *out_ms = -1.0;
    const int p = c->parity;
    const int n = c->n_inst;
    std::vector<char*> saved(n, nullptr);
    auto cnt_of = [&](int k) { return (void*)&c->inst[k].dev.ctl->cnt[p]; };
    auto off = [&](int k) { return ((size_t)c->inst[k].dev.N * 9 + 255) / 256 * 256; };
    bool room = true;
    for (int k = 0; k < n && room; ++k)
        room = hipMalloc((void**)&saved[k], off(k) + sizeof(StepCounters)) == hipSuccess;
    (void)hipGetLastError();
    int rc = LBM_OK;
    auto copies = [&](bool save) {
        for (int k = 0; k < n; ++k) {
            const Inst& I = c->inst[k].dev;
            const size_t N = (size_t)I.N;
            void* dev[4] = {I.m_hi, I.m_lo, I.flags, cnt_of(k)};
            void* keep[4] = {saved[k], saved[k] + 4 * N, saved[k] + 8 * N, saved[k] + off(k)};
            const size_t bytes[4] = {4 * N, 4 * N, N, sizeof(StepCounters)};
            for (int q = 0; q < 4; ++q)
                (void)hipMemcpyAsync(save ? keep[q] : dev[q], save ? dev[q] : keep[q], bytes[q],
                                     hipMemcpyDeviceToDevice, c->stream);
        }
    };
    const BatchGrid bnd{c->d_tab, c->d_bnd_off, n, c->bnd_total, c->bnd_fits};
    auto boundary = [&](hipEvent_t a, hipEvent_t b) {
        if (c->batched) launch_sweep_boundary_batch(bnd, c->inst[0].cfg.storage, p, c->bnd_layout, c->stream, a, b);
        else
            for (InstHost& h : c->inst) launch_sweep_boundary(h.dev, p, c->bnd_layout, c->stream, a, b);
    };
    if (room) {
        // the state a step's boundary sweep starts from
        if (c->batched) {
            launch_sweep_bulk_batch(BatchGrid{c->d_tab, c->d_bulk_off, n, c->bulk_total}, c->inst[0].cfg.storage,
                                    c->tile_x, c->nt_store, p, c->stream);
            bool tension = false;
            for (int k = 0; k < n; ++k) tension |= c->inst[k].dev.lap != 0.f;
            if (tension) launch_curvature_batch(bnd, p, c->stream);
        } else {
            for (InstHost& h : c->inst) {
                launch_sweep_bulk(h.dev, p, c->tile_x, c->nt_store, c->stream);
                if (h.dev.lap != 0.f) launch_curvature(h.dev, p, c->stream);
            }
        }
        copies(true);
        const int keep = c->bnd_layout;
        double best_t = 1e30;
        int best = keep;
        for (int layout = 0; layout < 2 && rc == LBM_OK; ++layout) {
            c->bnd_layout = layout;
            boundary(nullptr, nullptr);
            copies(false);
            double total = 0.0;
            for (int r = 0; r < reps && rc == LBM_OK; ++r) {
                if (hipEventRecord(e0, c->stream) != hipSuccess) rc = fail(LBM_ERR_DEVICE, "autotune: event failed");
                boundary(nullptr, nullptr);
                if (hipEventRecord(e1, c->stream) != hipSuccess) rc = fail(LBM_ERR_DEVICE, "autotune: event failed");
                copies(false);
                float ms = 0.f;
                if (rc == LBM_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = fail(LBM_ERR_DEVICE, "autotune: timing failed");
                total += ms;
            }
            if (rc == LBM_OK && hipGetLastError() != hipSuccess) rc = fail(LBM_ERR_DEVICE, "autotune: launch failed");
            if (rc == LBM_OK && total / reps < best_t) {
                best_t = total / reps;
                best = layout;
            }
        }
        c->bnd_layout = rc == LBM_OK ? best : keep;
        if (rc == LBM_OK) *out_ms = best_t;
        // the list count back to the start of the step
        for (InstHost& h : c->inst) hipLaunchKernelGGL(k_reset_bnd, dim3(1), dim3(64), 0, c->stream, h.dev.ctl, p);
        if (hipStreamSynchronize(c->stream) != hipSuccess && rc == LBM_OK) rc = fail(LBM_ERR_DEVICE, "autotune: sync failed");
    }
    for (char* q : saved)
        if (q) (void)hipFree(q);
    return rc;
}

int32_t lbm_autotune(lbm_ctx* c, int32_t reps, int32_t* tile_x, int32_t* stream_store, int32_t* boundary_layout,
                     double* bulk_ms, double* boundary_ms) {
    if (!c) return fail(LBM_ERR_INVALID, "context is NULL");
    if (reps <= 0 || reps > 64) return fail(LBM_ERR_INVALID, "autotune: reps must be 1..64");
    HIP_OK(hipStreamSynchronize(c->stream));
    drop_graph(c);
    const int p = c->parity;
    const int widths[4] = {32, 64, 128, 0};
    int best = c->tile_x;
    bool best_nt = c->nt_store;
    double best_t = 1e30;
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    int rc = LBM_OK;
    // Each candidate sweeps the current state (reads parity p, writes the
    // other lattice, which the next step overwrites); the boundary-list
    // counts it appends to are reset after every launch.
    auto reset = [&]() {
        for (InstHost& h : c->inst) hipLaunchKernelGGL(k_reset_bnd, dim3(1), dim3(64), 0, c->stream, h.dev.ctl, p);
    };
    // the candidates sweep the grids the steps launch (cut to the layer bounds)
    auto sweep = [&]() {
        if (c->batched) {
            std::vector<int> layers(c->n_inst, 0);
            BatchOff hoff;
            BatchGrid bulk{c->d_tab, c->d_bulk_off, c->n_inst, c->bulk_total};
            if (batch_cut(c, hoff, layers)) bulk.hoff = &hoff;
            launch_sweep_bulk_batch(bulk, c->inst[0].cfg.storage, c->tile_x, c->nt_store, p, c->stream);
        } else {
            for (InstHost& h : c->inst)
                launch_sweep_bulk(h.dev, p, c->tile_x, c->nt_store, c->stream, nullptr, nullptr, layer_bound(c, h));
        }
    };
    // Streaming-store candidates only where a step's populations exceed the
    // cache: below it, repeated sweeps of one source favour them (their
    // writes leave that source cached, while a step's next source, written
    // with streaming stores, is not).
    const double moved = moved_bytes(c);
    const bool try_nt = moved > CACHE_BYTES;
    c->max_lag = lag_limit(moved);
    for (int cand = 0; cand < 8 && rc == LBM_OK; ++cand) {
        if (cand >= 4 && !try_nt) break;
        c->tile_x = widths[cand % 4];
        c->nt_store = cand >= 4;
        rc = upload_batch(c);
        if (rc) break;
        sweep();
        reset();
        float total = 0.f;
        for (int r = 0; r < reps; ++r) {
            if (hipEventRecord(e0, c->stream) != hipSuccess) break;
            sweep();
            if (hipEventRecord(e1, c->stream) != hipSuccess) break;
            reset();
            float ms = 0.f;
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) break;
            total += ms;
        }
        if (hipGetLastError() != hipSuccess) {
            rc = fail(LBM_ERR_DEVICE, "autotune: launch failed");
            break;
        }
        const double avg = total / reps;
        if (avg < best_t) {
            best_t = avg;
            best = c->tile_x;
            best_nt = c->nt_store;
        }
    }
    c->tile_x = best;
    c->nt_store = best_nt;
    if (rc == LBM_OK) rc = upload_batch(c);
    double bnd_t = -1.0;
    if (rc == LBM_OK) rc = tune_boundary(c, reps, e0, e1, &bnd_t);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == LBM_OK && tile_x) *tile_x = best;
    if (rc == LBM_OK && stream_store) *stream_store = best_nt ? 1 : 0;
    if (rc == LBM_OK && boundary_layout) *boundary_layout = c->bnd_layout;
    if (rc == LBM_OK && bulk_ms) *bulk_ms = best_t;
    if (rc == LBM_OK && boundary_ms) *boundary_ms = bnd_t;
    return rc;
}

int32_t lbm_step_phases(lbm_ctx* c, int32_t mask) {
    if (!c) return fail(LBM_ERR_INVALID, "context is NULL");
    if (mask <= 0 || mask > LBM_PHASE_ALL) return fail(LBM_ERR_INVALID, "step_phases: bad mask");
    return run_step(c, mask);
}

static int sync_and_check(lbm_ctx* c) {
    HIP_OK(hipStreamSynchronize(c->stream));
    for (int k = 0; k < c->n_inst; ++k) {
        int flags[2] = {0, 0};
        Ctl* ctl = c->inst[k].dev.ctl;
        HIP_OK(hipMemcpy(&flags[0], &ctl->nonfinite, sizeof(int), hipMemcpyDeviceToHost));
        int ov[2];
        HIP_OK(hipMemcpy(&ov[0], &ctl->cnt[0].overflow, sizeof(int), hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(&ov[1], &ctl->cnt[1].overflow, sizeof(int), hipMemcpyDeviceToHost));
        int berr = 0;
        HIP_OK(hipMemcpy(&berr, &ctl->body_err, sizeof(int), hipMemcpyDeviceToHost));
        if (flags[0] & NONFINITE_LAYERS)
            return fail(LBM_ERR_DEVICE, "bulk sweep: a launch's layer bound missed a layer holding fluid");
        if (flags[0]) return fail(LBM_ERR_UNSTABLE, "non-finite or non-positive density detected");
        if (berr) {
            std::string why;
            if (berr & BODY_ERR_WALL) why += " left the domain interior;";
            if (berr & BODY_ERR_SPEED) why += " surface speed reached one cell per step;";
            if (berr & BODY_ERR_CLOSE) why += " bodies closer than three cells;";
            if (berr & BODY_ERR_JUMP) why += " moved a cell from its mapping;";
            return fail(LBM_ERR_UNSTABLE, "free-body update rejected:" + why);
        }
        if (ov[0] || ov[1]) return fail(LBM_ERR_UNSTABLE, "conversion list overflow");
    }
    return LBM_OK;
}

int32_t lbm_sync(lbm_ctx* c) {
    if (!c) return fail(LBM_ERR_INVALID, "context is NULL");
    return sync_and_check(c);
}

int32_t lbm_enable_kernel_timing(lbm_ctx* c, int32_t enable) {
    if (!c) return fail(LBM_ERR_INVALID, "context is NULL");
    HIP_OK(hipStreamSynchronize(c->stream));
    c->timing = enable != 0;
    c->ev_used = 0;
    return LBM_OK;
}

int32_t lbm_kernel_time(lbm_ctx* c, int32_t kernel, double* total_ms, int64_t* launches) {
    if (!c || !total_ms || !launches) return fail(LBM_ERR_INVALID, "kernel_time: bad arguments");
    if (kernel < 0 || kernel > 2) return fail(LBM_ERR_INVALID, "kernel_time: unknown kernel id");
    HIP_OK(hipStreamSynchronize(c->stream));
    // four events per timed sweep: bulk start / end, boundary start / end
    double tot = 0.0;
    for (size_t k = 0; k + 3 < c->ev_used; k += 4) {
        float ms = 0.f;
        if (kernel != 1) {
            HIP_OK(hipEventElapsedTime(&ms, c->ev_pool[k], c->ev_pool[k + 1]));
            tot += ms;
        }
        if (kernel != 0) {
            HIP_OK(hipEventElapsedTime(&ms, c->ev_pool[k + 2], c->ev_pool[k + 3]));
            tot += ms;
        }
    }
    *total_ms = tot;
    *launches = (int64_t)(c->ev_used / 4);
    return LBM_OK;
}

int32_t lbm_boundary_cells(lbm_ctx* c, int32_t inst, int64_t* n) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    if (!n) return fail(LBM_ERR_INVALID, "boundary_cells: NULL output");
    HIP_OK(hipStreamSynchronize(c->stream));
    int v = 0;
    HIP_OK(hipMemcpy(&v, &c->inst[inst].dev.ctl->cnt[c->last_parity].n_bnd, sizeof(int), hipMemcpyDeviceToHost));
    *n = v;
    return LBM_OK;
}

int32_t lbm_body_forces(lbm_ctx* c, int32_t inst, int32_t k, double force[3], double torque[3]) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    InstHost& h = c->inst[inst];
    if (k < 0 || k >= h.dev.nbodies || !h.bodies[k].active) return fail(LBM_ERR_INVALID, "body_forces: no such body");
    if (!force || !torque) return fail(LBM_ERR_INVALID, "body_forces: NULL output");
    HIP_OK(hipStreamSynchronize(c->stream));
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (c->have_forces)
        HIP_OK(hipMemcpy(v, &h.dev.ctl->cnt[c->last_parity].acc[k][0], sizeof v, hipMemcpyDeviceToHost));
    for (int a = 0; a < 3; ++a) {
        force[a] = v[a];
        torque[a] = v[3 + a];
    }
    return LBM_OK;
}

int32_t lbm_conversion_counts(lbm_ctx* c, int32_t inst, int64_t counts[4]) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(c->stream));
    StepCounters sc;
    HIP_OK(hipMemcpy(&sc, &c->inst[inst].dev.ctl->cnt[c->last_parity], sizeof sc, hipMemcpyDeviceToHost));
    counts[0] = sc.filled;
    counts[1] = sc.emptied;
    counts[2] = sc.newg;
    counts[3] = sc.newl;
    return LBM_OK;
}

int32_t lbm_mass_total(lbm_ctx* c, int32_t inst, double* total, double* ledger) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    const Inst& I = c->inst[inst].dev;
    launch_mass_total(I, c->parity, I.mass_part, &I.ctl->mass_total, c->stream);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(c->stream));
    double v[2];
    HIP_OK(hipMemcpy(&v[0], &I.ctl->mass_total, sizeof(double), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&v[1], &I.ctl->ledger, sizeof(double), hipMemcpyDeviceToHost));
    if (total) *total = v[0];
    if (ledger) *ledger = v[1];
    return LBM_OK;
}

int32_t lbm_mass_total_noalloc(lbm_ctx* c, int32_t inst, double* total, double* ledger) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    const Inst& I = c->inst[inst].dev;
    if (mass_parts(I.N) > MASS_PARTS_MAX)
        return fail(LBM_ERR_INVALID, "mass_total_noalloc: more than " + std::to_string((long long)MASS_PARTS_MAX * MASS_CHUNK) +
                                         " cells (the static scratch holds " + std::to_string(MASS_PARTS_MAX) +
                                         " partial sums); use lbm_mass_total");
    double* sp = scratch_of(c->device);
    if (!sp) return fail(LBM_ERR_STATE, "mass_total_noalloc: scratch of the context's device not set up");
    launch_mass_total(I, c->parity, sp, sp + MASS_PARTS_MAX, c->stream);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(c->stream));
    double v[2];
    HIP_OK(hipMemcpy(&v[0], sp + MASS_PARTS_MAX, sizeof(double), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(&v[1], &I.ctl->ledger, sizeof(double), hipMemcpyDeviceToHost));
    if (total) *total = v[0];
    if (ledger) *ledger = v[1];
    return LBM_OK;
}

int32_t lbm_set_ledger(lbm_ctx* c, int32_t inst, double ledger) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(c->stream));
    HIP_OK(hipMemcpy(&c->inst[inst].dev.ctl->ledger, &ledger, sizeof(double), hipMemcpyHostToDevice));
    return LBM_OK;
}

int32_t lbm_liq_gas_contacts(lbm_ctx* c, int32_t inst, int64_t* contacts) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    const Inst& I = c->inst[inst].dev;
    launch_contacts(I, c->stream);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(c->stream));
    unsigned long long v = 0;
    HIP_OK(hipMemcpy(&v, &I.ctl->contacts, sizeof v, hipMemcpyDeviceToHost));
    *contacts = (int64_t)v;
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// field I/O (host side conversion; not on the hot path)
// ---------------------------------------------------------------------------
static double wq(int i) { return wgtd(i); }

static float half_to_float(uint16_t h) {
    __half v;
    memcpy(&v, &h, 2);
    return __half2float(v);
}
static uint16_t float_to_half(float f) {
    __half v = __float2half(f);
    uint16_t h;
    memcpy(&h, &v, 2);
    return h;
}
static float bf16_to_float(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}
static uint16_t float_to_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (uint16_t)(u >> 16);
}

int32_t lbm_read_fields(lbm_ctx* c, int32_t inst, int32_t field, int32_t dtype, void* dst, size_t bytes) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    const InstHost& h = c->inst[inst];
    const Inst& I = h.dev;
    const size_t N = (size_t)I.N;
    const int p = c->parity;
    size_t comps = field == LBM_FIELD_POP ? Q : (field == LBM_FIELD_VEL ? 3 : 1);
    size_t esz = dtype == LBM_F64 ? 8 : (dtype == LBM_F32 ? 4 : 1);
    if (field == LBM_FIELD_FLAGS ? dtype != LBM_U8 : dtype == LBM_U8)
        return fail(LBM_ERR_INVALID, "read_fields: dtype does not fit the field");
    if (!dst || bytes != N * comps * esz) return fail(LBM_ERR_INVALID, "read_fields: wrong byte count");
    HIP_OK(hipStreamSynchronize(c->stream));
    auto put = [&](size_t k, double v) {
        if (dtype == LBM_F64) ((double*)dst)[k] = v;
        else ((float*)dst)[k] = (float)v;
    };
    if (field == LBM_FIELD_FLAGS) {
        HIP_OK(hipMemcpy(dst, I.flags, N, hipMemcpyDeviceToHost));
        for (size_t k = 0; k < N; ++k) ((uint8_t*)dst)[k] &= KEEP_MASK;
        return LBM_OK;
    }
    if (field == LBM_FIELD_PHI || field == LBM_FIELD_MASS) {
        std::vector<float> a(N), b(N);
        if (field == LBM_FIELD_PHI) {
            HIP_OK(hipMemcpy(a.data(), I.phi[p], 4 * N, hipMemcpyDeviceToHost));
            for (size_t k = 0; k < N; ++k) put(k, a[k]);
        } else {
            HIP_OK(hipMemcpy(a.data(), I.m_hi, 4 * N, hipMemcpyDeviceToHost));
            HIP_OK(hipMemcpy(b.data(), I.m_lo, 4 * N, hipMemcpyDeviceToHost));
            for (size_t k = 0; k < N; ++k) put(k, (double)a[k] + (double)b[k]);
        }
        return LBM_OK;
    }
    if (field != LBM_FIELD_POP && field != LBM_FIELD_RHO && field != LBM_FIELD_VEL)
        return fail(LBM_ERR_INVALID, "read_fields: unknown field");
    const size_t sb = storage_bytes(I.storage);
    std::vector<char> raw(Q * N * sb);
    // planes are ps apart on the device, N apart here
    HIP_OK(hipMemcpy2D(raw.data(), N * sb, I.pop[p], I.ps * sb, N * sb, Q, hipMemcpyDeviceToHost));
    auto dev = [&](int i, size_t k) -> double {
        const size_t j = (size_t)i * N + k;
        if (I.storage == LBM_FP32) return (double)((const float*)raw.data())[j];
        if (I.storage == LBM_FP16_DEV) return (double)half_to_float(((const uint16_t*)raw.data())[j]) / I.scale;
        return (double)bf16_to_float(((const uint16_t*)raw.data())[j]);
    };
    if (field == LBM_FIELD_POP) {
        for (int i = 0; i < Q; ++i)
            for (size_t k = 0; k < N; ++k) put((size_t)i * N + k, wq(i) + dev(i, k));
        return LBM_OK;
    }
    for (size_t k = 0; k < N; ++k) {
        double r = 0, j0 = 0, j1 = 0, j2 = 0;
        for (int i = 0; i < Q; ++i) {
            const double f = wq(i) + dev(i, k);
            r += f;
            j0 += cx(i) * f;
            j1 += cy(i) * f;
            j2 += cz(i) * f;
        }
        if (field == LBM_FIELD_RHO) {
            put(k, r);
        } else {
            const double ir = r != 0 ? 1.0 / r : 0.0;
            put(k, j0 * ir);
            put(N + k, j1 * ir);
            put(2 * N + k, j2 * ir);
        }
    }
    return LBM_OK;
}

// Near marks of written cell types (a, masked): 1 for every cell with a gas
// or obstacle cell among its 18 neighbours (periodic images included, walls
// not).  Written types may leave liquid next to gas, which the conversions
// never do; the bulk sweep checks the sources of exactly the marked cells.
static std::vector<uint8_t> near_marks(const Inst& I, const std::vector<uint8_t>& a) {
    const int n[3] = {I.nx, I.ny, I.nz};
    std::vector<uint8_t> m(a.size(), 0);
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                const size_t id = (size_t)x + (size_t)n[0] * ((size_t)y + (size_t)n[1] * z);
                for (int i = 1; i < Q && !m[id]; ++i) {
                    int c[3] = {x + cx(i), y + cy(i), z + cz(i)};
                    bool wall = false;
                    for (int k = 0; k < 3; ++k) {
                        if (c[k] >= 0 && c[k] < n[k]) continue;
                        if ((I.periodic >> k) & 1u) c[k] = (c[k] + n[k]) % n[k];
                        else wall = true;
                    }
                    if (wall) continue;
                    const int t = a[(size_t)c[0] + (size_t)n[0] * ((size_t)c[1] + (size_t)n[1] * c[2])] & TYPE_MASK;
                    if (t == GAS || t == OBS) m[id] = 1;
                }
            }
    return m;
}

int32_t lbm_write_fields(lbm_ctx* c, int32_t inst, int32_t field, int32_t dtype, const void* src, size_t bytes) {
    int rc = check_inst(c, inst);
    if (rc) return rc;
    InstHost& h = c->inst[inst];
    const Inst& I = h.dev;
    const size_t N = (size_t)I.N;
    const int p = c->parity;
    size_t comps = field == LBM_FIELD_POP ? Q : 1;
    size_t esz = dtype == LBM_F64 ? 8 : (dtype == LBM_F32 ? 4 : 1);
    if (field == LBM_FIELD_FLAGS ? dtype != LBM_U8 : dtype == LBM_U8)
        return fail(LBM_ERR_INVALID, "write_fields: dtype does not fit the field");
    if (!src || bytes != N * comps * esz) return fail(LBM_ERR_INVALID, "write_fields: wrong byte count");
    auto get = [&](size_t k) -> double {
        return dtype == LBM_F64 ? ((const double*)src)[k] : (double)((const float*)src)[k];
    };
    HIP_OK(hipStreamSynchronize(c->stream));
    if (field == LBM_FIELD_FLAGS) {
        std::vector<uint8_t> a((const uint8_t*)src, (const uint8_t*)src + N);
        for (size_t k = 0; k < N; ++k) {
            a[k] &= KEEP_MASK;
            if ((a[k] & TYPE_MASK) == OBS) {
                const int b = (a[k] >> 2) & 15;
                if (b >= h.dev.nbodies || !h.bodies[b].active)
                    return fail(LBM_ERR_INVALID, "write_fields: obstacle cell of an unknown body");
            } else {
                a[k] &= TYPE_MASK;
            }
        }
        HIP_OK(hipMemcpy(I.flags, a.data(), N, hipMemcpyHostToDevice));
        int ztop = 0;  // highest layer with a liquid or interface cell (the marks were dropped)
        for (size_t k = 0; k < N; ++k)
            if ((a[k] & TYPE_MASK) == LIQ || (a[k] & TYPE_MASK) == IFC) ztop = (int)(k / ((size_t)I.nx * I.ny));
        HIP_OK(hipMemcpy(&I.ctl->ztop, &ztop, sizeof(int), hipMemcpyHostToDevice));
        if (h.zpin_host) *(volatile unsigned long long*)h.zpin_host = ((unsigned long long)(unsigned)h.steps << 32) | (unsigned)ztop;
        const std::vector<uint8_t> nm = near_marks(I, a);
        HIP_OK(hipMemcpy(I.nearo, nm.data(), N, hipMemcpyHostToDevice));
        // the written obstacle cells are the bodies' mappings at their poses
        rc = pull_bodies(c, h);
        if (rc) return rc;
        for (int k = 0; k < h.dev.nbodies; ++k) {
            DevBody& d = h.bodies[k];
            if (!d.active) continue;
            d.moved = 0;
            d.mapped = 1;
            for (int a2 = 0; a2 < 3; ++a2) {
                d.prev_pos[a2] = d.pos[a2];
                d.prev_ext[a2] = d.ext[a2];
            }
            launch_set_body(I, k, d, c->stream);
        }
        h.need_remap = false;
        HIP_OK(hipStreamSynchronize(c->stream));
        return LBM_OK;
    }
    if (field == LBM_FIELD_PHI) {
        std::vector<float> a(N);
        for (size_t k = 0; k < N; ++k) a[k] = (float)get(k);
        HIP_OK(hipMemcpy(I.phi[p], a.data(), 4 * N, hipMemcpyHostToDevice));
        return LBM_OK;
    }
    if (field == LBM_FIELD_MASS) {
        std::vector<float> a(N), b(N);
        for (size_t k = 0; k < N; ++k) {
            const double m = get(k);
            a[k] = (float)m;
            b[k] = (float)(m - (double)a[k]);
        }
        HIP_OK(hipMemcpy(I.m_hi, a.data(), 4 * N, hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(I.m_lo, b.data(), 4 * N, hipMemcpyHostToDevice));
        return LBM_OK;
    }
    if (field != LBM_FIELD_POP) return fail(LBM_ERR_INVALID, "write_fields: field is read-only or unknown");
    const size_t sb = storage_bytes(I.storage);
    std::vector<char> raw(Q * N * sb);
    for (int i = 0; i < Q; ++i)
        for (size_t k = 0; k < N; ++k) {
            const size_t j = (size_t)i * N + k;
            const double d = get(j) - wq(i);
            if (I.storage == LBM_FP32) ((float*)raw.data())[j] = (float)d;
            else if (I.storage == LBM_FP16_DEV) ((uint16_t*)raw.data())[j] = float_to_half((float)(d * I.scale));
            else ((uint16_t*)raw.data())[j] = float_to_bf16((float)d);
        }
    HIP_OK(hipMemcpy2D(I.pop[p], I.ps * sb, raw.data(), N * sb, N * sb, Q, hipMemcpyHostToDevice));
    return LBM_OK;
}

// ---------------------------------------------------------------------------
// host rigid-body update
// ---------------------------------------------------------------------------
int32_t lbm_integrate_body(const lbm_body* in, const double F[3], const double T[3], const double accel[3],
                           uint32_t dof, lbm_body* out) {
    if (!in || !F || !T || !accel || !out) return fail(LBM_ERR_INVALID, "integrate_body: NULL argument");
    lbm_body o = *in;
    if (in->shape != LBM_SHAPE_CUBOID && in->shape != LBM_SHAPE_SPHERE)
        return fail(LBM_ERR_INVALID, "integrate_body: unknown shape");
    if (!integrate_rigid((int)in->shape, in->half_ext, in->pos, in->quat, in->vel, in->omega, in->density, F, T, accel,
                         dof, o.pos, o.quat, o.vel, o.omega))
        return fail(LBM_ERR_INVALID, "integrate_body: body mass must be positive");
    *out = o;
    return LBM_OK;
}

}  // extern "C"

// copy the current state into the other lattice (conversion-only phase)
__global__ __launch_bounds__(256) void k_copy_state(Inst I, int from) {
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= I.N) return;
    const size_t N = (size_t)I.N;
    const size_t sb = I.storage == LBM_FP32 ? 4 : 2;
    const char* s = (const char*)I.pop[from];
    char* d = (char*)I.pop[from ^ 1];
    for (int i = 0; i < Q; ++i) memcpy(d + ((size_t)i * I.ps + id) * sb, s + ((size_t)i * I.ps + id) * sb, sb);
    I.phi[from ^ 1][id] = I.phi[from][id];
}
