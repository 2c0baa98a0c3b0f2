// lgs_internal.h -- device-side data structures and helpers shared by the
// kernels of the liquid-gas-solid LBM library (gfx950 / CDNA4).
//
// Layout of one lattice instance in device memory (all arrays x fastest,
// cell index id = x + nx (y + ny z), N cells):
//   pop[2]    two population lattices (ping-pong), structure of arrays
//             [19][N] of the storage type, holding the deviation f_i - w_i
//             (FP32) or (f_i - w_i) * scale (FP16) / (f_i - w_i) (BF16)
//   flags     u8[N]: bits 0-1 type, bits 2-5 body of an obstacle cell,
//             bit 6 "filled" and bit 7 "emptied" marks (transient, between
//             the sweep and the end of the conversion phase)
//   phi[2]    f32[N] fill level, ping-pong (neighbours read phi(t))
//   m_hi,m_lo f32[N] interface mass as an unevaluated sum hi + lo
//             (compensated accumulation of the mass exchange)
//   share     f32[N] excess-mass share of converted cells / remap rho
//   aux       f32[N] remap fill level
//   rule      u8[N] remap rule of uncovered cells
//   claim(2)  u32[N/32+1] claim bitmaps for building deduplicated lists
//   lists     i32 boundary-cell / candidate / new-gas / new-liquid / receiver lists
//   ctl       per-instance counters and FP64 accumulators
//   bodies    DevBody[LBM_MAX_BODIES]
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "lgs_lbm.h"

namespace lgs {

constexpr int Q = 19;
constexpr int MAXB = LBM_MAX_BODIES;

enum : uint8_t { GAS = 0, LIQ = 1, IFC = 2, OBS = 3 };
constexpr uint8_t TYPE_MASK = 3;
constexpr uint8_t MARK_FILL = 0x40;
constexpr uint8_t MARK_EMPTY = 0x80;
constexpr uint8_t KEEP_MASK = 0x3F;

// D3Q19 in the order of the caption of Fig. d3q19 (Sec. 2.1):
// C W E N S T B TW TE TN TS NW NE SW SE BW BE BN BS; E = +x, N = +y, T = +z.
__host__ __device__ constexpr int cx(int i) {
    constexpr int v[Q] = {0, -1, 1, 0, 0, 0, 0, -1, 1, 0, 0, -1, 1, -1, 1, -1, 1, 0, 0};
    return v[i];
}
__host__ __device__ constexpr int cy(int i) {
    constexpr int v[Q] = {0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, 1, -1, -1, 0, 0, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int cz(int i) {
    constexpr int v[Q] = {0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, 0, 0, 0, 0, -1, -1, -1, -1};
    return v[i];
}
// opposite direction: pairs (1,2) (3,4) (5,6) and the diagonals
__host__ __device__ constexpr int opp(int i) {
    constexpr int v[Q] = {0, 2, 1, 4, 3, 6, 5, 16, 15, 18, 17, 14, 13, 12, 11, 8, 7, 10, 9};
    return v[i];
}
__host__ __device__ constexpr float wgt(int i) {
    return i == 0 ? 1.0f / 3.0f : (i < 7 ? 1.0f / 18.0f : 1.0f / 36.0f);
}
__host__ __device__ constexpr double wgtd(int i) {
    return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// --------------------------------------------------------------------------
// per-instance control block (device memory)
// --------------------------------------------------------------------------
struct StepCounters {
    int n_cand, n_newg, n_newl, n_recv;
    int filled, emptied, newg, newl;
    int overflow, n_bnd, pad[2];
    double acc[MAXB][6];  // per body: F (3), T (3), FP64
};

struct Ctl {
    StepCounters cnt[2];  // by step parity
    double ledger;
    double mass_total;
    unsigned long long contacts;
    int nonfinite;
    int pad;
};

// Momentum-exchange partial sum of one wavefront of the boundary sweep (over
// its grid-stride loop) for one body (the first body the wavefront touches; further bodies of the same
// wavefront go to the FP64 accumulators with atomics).  Records are summed in
// slot order, so the force / torque sums do not depend on scheduling.
struct ForceRec {
    int body;  // -1: no contribution
    int pad;
    double v[6];
};

// Per-instance record in mapped, coherent host memory: the end-of-step
// kernel writes the body forces of the step, then (after a system-scope
// fence) the step's sequence number, which the host spins on.
struct HostOut {
    double acc[MAXB][6];
    volatile unsigned long long seq;
    unsigned long long pad[7];
};

struct DevBody {
    double pos[3];
    double R[9];  // body -> world, row major
    double half[3];
    double vel[3];
    double omega[3];
    double prev_pos[3];
    double ext[3];  // world-frame half extent of the bounding box
    int active;
    int moved;  // pose changed since the last remap
};

// Everything a kernel needs about one instance (passed by value).
struct Inst {
    int nx, ny, nz, N;
    uint32_t periodic;
    int recon_mode;
    int storage;
    int nbodies;
    float omega;       // 1 / tau
    float ax, ay, az;  // body acceleration
    float rho_g;
    float scale, inv_scale;  // storage scale (FP16), 1 otherwise
    double eps;
    void* pop[2];
    uint8_t* flags;
    float* phi[2];
    float* m_hi;
    float* m_lo;
    float* share;
    float* aux;
    uint8_t* rule;
    uint32_t* claim;   // new-interface claims
    uint32_t* claim2;  // receiver claims
    int* cand;
    int* newg;
    int* newl;
    int* recv;
    int* bnd;  // cells the bulk sweep leaves to the boundary sweep
    ForceRec* frec;  // one record per wavefront of the boundary sweep's grid
    HostOut* hout;   // device view of the mapped host record (or null)
    int list_cap;
    Ctl* ctl;
    DevBody* bodies;
};

// --------------------------------------------------------------------------
// storage types
// --------------------------------------------------------------------------
template <typename S>
struct Store;
// Streaming accesses of the sweep: `load` / `store`; random accesses: `ld` /
// `st`.  LGS_STREAM_NT_LOAD / LGS_STREAM_NT_STORE select non-temporal
// (streaming) cache policy for the sweep's population traffic.
#ifndef LGS_STREAM_NT_LOAD
#define LGS_STREAM_NT_LOAD 0
#endif
#ifndef LGS_STREAM_NT_STORE
#define LGS_STREAM_NT_STORE 0
#endif
template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
#if LGS_STREAM_NT_LOAD
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}
template <typename T>
__device__ __forceinline__ void stream_store(T v, T* p) {
#if LGS_STREAM_NT_STORE
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}

template <>
struct Store<float> {
    __device__ static inline float load(const float* p, size_t k, float) { return stream_load(p + k); }
    __device__ static inline float ld(const float* p, size_t k, float) { return p[k]; }
    __device__ static inline void store(float* p, size_t k, float v, float) { stream_store(v, p + k); }
    __device__ static inline void st(float* p, size_t k, float v, float) { p[k] = v; }
};
// 16-bit storage: the bits are moved as unsigned short so the streaming
// policy applies; conversion is round-to-nearest-even.
__device__ __forceinline__ float h2f(unsigned short b) {
    __half h;
    __builtin_memcpy(&h, &b, 2);
    return __half2float(h);
}
__device__ __forceinline__ unsigned short f2h(float f) {
    __half h = __float2half_rn(f);
    unsigned short b;
    __builtin_memcpy(&b, &h, 2);
    return b;
}
__device__ __forceinline__ float b2f(unsigned short b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ unsigned short f2b(float f) {
    __hip_bfloat16 h = __float2bfloat16(f);
    unsigned short b;
    __builtin_memcpy(&b, &h, 2);
    return b;
}
template <>
struct Store<__half> {
    using U = unsigned short;
    __device__ static inline float load(const __half* p, size_t k, float inv) {
        return h2f(stream_load((const U*)p + k)) * inv;
    }
    __device__ static inline float ld(const __half* p, size_t k, float inv) { return h2f(((const U*)p)[k]) * inv; }
    __device__ static inline void store(__half* p, size_t k, float v, float sc) { stream_store(f2h(v * sc), (U*)p + k); }
    __device__ static inline void st(__half* p, size_t k, float v, float sc) { ((U*)p)[k] = f2h(v * sc); }
};
template <>
struct Store<__hip_bfloat16> {
    using U = unsigned short;
    __device__ static inline float load(const __hip_bfloat16* p, size_t k, float) {
        return b2f(stream_load((const U*)p + k));
    }
    __device__ static inline float ld(const __hip_bfloat16* p, size_t k, float) { return b2f(((const U*)p)[k]); }
    __device__ static inline void store(__hip_bfloat16* p, size_t k, float v, float) {
        stream_store(f2b(v), (U*)p + k);
    }
    __device__ static inline void st(__hip_bfloat16* p, size_t k, float v, float) { ((U*)p)[k] = f2b(v); }
};

// --------------------------------------------------------------------------
// neighbour arithmetic: coordinate of x + d on an axis of length n, or -1
// beyond a wall
// --------------------------------------------------------------------------
__device__ __forceinline__ int step_axis(int x, int d, int n, bool per) {
    int v = x + d;
    if (v < 0) return per ? v + n : -1;
    if (v >= n) return per ? v - n : -1;
    return v;
}

__device__ __forceinline__ int nbr_index(const Inst& I, int x, int y, int z, int dx, int dy, int dz) {
    int X = step_axis(x, dx, I.nx, I.periodic & 1);
    int Y = step_axis(y, dy, I.ny, I.periodic & 2);
    int Z = step_axis(z, dz, I.nz, I.periodic & 4);
    if ((X | Y | Z) < 0) return -1;
    return X + I.nx * (Y + I.ny * Z);
}

__device__ __forceinline__ void cell_coords(const Inst& I, int id, int& x, int& y, int& z) {
    x = id % I.nx;
    int r = id / I.nx;
    y = r % I.ny;
    z = r / I.ny;
}

// minimum image on periodic axes (same operations as the reference code so
// that mapping decisions agree bit for bit)
__host__ __device__ inline double wrap_rel(double d, double L, bool per) {
    if (!per) return d;
    if (d >= 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

// Is the centre of cell (x,y,z) inside body b?  FP64, no contraction.
__device__ inline bool inside_body(const Inst& I, const DevBody& b, int x, int y, int z) {
#pragma clang fp contract(off)
    double d0 = wrap_rel((x + 0.5) - b.pos[0], (double)I.nx, I.periodic & 1);
    double d1 = wrap_rel((y + 0.5) - b.pos[1], (double)I.ny, I.periodic & 2);
    double d2 = wrap_rel((z + 0.5) - b.pos[2], (double)I.nz, I.periodic & 4);
    double r0 = b.R[0] * d0 + b.R[3] * d1 + b.R[6] * d2;
    double r1 = b.R[1] * d0 + b.R[4] * d1 + b.R[7] * d2;
    double r2 = b.R[2] * d0 + b.R[5] * d1 + b.R[8] * d2;
    return fabs(r0) <= b.half[0] && fabs(r1) <= b.half[1] && fabs(r2) <= b.half[2];
}

__device__ inline int body_at(const Inst& I, int x, int y, int z) {
    for (int k = 0; k < I.nbodies; ++k)
        if (I.bodies[k].active && inside_body(I, I.bodies[k], x, y, z)) return k;
    return -1;
}

// Cells a body remap visits: per body an axis-aligned box covering its old
// and new bounding boxes plus two cells (origin lo, extent dim; cells = 0 for
// bodies that did not move).
struct RemapRegions {
    int lo[MAXB][3];
    int dim[MAXB][3];
    int cells[MAXB];
};

// Grid of the boundary sweep (256-thread workgroups, four wavefronts each);
// every wavefront of it writes one force record per step.
constexpr int BND_BLOCKS_MAX = 4096;
__host__ __device__ inline int boundary_blocks(const Inst& I) {
    const int need = (I.N + 255) / 256;
    return need < BND_BLOCKS_MAX ? need : BND_BLOCKS_MAX;
}

// --------------------------------------------------------------------------
// kernel launchers (implemented in the .hip files)
// --------------------------------------------------------------------------
void launch_init(const Inst& I, const lbm_config& c, hipStream_t s);
void launch_sweep_bulk(const Inst& I, int parity, hipStream_t s);
void launch_sweep_boundary(const Inst& I, int parity, hipStream_t s);
void launch_mark(const Inst& I, int parity, hipStream_t s);
void launch_convert(const Inst& I, int parity, bool retire_moves, unsigned long long seq, hipStream_t s);
void launch_finish(const Inst& I, int parity, bool reduce, bool zero_other, bool retire_moves, hipStream_t s);
void launch_remap(const Inst& I, int parity, const RemapRegions& R, hipStream_t s);
void launch_set_body(const Inst& I, int slot, const DevBody& b, hipStream_t s);
void launch_mass_total(const Inst& I, int parity, hipStream_t s);
void launch_contacts(const Inst& I, hipStream_t s);

}  // namespace lgs
