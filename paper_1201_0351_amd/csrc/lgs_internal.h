// lgs_internal.h -- device-side data structures and helpers shared by the
// kernels of the liquid-gas-solid LBM library (gfx950 / CDNA4).
//
// Layout of one lattice instance in device memory (all arrays x fastest,
// cell index id = x + nx (y + ny z), N cells):
//   pop[2]    two population lattices (ping-pong), structure of arrays
//             [19][ps] of the storage type (planes ps >= N elements apart,
//             first N used), holding the deviation f_i - w_i
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
// The nine pairs (i, ibar) of opposite links, primary member first.
__host__ __device__ constexpr int pair_p(int k) {
    constexpr int v[9] = {2, 3, 5, 8, 9, 10, 12, 14, 16};
    return v[k];
}
// weight class of a link: 0 rest, 1 axis (1/18), 2 diagonal (1/36)
__host__ __device__ constexpr int wclass(int i) { return i == 0 ? 0 : (i < 7 ? 1 : 2); }

// Constants of the bulk collision, computed on the host once per instance.
// The device has no scalar floating-point unit: a product of two uniform
// values costs one vector instruction per wavefront, as much as a per-cell
// one.  s is the storage scale (deviations are held as s (f_i - w_i)).
struct CollideConst {
    float om1;     // 1 - omega
    float om15;    // 1.5 omega
    float om45;    // 4.5 omega
    float om3;     // 3 omega
    float a3[3];   // 3 a
    float ca9[9];  // 9 c_p.a of pair k (p = pair_p(k))
    float ca3[9];  // 3 c_p.a
    float omw[3];  // omega w per weight class
    float sw[3];   // s w per weight class
    float inv;     // 1 / s
};

// --------------------------------------------------------------------------
// per-instance control block (device memory)
// --------------------------------------------------------------------------
struct StepCounters {
    int n_cand, n_newg, n_newl, n_recv;
    int filled, emptied, newg, newl;
    int overflow, n_bnd;
    int n_strd;  // stranded candidates the sweep listed (in Inst::recv)
    int n_se;    // of those, the ones that empty (listed after the sweep's candidates)
    int n_frec;  // force records the boundary sweep wrote (its workgroups that had listed cells)
    double acc[MAXB][6];  // per body: F (3), T (3), FP64, formed from the fixed-point sums
    long long facc[MAXB][12];  // fixed-point sums added by atomics (a cell touching a second body)
};

// Momentum exchange in fixed point.  A term x (an FP32 partial sum over one
// lane's links) is carried as two 64-bit integers, h = rint(x 2^24) and
// l = rint((x - h 2^-24) 2^60): exactly for every FP32 term of magnitude at
// least 2^-36, to within 2^-61 below that.  Integer sums are exact and do
// not depend on their order (wrap-around included), so a body's force and
// torque are the same however the boundary list was split among workgroups
// and whichever atomic lands first; h 2^-24 + l 2^-60 is formed once, from
// the totals.  Range: a total below 2^39 in magnitude, at most 2^27 terms
// per body and step.  Words of one body: h of F, T (6), then l of F, T (6).
constexpr int FXW = 12;
__device__ __forceinline__ void fx_split(float x, long long& h, long long& l) {
    // fmaxf / fminf map NaN to a bound: the sweep flags a non-finite cell itself
    const double xd = (double)fminf(fmaxf(x, -0x1p38f), 0x1p38f);
    const double hd = rint(xd * 0x1p24);
    h = (long long)hd;
    l = (long long)rint((xd - hd * 0x1p-24) * 0x1p60);
}
__host__ __device__ inline double fx_value(long long h, long long l) {
    return (double)h * 0x1p-24 + (double)l * 0x1p-60;
}

struct Ctl {
    StepCounters cnt[2];  // by step parity
    double ledger;
    double mass_total;
    unsigned long long contacts;
    int nonfinite;  // 1: a non-finite or non-positive density; NONFINITE_LAYERS: a bulk grid missed a fluid layer
    int body_err;  // BODY_ERR_* bits of a rejected free-body update
    // Highest z-layer that may hold a liquid or interface cell or a
    // conversion mark: scanned after init, computed on the host when flags
    // are written, raised by every step that turns a cell fluid (new
    // interface cells from gas, refilled cells); never lowered by a step.
    // The bulk sweep visits layers 0..ztop only.
    int ztop;
};

// Reasons the device update of a free body was rejected (the body keeps its
// pose; the next synchronising call reports the error).
constexpr int NONFINITE_LAYERS = 2;
enum : int { BODY_ERR_WALL = 1, BODY_ERR_SPEED = 2, BODY_ERR_CLOSE = 4, BODY_ERR_JUMP = 8 };

struct DevBody {
    double pos[3];   // centre of gravity o
    double quat[4];  // orientation (w, x, y, z), unit
    double R[9];     // body -> world, row major
    double half[3];
    double vel[3];
    double omega[3];
    double ext[3];       // world-frame half extent of the bounding box
    double prev_pos[3];  // pose of the last mapping (valid if mapped)
    double prev_ext[3];
    double fprev[6];  // previous step's force / torque (free bodies)
    double density;
    uint32_t dof;  // free bodies: DOF mask (bits 0-2 translation, 3-5 rotation)
    int shape;     // LBM_SHAPE_CUBOID, or LBM_SHAPE_SPHERE of radius half[0] (= half[1] = half[2])
    int active;
    int moved;      // pose changed since the last remap
    int mapped;     // the obstacle cells of the body exist
    int free_body;  // integrated on the device after every full step
    int have_prev;
};

// Everything a kernel needs about one instance (passed by value).
struct Inst {
    int nx, ny, nz, N;
    size_t ps;  // elements between two population planes (>= N)
    uint32_t periodic;
    int recon_mode;
    int storage;
    int nbodies;
    float omega;       // 1 / tau
    float ax, ay, az;  // body acceleration
    float rho_g;
    float wall_u[3];   // velocity of the non-periodic faces (moving no-slip walls)
    int wall_moving;   // wall_u != 0
    float lap;         // 2 sigma / cs^2: Laplace density jump per unit curvature (0: no surface tension)
    float scale, inv_scale;  // storage scale (FP16), 1 otherwise
    CollideConst cc;
    double eps;
    void* pop[2];
    uint8_t* flags;
    float* phi[2];
    float* m_hi;
    float* m_lo;
    float* share;
    float* aux;
    uint8_t* rule;
    float* kap;        // mean curvature of the interface cells of this step (surface tension only)
    // Per cell: 1 where the cell may have a gas or obstacle neighbour.  Set
    // by the remap around covered and on uncovered cells, and by written
    // types; cleared by the bulk sweep for a liquid cell whose 18 sources it
    // found fluid or wall.  The conversions keep an interface layer between
    // liquid and gas (Sec. 2.2), so a liquid cell with 0 here has neither.
    uint8_t* nearo;
    // Per interface cell: 1 if one of its 18 neighbours is liquid (written
    // by the sweep every step; stale for other cells)
    uint8_t* lnb;
    uint32_t* claim;   // new-interface claims
    uint32_t* cmask;   // per cell: bit l set when the neighbour over link l converted this step
    int* cand;
    int* newg;
    int* newl;
    // receivers of excess mass (appended by the middle conversion launch);
    // before that, from the sweep to the claim launch, the stranded
    // candidates: interface cells without a liquid neighbour and without a
    // conversion mark
    int* recv;
    int* bnd;  // cells the bulk sweep leaves to the boundary sweep
    // Momentum-exchange partial sums of the boundary sweep, one record per
    // workgroup of its grid and body: bit b of frec_mask[block] says the
    // workgroup met body b, whose fixed-point words (FXW of them, see
    // fx_split) sit at frec_v[(b * FXW + q) * BND_BLOCKS_MAX + block].  (A
    // cell touching two bodies at once adds to the second by integer atomics
    // on StepCounters::facc; the pose checks keep bodies three cells apart,
    // so none does.)
    uint32_t* frec_mask;
    long long* frec_v;
    // A word of pinned host memory (device-visible) where the conversions'
    // commit launch of step s reports (s << 32) | ctl->ztop, the layer bound
    // the host sizes later bulk grids with (nullptr: no report)
    unsigned long long* zpin;
    // FP64 partial sums of the liquid-mass total, one per chunk of
    // MASS_CHUNK cells (mass_parts(N) of them)
    double* mass_part;
    int list_cap;
    Ctl* ctl;
    DevBody* bodies;
};

// Lattice of a parity by selection, not by indexing: a descriptor copied into
// a kernel's registers stays there (a run-time index into its arrays would
// move it to scratch memory).
__device__ __forceinline__ void* pop_of(const Inst& I, int p) { return p ? I.pop[1] : I.pop[0]; }
__device__ __forceinline__ float* phi_of(const Inst& I, int p) { return p ? I.phi[1] : I.phi[0]; }

// --------------------------------------------------------------------------
// storage types
// --------------------------------------------------------------------------
template <typename S>
struct Store;
// Streaming accesses of the sweep: `load` / `store` (`store<true>`:
// non-temporal, streaming past the caches, for lattices larger than the cache
// in front of HBM); random accesses: `ld` / `st`.
template <bool NT, typename T>
__device__ __forceinline__ void stream_store(T v, T* p) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <>
struct Store<float> {
    __device__ static inline float load(const float* p, size_t k, float) { return p[k]; }
    __device__ static inline float ld(const float* p, size_t k, float) { return p[k]; }
    template <bool NT = false>
    __device__ static inline void store(float* p, size_t k, float v, float) { stream_store<NT>(v, p + k); }
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
    __device__ static inline float load(const __half* p, size_t k, float inv) { return h2f(((const U*)p)[k]) * inv; }
    __device__ static inline float ld(const __half* p, size_t k, float inv) { return h2f(((const U*)p)[k]) * inv; }
    template <bool NT = false>
    __device__ static inline void store(__half* p, size_t k, float v, float sc) {
        stream_store<NT>(f2h(v * sc), (U*)p + k);
    }
    __device__ static inline void st(__half* p, size_t k, float v, float sc) { ((U*)p)[k] = f2h(v * sc); }
};
template <>
struct Store<__hip_bfloat16> {
    using U = unsigned short;
    __device__ static inline float load(const __hip_bfloat16* p, size_t k, float) { return b2f(((const U*)p)[k]); }
    __device__ static inline float ld(const __hip_bfloat16* p, size_t k, float) { return b2f(((const U*)p)[k]); }
    template <bool NT = false>
    __device__ static inline void store(__hip_bfloat16* p, size_t k, float v, float) {
        stream_store<NT>(f2b(v), (U*)p + k);
    }
    __device__ static inline void st(__hip_bfloat16* p, size_t k, float v, float) { ((U*)p)[k] = f2b(v); }
};

// Buffer access to the population planes of one lattice: a gfx9 buffer
// resource (base, byte range, default format word) with a per-lane byte
// offset (VGPR) and a uniform byte offset (SGPR), so that the 19 planes of a
// cell share one per-lane offset and a plane costs no per-lane address
// arithmetic.  The planes must span less than 2^32 bytes.
constexpr int BUF_RSRC_WORD3 = 0x00020000;
constexpr int BUF_NT = 2;  // the nt (non-temporal) cache-policy bit of gfx94x / gfx950 buffer accesses
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, BUF_RSRC_WORD3);
}
template <typename S>
struct BufIO;
// load_raw / store_raw: the value at the storage scale (no scaling).
template <>
struct BufIO<float> {
    __device__ static inline float load(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
    }
    __device__ static inline float load_raw(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0));
    }
    template <bool NT>
    __device__ static inline void store_raw(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)vo, (int)so, NT ? BUF_NT : 0);
    }
    template <bool NT>
    __device__ static inline void store(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float v, float) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)vo, (int)so, NT ? BUF_NT : 0);
    }
};
template <>
struct BufIO<__half> {
    __device__ static inline float load(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float inv) {
        return h2f(__builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, 0)) * inv;
    }
    __device__ static inline float load_raw(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
        return h2f(__builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, 0));
    }
    template <bool NT>
    __device__ static inline void store_raw(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(f2h(v), r, (int)vo, (int)so, NT ? BUF_NT : 0);
    }
    template <bool NT>
    __device__ static inline void store(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float v, float sc) {
        __builtin_amdgcn_raw_buffer_store_b16(f2h(v * sc), r, (int)vo, (int)so, NT ? BUF_NT : 0);
    }
};
template <>
struct BufIO<__hip_bfloat16> {
    __device__ static inline float load(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float) {
        return b2f(__builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, 0));
    }
    __device__ static inline float load_raw(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
        return b2f(__builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, 0));
    }
    template <bool NT>
    __device__ static inline void store_raw(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(f2b(v), r, (int)vo, (int)so, NT ? BUF_NT : 0);
    }
    template <bool NT>
    __device__ static inline void store(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so, float v, float) {
        __builtin_amdgcn_raw_buffer_store_b16(f2b(v), r, (int)vo, (int)so, NT ? BUF_NT : 0);
    }
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

// instance k of a batch: off[k] <= block < off[k + 1]
__device__ __forceinline__ int batch_instance(const int* __restrict__ off, int n, int block) {
    int lo = 0, hi = n;  // off[lo] <= block < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= block) lo = mid;
        else hi = mid;
    }
    return lo;
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
    if (b.shape == LBM_SHAPE_SPHERE) return d0 * d0 + d1 * d1 + d2 * d2 <= b.half[0] * b.half[0];
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

// Cells a body remap visits: an axis-aligned box covering the bounding boxes
// of the body's last mapped pose and its new pose plus two cells (origin lo,
// extent dim).  On a periodic axis the new pose is taken at its minimum image
// relative to the old one, and a box as wide as the axis covers it once.
struct Region {
    int lo[3];
    int dim[3];
    int cells;
};

__host__ __device__ inline Region body_region(const DevBody& d, int nx, int ny, int nz, uint32_t periodic) {
    Region R;
    const int n[3] = {nx, ny, nz};
    R.cells = 1;
    for (int a = 0; a < 3; ++a) {
        const double pp = d.mapped ? d.prev_pos[a] : d.pos[a];
        const double pe = d.mapped ? d.prev_ext[a] : d.ext[a];
        const double np = pp + wrap_rel(d.pos[a] - pp, (double)n[a], periodic & (1u << a));
        const double lo = floor(fmin(pp - pe, np - d.ext[a]) - 2.0);
        const double hi = ceil(fmax(pp + pe, np + d.ext[a]) + 2.0);
        int l0 = (int)lo;
        int dim = (int)hi - l0 + 1;
        if ((periodic & (1u << a)) && dim >= n[a]) {
            l0 = 0;
            dim = n[a];
        }
        R.lo[a] = l0;
        R.dim[a] = dim;
        R.cells *= dim;
    }
    return R;
}

// Rotation matrix (body -> world, row major) of a unit quaternion (w,x,y,z).
__host__ __device__ inline void quat_to_R(const double q[4], double R[9]) {
#pragma clang fp contract(off)
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// World-frame half extents of the bounding box of a body: a cuboid's rotated
// extents, a sphere's radius.
__host__ __device__ inline void box_extent(int shape, const double R[9], const double half[3], double ext[3]) {
#pragma clang fp contract(off)
    for (int a = 0; a < 3; ++a)
        ext[a] = shape == LBM_SHAPE_SPHERE
                     ? half[0]
                     : fabs(R[a * 3 + 0]) * half[0] + fabs(R[a * 3 + 1]) * half[1] + fabs(R[a * 3 + 2]) * half[2];
}

// Rigid-body update of a cuboid of density rho_s (relative to the liquid)
// over one time step (Sec. 2.3: the fluid force and torque drive the body,
// which the next step maps anew): semi-implicit Euler,
//   V' = V + (F + M a) / M                     (translation DOFs in `dof`)
//   I_w (Omega' - Omega) = T                   (rotation DOFs, restricted to
//                                               the selected axes)
//   o' = o + V',  q' = exp(Omega' / 2) q  (renormalised)
// with M = rho_s l b h and I_w = R diag(M/3 (h_y^2 + h_z^2), ...) R^T.
// Returns false if the mass is not positive.  FP64, no contraction, so host
// and device evaluate the same operations.
// sin(th/2)/th and cos(th/2) of a rotation by th per step.  Below half-angle
// 0.05 both come from their Taylor series in nested form (the first omitted
// terms are under 3e-20 there, far below double rounding), above it from
// sin and cos.
__host__ __device__ inline void half_angle(double th, double& s_over_th, double& c) {
#pragma clang fp contract(off)
    const double x = 0.5 * th;
    if (x < 0.05) {
        const double x2 = x * x;
        const double sx = 1.0 - x2 * (1.0 / 6.0) * (1.0 - x2 * (1.0 / 20.0) * (1.0 - x2 * (1.0 / 42.0) * (1.0 - x2 * (1.0 / 72.0))));
        s_over_th = 0.5 * sx;
        c = 1.0 - x2 * 0.5 * (1.0 - x2 * (1.0 / 12.0) * (1.0 - x2 * (1.0 / 30.0) * (1.0 - x2 * (1.0 / 56.0))));
    } else {
        s_over_th = sin(x) / th;
        c = cos(x);
    }
}

__host__ __device__ inline bool integrate_rigid(int shape, const double half[3], const double pos[3],
                                                const double quat[4], const double vel[3], const double omega[3],
                                                double density, const double F[3], const double T[3],
                                                const double accel[3], uint32_t dof, double opos[3], double oquat[4],
                                                double ovel[3], double oomega[3]) {
#pragma clang fp contract(off)
    // mass of the body's own volume: cuboid 8 h0 h1 h2, sphere 4/3 pi r^3
    const bool sphere = shape == LBM_SHAPE_SPHERE;
    const double r3 = half[0] * half[0] * half[0];
    const double M = sphere ? density * (4.0 / 3.0) * 3.14159265358979323846 * r3
                            : density * 8.0 * half[0] * half[1] * half[2];
    if (!(M > 0.0)) return false;
    for (int a = 0; a < 3; ++a) {
        ovel[a] = (dof & (1u << a)) ? vel[a] + (F[a] + M * accel[a]) / M : vel[a];
        oomega[a] = omega[a];
    }
    double R[9];
    quat_to_R(quat, R);
    // principal moments: cuboid M/3 (h_j^2 + h_k^2), sphere 2/5 M r^2
    const double Is = 0.4 * M * half[0] * half[0];
    const double Ib[3] = {sphere ? Is : M / 3.0 * (half[1] * half[1] + half[2] * half[2]),
                          sphere ? Is : M / 3.0 * (half[0] * half[0] + half[2] * half[2]),
                          sphere ? Is : M / 3.0 * (half[0] * half[0] + half[1] * half[1])};
    double Iw[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += R[r * 3 + k] * Ib[k] * R[c * 3 + k];
            Iw[r * 3 + c] = acc;
        }
    // Gaussian elimination with partial pivoting on the system restricted to
    // the selected axes S (in increasing axis order).  Every loop has a
    // constant trip count and every array a constant index after unrolling
    // (selects instead of indexing), so the device keeps it in registers.
    int S[3] = {0, 0, 0}, ns = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (dof & (8u << a)) {
            if (ns == 0) S[0] = a;
            else if (ns == 1) S[1] = a;
            else S[2] = a;
            ++ns;
        }
    if (ns > 0) {
        double A[3][4];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double v = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        if (S[r] == i && S[c] == j) v = Iw[i * 3 + j];
                A[r][c] = (r < ns && c < ns) ? v : 0.0;
            }
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (S[r] == i) t = T[i];
            A[r][3] = r < ns ? t : 0.0;
        }
        // the right-hand side sits in column ns of the reduced system
        double rhs[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) rhs[r] = A[r][3];
#pragma unroll
        for (int pv = 0; pv < 3; ++pv) {
            if (pv >= ns) break;
            int best = pv;
#pragma unroll
            for (int r = pv + 1; r < 3; ++r)
                if (r < ns && fabs(A[r][pv]) > fabs(best == 0 ? A[0][pv] : (best == 1 ? A[1][pv] : A[2][pv])))
                    best = r;
            if (best != pv) {
#pragma unroll
                for (int r = pv + 1; r < 3; ++r)
                    if (r == best) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            const double t = A[pv][c];
                            A[pv][c] = A[r][c];
                            A[r][c] = t;
                        }
                        const double t = rhs[pv];
                        rhs[pv] = rhs[r];
                        rhs[r] = t;
                    }
            }
#pragma unroll
            for (int r = pv + 1; r < 3; ++r) {
                if (r >= ns) break;
                const double f = A[r][pv] / A[pv][pv];
#pragma unroll
                for (int c = pv; c < 3; ++c)
                    if (c < ns) A[r][c] -= f * A[pv][c];
                rhs[r] -= f * rhs[pv];
            }
        }
        double dw[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int r = 2; r >= 0; --r) {
            if (r >= ns) continue;
            double acc = rhs[r];
#pragma unroll
            for (int c = r + 1; c < 3; ++c)
                if (c < ns) acc -= A[r][c] * dw[c];
            dw[r] = acc / A[r][r];
        }
#pragma unroll
        for (int r = 0; r < 3; ++r)
            if (r < ns) {
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    if (S[r] == i) oomega[i] = omega[i] + dw[r];
            }
    }
    for (int a = 0; a < 3; ++a) opos[a] = pos[a] + ovel[a];
    const double th = sqrt(oomega[0] * oomega[0] + oomega[1] * oomega[1] + oomega[2] * oomega[2]);
    for (int a = 0; a < 4; ++a) oquat[a] = quat[a];
    if (th > 0.0) {
        double s, ch;
        half_angle(th, s, ch);
        const double dq[4] = {ch, s * oomega[0], s * oomega[1], s * oomega[2]};
        const double* q = quat;
        const double r[4] = {dq[0] * q[0] - dq[1] * q[1] - dq[2] * q[2] - dq[3] * q[3],
                             dq[0] * q[1] + dq[1] * q[0] + dq[2] * q[3] - dq[3] * q[2],
                             dq[0] * q[2] - dq[1] * q[3] + dq[2] * q[0] + dq[3] * q[1],
                             dq[0] * q[3] + dq[1] * q[2] - dq[2] * q[1] + dq[3] * q[0]};
        const double nn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
        for (int a = 0; a < 4; ++a) oquat[a] = r[a] / nn;
    }
    return true;
}

// Grid of the boundary sweep (256-thread workgroups, four wavefronts each);
// every workgroup of it writes one force record per step.
constexpr int BND_BLOCKS_MAX = 1024;
__host__ __device__ inline int boundary_blocks(const Inst& I) {
    const int need = (I.N + 255) / 256;
    return need < BND_BLOCKS_MAX ? need : BND_BLOCKS_MAX;
}

// --------------------------------------------------------------------------
// 32-lane groups (half a wavefront): lane i of a group owns D3Q19 link i
// --------------------------------------------------------------------------
// link tables packed into constants: 2 bits (c + 1) per link, 5 bits per
// opposite index (links 0..11 in OPP_LO, 12..18 in OPP_HI)
constexpr unsigned long long pack_c(int a) {
    unsigned long long v = 0;
    for (int i = 0; i < Q; ++i) v |= (unsigned long long)((a == 0 ? cx(i) : a == 1 ? cy(i) : cz(i)) + 1) << (2 * i);
    return v;
}
constexpr unsigned long long pack_opp(int lo, int hi) {
    unsigned long long v = 0;
    for (int i = lo; i < hi; ++i) v |= (unsigned long long)opp(i) << (5 * (i - lo));
    return v;
}
constexpr unsigned long long CXP = pack_c(0), CYP = pack_c(1), CZP = pack_c(2);
constexpr unsigned long long OPP_LO = pack_opp(0, 12), OPP_HI = pack_opp(12, Q);

__device__ __forceinline__ int lane_c(unsigned long long P, int i) { return (int)((P >> (2 * i)) & 3ull) - 1; }
__device__ __forceinline__ int lane_opp(int i) {
    return i < 12 ? (int)((OPP_LO >> (5 * i)) & 31ull) : (int)((OPP_HI >> (5 * (i - 12))) & 31ull);
}
__device__ __forceinline__ float lane_w(int i) { return i == 0 ? 1.f / 3.f : (i < 7 ? 1.f / 18.f : 1.f / 36.f); }

// sum over the 32-lane group of the calling lane (butterfly: every lane
// ends with the same operations in a different order)
__device__ __forceinline__ float gsum(float v) {
#pragma unroll
    for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}


__device__ __forceinline__ int g_lane() { return threadIdx.x & 31; }
__device__ __forceinline__ int g_base() { return threadIdx.x & 32; }  // first lane of the group in its wavefront
__device__ __forceinline__ unsigned g_ballot(bool p) { return (unsigned)(__ballot(p) >> g_base()); }
__device__ __forceinline__ int g_bcast(int v, int src) { return __shfl(v, g_base() + src); }
__device__ __forceinline__ float g_bcastf(float v, int src) { return __shfl(v, g_base() + src); }

// --------------------------------------------------------------------------
// kernel launchers (implemented in the .hip files)
// --------------------------------------------------------------------------
void launch_init(const Inst& I, const lbm_config& c, hipStream_t s);
// raise ctl->ztop to the highest layer holding a liquid or interface cell or
// a mark (ctl->ztop is zero after the workspace's clearing at creation)
void launch_ztop(const Inst& I, hipStream_t s);
// A batch: instance descriptors in device memory and, per instance, the
// first workgroup of its share of a grid (off[0..n], each share a multiple
// of 8 workgroups so that a workgroup's XCD is its index modulo 8 in the
// share as in the whole grid).
// every array of the instance addressable with 32-bit byte offsets (elem:
// bytes per stored population)
__host__ __device__ inline bool bnd_buf_fits(const Inst& I, size_t elem) {
    return (size_t)Q * I.ps * elem <= 0xFFFFFFFFull && (size_t)I.N * 4 <= 0xFFFFFFFFull;
}

// A batch's per-instance workgroup offsets passed by value (a bulk grid cut
// per instance to its layer bound): batches of at most BATCH_OFF_MAX
// instances.
constexpr int BATCH_OFF_MAX = 256;
struct BatchOff {
    int off[BATCH_OFF_MAX + 1];
};

struct BatchGrid {
    const Inst* tab;
    const int* off;
    int n;
    int blocks;             // off[n]
    bool buf_fits = false;  // every instance's arrays addressable with 32-bit offsets (boundary sweep)
    const BatchOff* hoff = nullptr;  // host offsets of a cut bulk grid (blocks = hoff->off[n]), else off
};

// workgroups of one instance's bulk grid for a tile width (32, 64 or 128
// cells along x, 256 / width rows; 0: 256 consecutive cells of a layer),
// padded to a multiple of 8
int bulk_blocks(const Inst& I, int tile_x, int layers = 0);

// e0 / e1: optional events recorded at the start / end of the kernel itself;
// nt: non-temporal population stores; layers > 0: launch the tiles of layers
// 0 .. layers-1 only (a bound the host holds on ctl->ztop; the step's claim
// launch flags a bound that was too low), else all
void launch_sweep_bulk(const Inst& I, int parity, int tile_x, bool nt, hipStream_t s, hipEvent_t e0 = nullptr,
                       hipEvent_t e1 = nullptr, int layers = 0);
// Mean curvature of the cells of this step's boundary list (surface tension
// only; after the bulk sweep, before the boundary sweep).
void launch_curvature(const Inst& I, int parity, hipStream_t s);
void launch_curvature_batch(const BatchGrid& G, int parity, hipStream_t s);
// layout: 0 = 8 lanes per listed cell, 1 = one thread per listed cell
void launch_sweep_boundary(const Inst& I, int parity, int layout, hipStream_t s, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr);
void launch_sweep_bulk_batch(const BatchGrid& G, int storage, int tile_x, bool nt, int parity, hipStream_t s,
                             hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_sweep_boundary_batch(const BatchGrid& G, int storage, int parity, int layout, hipStream_t s,
                                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_mark(const Inst& I, int parity, hipStream_t s);
// step_tag: the step's index, reported with ctl->ztop through I.zpin
// (NO_STEP_TAG: no report); bulk_layers > 0: the step's bulk grid covered
// layers 0 .. bulk_layers-1 only (checked against ctl->ztop)
constexpr unsigned NO_STEP_TAG = 0xFFFFFFFFu;
void launch_convert(const Inst& I, int parity, bool retire_moves, bool integrate, hipStream_t s,
                    unsigned step_tag = NO_STEP_TAG, int bulk_layers = 0);
void launch_finish(const Inst& I, int parity, bool reduce, bool zero_other, bool retire_moves, hipStream_t s);
void launch_remap(const Inst& I, int parity, int blocks_per_body, hipStream_t s);
// batches of at most 64 instances (bit k of a mask belongs to instance k)
void launch_remap_batch(const Inst* tab, int n, int max_bodies, int storage, int parity, int blocks_per_body,
                        hipStream_t s);
// Workgroups of an instance's conversion grid (three launches of this many
// 256-thread workgroups): one per 512 cells of an x-y layer, the size of a
// basin's free surface, 8 .. 256.
__host__ __device__ inline int conv_blocks(const Inst& I) {
    const int b = (int)(((long long)I.nx * I.ny + 511) / 512);
    return b < 8 ? 8 : (b > 256 ? 256 : b);
}
// blocks: the largest conv_blocks of the batch's instances (at most 64);
// step_tag: as for launch_convert; bulk_layers: each instance's bulk layer
// count of the step (nullptr or 0: all layers)
struct GroupLayers {
    int v[64];
};
void launch_convert_batch(const Inst* tab, int n, int blocks, int storage, int parity, unsigned long long retire_mask,
                          unsigned long long integrate_mask, hipStream_t s, unsigned step_tag = NO_STEP_TAG,
                          const int* bulk_layers = nullptr);
void launch_set_body(const Inst& I, int slot, const DevBody& b, hipStream_t s);
// Liquid-mass total sum_LIQ rho + sum_IF m in two fixed-order passes: one
// FP64 partial per chunk of MASS_CHUNK cells into part[0 .. mass_parts(N)),
// then their sum in chunk order into *out.  The result does not depend on
// scheduling.
constexpr int MASS_CHUNK = 4096;
constexpr int MASS_PARTS_MAX = 16384;  // chunks of the allocation-free variant
__host__ __device__ inline int mass_parts(int N) { return (N + MASS_CHUNK - 1) / MASS_CHUNK; }
void launch_mass_total(const Inst& I, int parity, double* part, double* out, hipStream_t s);
void launch_contacts(const Inst& I, hipStream_t s);

}  // namespace lgs
