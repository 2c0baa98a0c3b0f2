// k_sweep.hip -- the fused per-cell time step of liquid and interface cells.
//
// Pull form of Sec. 2.1 Eq. stream: cell x takes f'_i from s = x - c_i.
//   s liquid/interface : f'_i = f_i(s)
//   s wall / obstacle  : moving-wall bounce-back, Eq. noslip,
//                        f'_i = f_ibar(x) + 6 w_i rho_x c_i.u_w
//   s gas              : Eq. reconstruct with this cell's own outgoing
//                        f_ibar(x): f'_i = f_eq,i + f_eq,ibar - f_ibar(x) at
//                        (rho_G, u_x); with surface tension, interface
//                        cells use rho_G + 2 sigma kappa / cs^2 (kappa from
//                        k_tension.hip, computed just before this sweep)
// Interface cells also rebuild links from the gas side (c_i.n < -1e-3|n|_1,
// n = -grad phi), add the mass exchange of Sec. 2.2 to m and set phi = m/rho.
// Collide: f = f' - (f' - f_eq(rho,u))/tau + F_i with F_i of Eq. forceterm
// (Luo: w_i rho [(c_i - u)/cs2 + (c_i.u) c_i/cs4] . a).  rho_x, u_x: moments
// of f(x, t).  Populations are handled as deviations d_i = f_i - w_i.
//
// Two kernels keep the common case lean:
//   k_sweep_bulk      one thread per cell; liquid cells whose sources are all
//                     liquid, interface or static wall (bounce-back from a
//                     static wall is only a different load address) are
//                     streamed and collided here at low register pressure.
//                     Interface cells and liquid cells next to gas or a body
//                     are appended to a boundary list (wavefront ballots,
//                     offsets combined in LDS, one atomic per workgroup).
//                     Gas and obstacle cells cost a flag byte.  Only liquid
//                     cells with a near mark (Inst::nearo) read the types of
//                     their 18 sources: the conversions keep an interface
//                     layer between liquid and gas, and the remap marks the
//                     neighbours of every obstacle cell it creates.
//   k_sweep_boundary  one thread per listed cell: the full rule set, the
//                     interface mass and fill level, the conversion marks and
//                     the momentum exchange (Eqs. momentumexchange,
//                     momentuminterface) of every link into a body, summed as
//                     FP32 partials, reduced per wavefront in FP64 and added
//                     with one FP64 atomic per body.  The exchange uses
//                     d_ibar + w_i (1 - rho_G), i.e. it drops the constant
//                     2 c_i w_i rho_G, whose sum (and moment) over the links of
//                     a closed obstacle vanishes: gas cells then contribute
//                     nothing and the sums keep their precision.
#include <algorithm>

#include <hip/hip_ext.h>

#include "lgs_internal.h"

namespace lgs {

namespace {

constexpr double NORMAL_TOL = 1e-3;


__device__ __forceinline__ int lane_id() { return __lane_id(); }

// wavefront-aggregated append of `id` to a list (one atomic per wavefront)
__device__ __forceinline__ void wave_append(bool pred, int id, int* list, int* counter, int cap, int* overflow) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0) return;
    int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, __popcll(mask));
    base = __shfl(base, leader);
    if (pred) {
        int pos = base + __popcll(mask & ((1ull << lane_id()) - 1ull));
        if (pos < cap) list[pos] = id;
        else atomicOr(overflow, 1);
    }
}

// Workgroup-aggregated append of `id` to a list: one atomic per workgroup
// (blockDim.x = 64 NW).  Every wavefront of the workgroup must call it.  A
// single counter takes the appends of the whole grid, and device-scope
// atomics on one address serialise, so fewer of them shorten the sweep.
template <int NW>
__device__ __forceinline__ void block_append(bool pred, int id, int* list, int* counter, int cap, int* overflow) {
    __shared__ int wc[NW + 1];
    const int w = threadIdx.x >> 6;
    const unsigned long long mask = __ballot(pred);
    if (lane_id() == 0) wc[w] = __popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int c = wc[k];
            wc[k] = tot;
            tot += c;
        }
        wc[NW] = tot ? atomicAdd(counter, tot) : 0;
    }
    __syncthreads();
    if (pred) {
        const int pos = wc[NW] + wc[w] + __popcll(mask & ((1ull << lane_id()) - 1ull));
        if (pos < cap) list[pos] = id;
        else atomicOr(overflow, 1);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// compensated m += dm on an unevaluated float pair (hi, lo)
__device__ __forceinline__ void two_sum_add(float& hi, float& lo, float dm) {
    float s = hi + dm;
    float bp = s - hi;
    float err = (hi - (s - bp)) + (dm - bp);
    float l = lo + err;
    float h = s + l;
    lo = l - (h - s);
    hi = h;
}

// BGK collision with the force term on pulled deviations held at the storage
// scale s (d[] = s (f_i - w_i)); post-collision values at the same scale in
// out[].  Per pair of opposite links (p, pbar), with cu = c_p.u and
// ca = c_p.a, the relaxation towards the equilibrium plus the force term is
//   omega (f_eq,i - w_i) + F_i = omega w drho + w rho (g +- h),
//   g = 4.5 omega cu^2 + 9 ca cu - (1.5 omega u.u + 3 u.a),
//   h = 3 omega cu + 3 ca            (+ for p, - for pbar),
// and f*_i - w_i = (1 - omega) d_i + that.  Uniform factors come from the
// host (CollideConst).
__device__ __forceinline__ void collide(const CollideConst& K, int* nonfinite, const float (&d)[Q], float (&out)[Q]) {
    float drho = d[0], j0 = 0.f, j1 = 0.f, j2 = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int p = pair_p(k), q = opp(p);
        drho += d[p] + d[q];
        const float od = d[p] - d[q];
        j0 += cx(p) * od;
        j1 += cy(p) * od;
        j2 += cz(p) * od;
    }
    const float rho = fmaf(drho, K.inv, 1.f);
    if (!(rho > 0.f && rho < 1e6f)) atomicOr(nonfinite, 1);
    const float ir = K.inv * __builtin_amdgcn_rcpf(rho);  // 1-ulp reciprocal
    const float u0 = j0 * ir, u1 = j1 * ir, u2 = j2 * ir;
    const float base = -fmaf(K.om15, fmaf(u2, u2, fmaf(u1, u1, u0 * u0)),
                             fmaf(u2, K.a3[2], fmaf(u1, K.a3[1], u0 * K.a3[0])));
    float rw[3], omd[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        rw[c] = K.sw[c] * rho;
        omd[c] = K.omw[c] * drho;
    }
    out[0] = fmaf(K.om1, d[0], fmaf(rw[0], base, omd[0]));
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int p = pair_p(k), q = opp(p), c = wclass(p);
        const float cu = cx(p) * u0 + cy(p) * u1 + cz(p) * u2;
        const float g = fmaf(fmaf(K.om45, cu, K.ca9[k]), cu, base);
        const float h = fmaf(K.om3, cu, K.ca3[k]);
        const float E = fmaf(rw[c], g, omd[c]), O = rw[c] * h;
        out[p] = fmaf(K.om1, d[p], E + O);
        out[q] = fmaf(K.om1, d[q], E - O);
    }
}

// Post-collision values to the 19 planes of cell id.  fits (uniform): the
// planes span less than 2^32 bytes, so buffer stores take the cell's byte
// offset once and a uniform offset per plane.
template <typename S, bool NT>
__device__ __forceinline__ void collide_store(const Inst& I, const CollideConst& K, const float (&d)[Q],
                                              S* __restrict__ dst, int id, bool fits) {
    float o[Q];
    collide(K, &I.ctl->nonfinite, d, o);
    if (fits) {
        const uint32_t psb = (uint32_t)(I.ps * sizeof(S));
        const auto rd = buf_rsrc(dst, (uint32_t)Q * psb);
        const uint32_t ub = (uint32_t)id * (uint32_t)sizeof(S);
#pragma unroll
        for (int i = 0; i < Q; ++i) BufIO<S>::template store_raw<NT>(rd, ub, (uint32_t)i * psb, o[i]);
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) Store<S>::template store<NT>(dst, (size_t)i * I.ps + id, o[i], 1.f);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// bulk sweep
// ---------------------------------------------------------------------------
// One liquid cell: true if a source is gas or an obstacle (the cell is left
// to the boundary sweep), else pull, collide and store.  chk (the cell's near
// mark): read the 18 source types, and clear the mark if none is gas or an
// obstacle; without it every source is known to be liquid, interface or a
// static wall.  The population loads go out first.  Values stay at the
// storage scale from load to store.  PX: periodic in x.
template <typename S, bool NT, bool PX>
__device__ __forceinline__ bool bulk_cell(const Inst& I, const CollideConst& K, const S* __restrict__ src,
                                          S* __restrict__ dst, int x, int y, int z, int id, bool chk) {
    float d[Q];
    const int nx = I.nx, ny = I.ny, sxy = nx, sz = nx * ny;
    const bool py = I.periodic & 2, pz = I.periodic & 4;
    // Wavefronts whose cells all lie away from the y and z faces (x faces
    // included): one load per link and lane at a 32-bit offset from plane 0,
    // an x-face lane taking its periodic image or (wall) its own f_ibar by a
    // select.  Every 64-wide row segment holds an x-face cell; a separate
    // path for those lanes made each wavefront wait for one set of loads
    // before issuing the other.  Other wavefronts take the general sources
    // for all their lanes.
    const bool fits = (size_t)Q * I.ps * sizeof(S) <= 0xFFFFFFFFull;
    const bool inner = y > 0 && y < ny - 1 && z > 0 && z < I.nz - 1 && fits;
    // decided per wavefront, so that exactly one of the two load paths runs
    const bool row = __builtin_amdgcn_readfirstlane((int)(__ballot(!inner) == 0ull)) != 0;
    const bool xlo = x == 0, xhi = x == nx - 1;
    const int xm = step_axis(x, -1, nx, PX), xp = step_axis(x, 1, nx, PX);
    const int ym = step_axis(y, -1, ny, py), yp = step_axis(y, 1, ny, py);
    const int zm = step_axis(z, -1, I.nz, pz), zp = step_axis(z, 1, I.nz, pz);
    // source of link i next to a y or z face: its periodic image, or -1 (a
    // wall) (captures plain values: a reference to the descriptor would move
    // it to scratch memory in the batched kernel)
    auto face_src = [=](int i) {
        const int X = cx(i) == 1 ? xm : (cx(i) == -1 ? xp : x);
        const int Y = cy(i) == 1 ? ym : (cy(i) == -1 ? yp : y);
        const int Z = cz(i) == 1 ? zm : (cz(i) == -1 ? zp : z);
        return (X | Y | Z) >= 0 ? X + nx * (Y + ny * Z) : -1;
    };
    if (row) {
        // Buffer loads: the source of link i is plane i at this cell's byte
        // offset ub, shifted by the link: a uniform offset per link.  An
        // x-face lane takes its periodic image (ub +- one row) or, at a wall,
        // its own f_ibar (plane ibar at ub); for walls the uniform offset is
        // the smaller of the two planes' so that both lane offsets are
        // non-negative.
        const uint32_t psb = (uint32_t)(I.ps * sizeof(S));
        const auto rs = buf_rsrc(src, (uint32_t)Q * psb);
        const uint32_t ub = (uint32_t)id * (uint32_t)sizeof(S);
        const uint32_t wrapb = (uint32_t)nx * (uint32_t)sizeof(S);
        const uint32_t ulo = xlo ? ub + wrapb : ub, uhi = xhi ? ub - wrapb : ub;  // periodic images
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int sh = (cx(i) + sxy * cy(i) + sz * cz(i)) * (int)sizeof(S);
            const uint32_t bn = (uint32_t)i * psb - (uint32_t)sh;
            if (cx(i) == 0) {
                d[i] = BufIO<S>::load_raw(rs, ub, bn);
            } else if (PX) {
                d[i] = BufIO<S>::load_raw(rs, cx(i) == 1 ? ulo : uhi, bn);
            } else {
                const bool face = cx(i) == 1 ? xlo : xhi;
                const uint32_t bw = (uint32_t)opp(i) * psb;
                const uint32_t so = bn < bw ? bn : bw;
                d[i] = BufIO<S>::load_raw(rs, ub + (face ? bw - so : bn - so), so);
            }
        }
        d[0] = BufIO<S>::load_raw(rs, ub, 0u);
    } else {
        // a wall source is the halfway bounce-back: this cell's own f_ibar
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int s = face_src(i);
            d[i] = Store<S>::load(src + (size_t)(s >= 0 ? i : opp(i)) * I.ps, (unsigned)(s >= 0 ? s : id), 1.f);
        }
        d[0] = Store<S>::load(src, (size_t)id, 1.f);
    }
    if (chk) {
        // the types of the 18 sources (a wall reads as this liquid cell):
        // bit 1 of type + 1 is clear exactly for gas (0) and obstacle (3)
        const auto rf = buf_rsrc(I.flags, (uint32_t)I.N);
        uint32_t ok = 2u;
        if (row) {
            // x-face lanes: the periodic image one row over, or (wall) the
            // cell itself
            const int alo = xlo ? (PX ? nx : 0) : 0, ahi = xhi ? (PX ? -nx : 0) : 0;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int sh = cx(i) + sxy * cy(i) + sz * cz(i);
                int s = id - sh;
                if (cx(i) == 1) s = PX ? s + alo : (xlo ? id : s);
                if (cx(i) == -1) s = PX ? s + ahi : (xhi ? id : s);
                ok &= __builtin_amdgcn_raw_buffer_load_b8(rf, s, 0, 0) + 1u;
            }
        } else {
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int s = face_src(i);
                ok &= __builtin_amdgcn_raw_buffer_load_b8(rf, s >= 0 ? s : id, 0, 0) + 1u;
            }
        }
        if (!(ok & 2u)) return true;
        I.nearo[id] = 0;
    }
    collide_store<S, NT>(I, K, d, dst, id, fits);
    return false;
}

// Workgroup b of nb (nb a multiple of 8, b % 8 the XCD it runs on) of one
// instance's bulk grid.
// Tile c of layer z: TX > 0: TX x (256 / TX) cells; TX = 0: 256 consecutive
// cells of the layer (rows packed, wavefronts may cross a row end: every
// lane holds a cell when nx ny is a multiple of 256).
template <int TX>
struct BulkTiles {
    static constexpr int TY = TX ? 256 / TX : 1;
    int tiles_x, per_layer;
    __device__ BulkTiles(const Inst& I) {
        tiles_x = TX ? (I.nx + TX - 1) / TX : (I.nx * I.ny + 255) / 256;
        per_layer = tiles_x * (TX ? (I.ny + TY - 1) / TY : 1);
    }
};

template <typename S, int TX, bool W, bool NT, bool PX>
__device__ __forceinline__ void bulk_tile(const Inst& I, const CollideConst& K, int parity, const BulkTiles<TX>& T,
                                          int z, int c) {
    int x, y;
    if constexpr (TX == 0) {
        // one row of tiles per layer: tile c starts at cell 256 c of it
        const unsigned off = (unsigned)c * 256u + threadIdx.x;
        y = (int)(off / (unsigned)I.nx);
        x = (int)off - y * I.nx;
    } else {
        const int tx = c % T.tiles_x, ty = c / T.tiles_x;
        x = tx * TX + (threadIdx.x % TX);
        y = ty * BulkTiles<TX>::TY + (threadIdx.x / TX);
    }

    const S* __restrict__ src = (const S*)pop_of(I, parity);
    S* __restrict__ dst = (S*)pop_of(I, parity ^ 1);
    StepCounters& C = I.ctl->cnt[parity];

    const bool inb = (x < I.nx) && (y < I.ny);
    const int id = inb ? x + I.nx * (y + I.ny * z) : 0;
    const uint8_t fl = inb ? I.flags[id] : (uint8_t)GAS;
    const bool near = inb && I.nearo[id] != 0;
    const int type = fl & TYPE_MASK;
    // drop the marks a previous conversion phase left on this cell
    if (inb && (fl & ~KEEP_MASK)) I.flags[id] = fl & KEEP_MASK;

    // next to a moving wall the boundary sweep adds the wall term
    const bool wall = W && I.wall_moving &&
                      ((!(I.periodic & 1) && (x == 0 || x == I.nx - 1)) ||
                       (!(I.periodic & 2) && (y == 0 || y == I.ny - 1)) ||
                       (!(I.periodic & 4) && (z == 0 || z == I.nz - 1)));
    bool defer = (type == IFC) || (type == LIQ && wall);
    if (type == LIQ && !wall) defer = bulk_cell<S, NT, PX>(I, K, src, dst, x, y, z, id, near);
    block_append<4>(defer, id, I.bnd, &C.n_bnd, I.list_cap, &C.overflow);
}

// Workgroup b of nb of an instance's bulk grid (one tile each).  XCD-aware
// tile order: workgroup b runs on XCD b % 8.  Whole z-layers go round-robin
// to the XCDs, so a layer's y-halo rows and flags stay in one L2 while liquid
// and gas layers spread evenly over all eight XCDs.  Tiles above the highest
// layer that may hold fluid (ctl->ztop) leave after one scalar load, without
// touching their cells.
template <typename S, int TX, bool W, bool NT, bool PX>
__device__ __forceinline__ void sweep_bulk(const Inst& I, const CollideConst& K, int parity, int b, int nb) {
    const BulkTiles<TX> T(I);
    // unsigned: the divisions by the tile count need no sign fix-ups
    const unsigned CH = (unsigned)T.per_layer;
    const unsigned full = (unsigned)nb / (8u * CH) * (8u * CH);
    unsigned t = (unsigned)b;
    if (t < full) {
        const unsigned xcd = t & 7u, kk = t >> 3;
        t = ((kk / CH) * 8u + xcd) * CH + kk % CH;
    }
    if (t >= CH * (unsigned)I.nz) return;  // padding of the grid to a multiple of 8
    const int z = (int)(t / CH);
    if (z > I.ctl->ztop) return;  // gas (and bodies) only
    bulk_tile<S, TX, W, NT, PX>(I, K, parity, T, z, (int)(t - (unsigned)z * CH));
}

// At most 64 VGPRs, so that eight wavefronts fit per SIMD.  W: the lattice
// has moving walls (a variant without their test runs otherwise).  NT:
// non-temporal population stores.  PX: periodic in x.
template <typename S, int TX, bool W, bool NT, bool PX>
__global__ __launch_bounds__(256, 8) void k_sweep_bulk(Inst I, int parity) {
    sweep_bulk<S, TX, W, NT, PX>(I, I.cc, parity, blockIdx.x, gridDim.x);
}

// all instances of a batch in one launch (instance table in device memory;
// the copied descriptor needs registers of its own, so no 64-VGPR bound; the
// collision constants are read from the table where they are used)
template <typename S, int TX, bool NT>
__device__ __forceinline__ void batch_bulk(const Inst* __restrict__ tab, const int* off, int n, int parity) {
    const int k = batch_instance(off, n, blockIdx.x);
    const Inst I = tab[k];
    const CollideConst& K = tab[k].cc;
    if (I.periodic & 1) sweep_bulk<S, TX, true, NT, true>(I, K, parity, blockIdx.x - off[k], off[k + 1] - off[k]);
    else sweep_bulk<S, TX, true, NT, false>(I, K, parity, blockIdx.x - off[k], off[k + 1] - off[k]);
}
template <typename S, int TX, bool NT>
__global__ __launch_bounds__(256) void kb_sweep_bulk(const Inst* __restrict__ tab, const int* __restrict__ off, int n,
                                                     int parity) {
    batch_bulk<S, TX, NT>(tab, off, n, parity);
}
// the same with the offsets of a grid cut per instance to its layer bound
template <typename S, int TX, bool NT>
__global__ __launch_bounds__(256) void kb_sweep_bulk_cut(const Inst* __restrict__ tab, const BatchOff o, int n,
                                                         int parity) {
    batch_bulk<S, TX, NT>(tab, o.off, n, parity);
}

// ---------------------------------------------------------------------------
// boundary sweep: interface cells, liquid cells next to gas or a body.
// One group of 8 lanes per listed cell; lane l owns links l, l+8, l+16.
// The links' loaded values go through LDS so that every lane can read the
// opposite link's, and sums over the links are 3-step butterflies.  A few
// thousand wavefronts, all resident at once: the chain of dependent loads is
// paid once and each lane's arithmetic is a sixth of the cell's.
// ---------------------------------------------------------------------------
namespace {
constexpr int BL = 8;             // lanes per cell
constexpr int BCELLS = 256 / BL;  // cells per workgroup pass

__device__ __forceinline__ float osum(float v) {
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 1);
    return v;
}
}  // namespace

// Workgroup wg of nwg takes list entries wg * per, wg * per + nwg * per, ...:
// the first ceil(nlist / per) workgroups have cells and write force records
// (their number goes to the counters for the reduction); the others leave at
// once, so that a grid sized for the lattice costs little when the list is
// short (a batch of small instances).
__device__ __forceinline__ bool active_workgroup(StepCounters& C, int wg, int nwg, int nlist, int per) {
    const int active = min(nwg, (nlist + per - 1) / per);
    if (wg == 0 && threadIdx.x == 0 && active > 0) C.n_frec = active;
    return wg < active;
}

// Momentum exchange per boundary workgroup and body, in fixed point
// (fx_split): every lane whose cell met a body adds its terms to the
// workgroup's slot of that body in LDS with integer atomics, and at the end
// the slots go to the workgroup's records.  Integer sums do not depend on the
// order of the additions.
struct ForceLDS {
    unsigned long long v[MAXB][FXW];
    uint32_t mask;
};

// clear the slots (every thread calls it; a barrier follows before use)
__device__ __forceinline__ void force_begin(ForceLDS& F) {
    unsigned long long* v = &F.v[0][0];
    for (int k = threadIdx.x; k < MAXB * FXW; k += blockDim.x) v[k] = 0ull;
    if (threadIdx.x == 0) F.mask = 0u;
}

// one pass: this lane's terms cv (force, torque) on body `body` (-1: none)
__device__ __forceinline__ void force_flush(ForceLDS& F, int body, const float (&cv)[6]) {
    if (body < 0) return;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        long long h, l;
        fx_split(cv[q], h, l);
        atomicAdd(&F.v[body][q], (unsigned long long)h);
        atomicAdd(&F.v[body][6 + q], (unsigned long long)l);
    }
    atomicOr(&F.mask, 1u << body);
}

// a term on a second body of one cell: integer atomics on the step's sums
__device__ __forceinline__ void force_atomic(StepCounters& C, int b, const float (&t)[6]) {
    unsigned long long* a = (unsigned long long*)&C.facc[b][0];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        long long h, l;
        fx_split(t[q], h, l);
        atomicAdd(a + q, (unsigned long long)h);
        atomicAdd(a + 6 + q, (unsigned long long)l);
    }
}

// the workgroup's records (every thread calls it)
__device__ __forceinline__ void force_record(const Inst& I, int wg, ForceLDS& F) {
    __syncthreads();
    const uint32_t mask = F.mask;
    const int t = threadIdx.x;
    if (t < MAXB * FXW) {
        const int b = t / FXW, q = t % FXW;
        if ((mask >> b) & 1u) I.frec_v[(b * FXW + q) * BND_BLOCKS_MAX + wg] = (long long)F.v[b][q];
    }
    if (t == 0) I.frec_mask[wg] = mask;
}

// Workgroup wg of nwg of one instance's boundary grid (wg is its
// force-record slot).
template <typename S, bool W>
__device__ __forceinline__ void sweep_boundary(const Inst& I, int parity, int wg, int nwg) {
    const S* __restrict__ src = (const S*)pop_of(I, parity);
    S* __restrict__ dst = (S*)pop_of(I, parity ^ 1);
    const float isc = I.inv_scale;
    StepCounters& C = I.ctl->cnt[parity];
    const int nlist = min(C.n_bnd, I.list_cap);
    if (!active_workgroup(C, wg, nwg, nlist, BCELLS)) return;
    const bool px = I.periodic & 1, py = I.periodic & 2, pz = I.periodic & 4;
    const float* __restrict__ phi_t = phi_of(I, parity);
    const int l = threadIdx.x & (BL - 1);
    const int cell = threadIdx.x / BL;
    // momentum exchange per pass and body, in a fixed order
    __shared__ ForceLDS fsum;
    force_begin(fsum);
    // the bodies' centre, velocity and angular velocity, read once per
    // workgroup
    __shared__ double bpos[MAXB][3];
    __shared__ float bvel[MAXB][3], bom[MAXB][3];
    // per cell of the pass and link: source flag (-1: wall), pulled raw
    // deviation f_i(x - c_i), own deviation f_i(x), fill level of the source
    __shared__ int lsf[BCELLS][Q];
    __shared__ float ldr[BCELLS][Q], ldx[BCELLS][Q], lsph[BCELLS][Q];
    if ((int)threadIdx.x < I.nbodies * 3) {
        const int b = threadIdx.x / 3, a = threadIdx.x % 3;
        const DevBody& B = I.bodies[b];
        bpos[b][a] = B.pos[a];
        bvel[b][a] = (float)B.vel[a];
        bom[b][a] = (float)B.omega[a];
    }

    for (int base = wg * BCELLS; base < nlist; base += nwg * BCELLS) {
        int cell_body = -1;
        float cv[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        const int k = base + cell;
        const bool active = k < nlist;
        const int id = active ? I.bnd[k] : I.bnd[base];
        int x, y, z;
        cell_coords(I, id, x, y, z);
        // the cell's own values are loaded before its type is known, so that
        // they travel with the link loads below
        const uint8_t fl = I.flags[id];
        const float phiraw = phi_t[id];
        const float mhiraw = I.m_hi[id], mloraw = I.m_lo[id];
        const int type = fl & TYPE_MASK;
        const float phix = type == IFC ? phiraw : 1.f;
        float mhi = 0.f, mlo = 0.f;
        if (type == IFC && l == 0) {
            mhi = mhiraw;
            mlo = mloraw;
        }
        // this lane's links: sources s_i = x - c_i (a wall reads as an
        // obstacle at rest) and everything read from them
        float dx[3], dr[3];
        int sfe[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int i = l + BL * j;
            dx[j] = 0.f;
            dr[j] = 0.f;
            sfe[j] = -1;
            if (i < Q) {
                const int ci = lane_c(CXP, i), cyi = lane_c(CYP, i), czi = lane_c(CZP, i);
                const int X = step_axis(x, -ci, I.nx, px), Y = step_axis(y, -cyi, I.ny, py);
                const int Z = step_axis(z, -czi, I.nz, pz);
                const bool ok = (X | Y | Z) >= 0;
                const int s = ok ? X + I.nx * (Y + I.ny * Z) : id;
                sfe[j] = ok ? (int)I.flags[s] : -1;
                dr[j] = Store<S>::ld(src, (size_t)i * I.ps + s, isc);
                dx[j] = Store<S>::ld(src, (size_t)i * I.ps + id, isc);
                const float sp = phi_t[s];
                lsf[cell][i] = sfe[j];
                ldr[cell][i] = dr[j];
                ldx[cell][i] = dx[j];
                lsph[cell][i] = sp;
            }
        }
        __syncthreads();

        // moments of f(x, t)
        float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int i = l + BL * j;
            if (i < Q) {
                p0 += dx[j];
                p1 += lane_c(CXP, i) * dx[j];
                p2 += lane_c(CYP, i) * dx[j];
                p3 += lane_c(CZP, i) * dx[j];
            }
        }
        const float drx = osum(p0), jx0 = osum(p1), jx1 = osum(p2), jx2 = osum(p3);
        // a liquid cell among the 18 neighbours (the sources of links 1..18)
        int liq = 0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int i = l + BL * j;
            if (i >= 1 && i < Q && sfe[j] >= 0 && (sfe[j] & TYPE_MASK) == LIQ) liq = 1;
        }
        liq |= __shfl_xor(liq, 4);
        liq |= __shfl_xor(liq, 2);
        liq |= __shfl_xor(liq, 1);
        const float rhox = 1.f + drx;
        const float ux0 = jx0 / rhox, ux1 = jx1 / rhox, ux2 = jx2 / rhox;
        const float uu = ux0 * ux0 + ux1 * ux1 + ux2 * ux2;

        // interface normal n = -grad(phi) from the fill of the sources of
        // links 1..6 (wall / obstacle: own fill); FP64 sign test, the same
        // operations on every lane
        double n0 = 0.0, n1 = 0.0, n2 = 0.0, nthr = 0.0;
        if (type == IFC && I.recon_mode != LBM_RECON_GAS_ONLY) {
            double f[7];
#pragma unroll
            for (int i = 1; i <= 6; ++i) {
                const int e = lsf[cell][i];
                const int st = e & TYPE_MASK;
                double v = (double)phix;
                if (e >= 0 && st == LIQ) v = 1.0;
                else if (e >= 0 && st == GAS) v = 0.0;
                else if (e >= 0 && st == IFC) v = (double)lsph[cell][i];
                f[i] = v;
            }
            // the source of link E (c = +x) is x-1, of W (c = -x) is x+1
            n0 = 0.5 * (f[2] - f[1]);
            n1 = 0.5 * (f[3] - f[4]);
            n2 = 0.5 * (f[5] - f[6]);
            nthr = NORMAL_TOL * ((fabs(n0) + fabs(n1)) + fabs(n2));
        }

        // gas density of this cell's reconstruction: rho_G plus the Laplace
        // jump 2 sigma kappa / cs^2 at interface cells
        float rg = I.rho_g;
        if (I.lap != 0.f && type == IFC) rg += I.lap * I.kap[id];

        // per link: mass exchange with x + c_i = s_ibar, incoming population,
        // momentum exchange with a body
        float pdm = 0.f;
        float d[3];
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f, a5 = 0.f;
        int abody = -1;
        const float xc0 = x + 0.5f, xc1 = y + 0.5f, xc2 = z + 0.5f;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int i = l + BL * j;
            d[j] = 0.f;
            if (i >= Q) continue;
            if (i == 0) {
                d[j] = dx[j];
                continue;
            }
            const int o = lane_opp(i);
            const float cxf = (float)lane_c(CXP, i), cyf = (float)lane_c(CYP, i), czf = (float)lane_c(CZP, i);
            const float wi = lane_w(i);
            const float dxo = ldx[cell][o];
            if (type == IFC) {
                const int eo = lsf[cell][o];
                if (eo >= 0) {
                    const int sto = eo & TYPE_MASK;
                    const float ex = ldr[cell][o] - dx[j];  // f_ibar(x + c_i) - f_i(x)
                    if (sto == LIQ) pdm += ex;
                    else if (sto == IFC) pdm += 0.5f * (phix + lsph[cell][o]) * ex;
                }
            }
            const int e = sfe[j];
            const int st = e & TYPE_MASK;
            if (e < 0 || st == OBS) {
                float cu = 0.f;
                int bk = -1;
                float r0 = 0.f, r1 = 0.f, r2 = 0.f;
                if (e >= 0) {
                    bk = (e >> 2) & 15;
                    // body velocity at the link midpoint x_c - c_i/2
                    const float q0 = (float)wrap_rel(xc0 - 0.5f * cxf - bpos[bk][0], I.nx, px);
                    const float q1 = (float)wrap_rel(xc1 - 0.5f * cyf - bpos[bk][1], I.ny, py);
                    const float q2 = (float)wrap_rel(xc2 - 0.5f * czf - bpos[bk][2], I.nz, pz);
                    const float w0 = bom[bk][0], w1 = bom[bk][1], w2 = bom[bk][2];
                    const float u0 = bvel[bk][0] + (w1 * q2 - w2 * q1);
                    const float u1 = bvel[bk][1] + (w2 * q0 - w0 * q2);
                    const float u2 = bvel[bk][2] + (w0 * q1 - w1 * q0);
                    cu = cxf * u0 + cyf * u1 + czf * u2;
                    r0 = (float)wrap_rel(xc0 - bpos[bk][0], I.nx, px);
                    r1 = (float)wrap_rel(xc1 - bpos[bk][1], I.ny, py);
                    r2 = (float)wrap_rel(xc2 - bpos[bk][2], I.nz, pz);
                }
                if (W && e < 0) cu = cxf * I.wall_u[0] + cyf * I.wall_u[1] + czf * I.wall_u[2];  // a moving wall
                const float mw = 6.f * wi * rhox * cu;
                d[j] = dxo + mw;
                if (bk >= 0 && active) {
                    // momentum the fluid gains on this link (deviation form);
                    // the body receives the opposite
                    const float phat = type == LIQ ? 1.f : phix;
                    const float amp = 2.f * phat * (dxo + wi * (1.f - I.rho_g) + 0.5f * mw);
                    const float j0 = amp * cxf, j1 = amp * cyf, j2 = amp * czf;
                    const float t3 = r1 * j2 - r2 * j1, t4 = r2 * j0 - r0 * j2, t5 = r0 * j1 - r1 * j0;
                    if (abody < 0) abody = bk;
                    if (bk == abody) {
                        a0 -= j0;
                        a1 -= j1;
                        a2 -= j2;
                        a3 -= t3;
                        a4 -= t4;
                        a5 -= t5;
                    } else {
                        // a second body on this lane's links
                        const float tb[6] = {-j0, -j1, -j2, -t3, -t4, -t5};
                        force_atomic(C, bk, tb);
                    }
                }
            } else {
                bool recon = st == GAS;
                if (!recon && type == IFC && I.recon_mode != LBM_RECON_GAS_ONLY) {
                    const double cn = cxf * n0 + cyf * n1 + czf * n2;
                    recon = I.recon_mode == LBM_RECON_GAS_SIDE ? (cn < -nthr) : (cn <= nthr);
                }
                if (recon) {
                    const float cu = cxf * ux0 + cyf * ux1 + czf * ux2;
                    // (f_eq,i + f_eq,ibar)(rho_G, u_x) - 2 w_i, minus d_ibar(x)
                    d[j] = 2.f * wi * (rg * (1.f + 4.5f * cu * cu - 1.5f * uu) - 1.f) - dxo;
                } else {
                    d[j] = dr[j];
                }
            }
        }
        const float dm = osum(pdm);

        // moments after streaming, fill level and marks, collision
        float q0 = 0.f, q1 = 0.f, q2 = 0.f, q3 = 0.f;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int i = l + BL * j;
            if (i < Q) {
                q0 += d[j];
                q1 += lane_c(CXP, i) * d[j];
                q2 += lane_c(CYP, i) * d[j];
                q3 += lane_c(CZP, i) * d[j];
            }
        }
        const float drho = osum(q0), j0 = osum(q1), j1 = osum(q2), j2 = osum(q3);
        const float rho = 1.f + drho;
        bool cand = false, strd = false;
        if (active && type == IFC && l == 0) {
            two_sum_add(mhi, mlo, dm);
            const float ph = (float)(((double)mhi + (double)mlo) / (1.0 + (double)drho));
            const double phd = (double)ph;
            // filled past 1 + eps, emptied past -eps; an unmarked cell
            // without a liquid neighbour is a stranded candidate, decided by
            // the claim launch from its neighbours' liquid contacts
            uint8_t mark = 0;
            if (phd >= 1.0 + I.eps) mark = MARK_FILL;
            else if (phd <= -I.eps) mark = MARK_EMPTY;
            I.m_hi[id] = mhi;
            I.m_lo[id] = mlo;
            phi_of(I, parity ^ 1)[id] = ph;
            I.aux[id] = drho;  // rho - 1 of this interface cell, for the conversion phase
            I.lnb[id] = (uint8_t)liq;
            if (mark) {
                I.flags[id] = (fl & KEEP_MASK) | mark;
                cand = true;
            }
            strd = !mark && !liq;
        }
        wave_append(cand, id, I.cand, &C.n_cand, I.list_cap, &C.overflow);
        wave_append(strd, id, I.recv, &C.n_strd, I.list_cap, &C.overflow);
        if (active) {
            const float irho = 1.f / rho;
            const float u0 = j0 * irho, u1 = j1 * irho, u2 = j2 * irho;
            const float uq = 1.5f * (u0 * u0 + u1 * u1 + u2 * u2);
            const float ua = u0 * I.ax + u1 * I.ay + u2 * I.az;
            if (l == 0 && !(rho > 0.f && rho < 1e6f)) atomicOr(&I.ctl->nonfinite, 1);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int i = l + BL * j;
                if (i >= Q) continue;
                const float cxf = (float)lane_c(CXP, i), cyf = (float)lane_c(CYP, i), czf = (float)lane_c(CZP, i);
                const float wi = lane_w(i);
                const float cu = cxf * u0 + cyf * u1 + czf * u2;
                const float ca = cxf * I.ax + cyf * I.ay + czf * I.az;
                const float deq = wi * (drho + rho * (3.f * cu + 4.5f * cu * cu - uq));
                const float F = wi * rho * (3.f * (ca - ua) + 9.f * cu * ca);
                Store<S>::store(dst, (size_t)i * I.ps + id, d[j] + I.omega * (deq - d[j]) + F, I.scale);
            }
            if (abody >= 0) {
                cell_body = abody;
                cv[0] = a0;
                cv[1] = a1;
                cv[2] = a2;
                cv[3] = a3;
                cv[4] = a4;
                cv[5] = a5;
            }
        }
        force_flush(fsum, cell_body, cv);
        __syncthreads();  // the next pass overwrites the LDS arrays
    }

    force_record(I, wg, fsum);
}

// ---------------------------------------------------------------------------
// boundary sweep, one thread per listed cell: the rules and operations of the
// 8-lane kernel link by link.  The bulk sweep lists cells in tile order, so
// consecutive entries are mostly consecutive cells of a row and every load
// of a wavefront is one coalesced segment, and a long list (a large free
// surface) is in flight at once instead of in serial passes of 32 cells
// per workgroup.  The sources are taken one link at a time (after the six
// that give the interface normal), so that only the cell's own and incoming
// populations stay live.  BUF: 32-bit buffer offsets (every array of the
// instance below 4 GiB).
// ---------------------------------------------------------------------------
template <typename S, bool BUF>
struct BndIO {
    const S* src;
    S* dst;
    const float* phi;
    const uint8_t* fl;
    __amdgpu_buffer_rsrc_t rs, rd, rp, rf;
    uint32_t psb;
    size_t ps;
    float isc, sc;
    __device__ BndIO(const Inst& I, int parity) {
        src = (const S*)pop_of(I, parity);
        dst = (S*)pop_of(I, parity ^ 1);
        phi = phi_of(I, parity);
        fl = I.flags;
        ps = I.ps;
        psb = (uint32_t)(I.ps * sizeof(S));
        isc = I.inv_scale;
        sc = I.scale;
        if (BUF) {
            rs = buf_rsrc(src, (size_t)Q * I.ps * sizeof(S));
            rd = buf_rsrc(dst, (size_t)Q * I.ps * sizeof(S));
            rp = buf_rsrc(phi, (size_t)I.N * 4);
            rf = buf_rsrc(fl, (size_t)I.N);
        }
    }
    __device__ float pop(int i, int c) const {
        if (BUF) return BufIO<S>::load(rs, (uint32_t)c * (uint32_t)sizeof(S), (uint32_t)i * psb, isc);
        return Store<S>::ld(src, (size_t)i * ps + c, isc);
    }
    __device__ void put(int i, int c, float v) const {
        if (BUF) BufIO<S>::template store<false>(rd, (uint32_t)c * (uint32_t)sizeof(S), (uint32_t)i * psb, v, sc);
        else Store<S>::store(dst, (size_t)i * ps + c, v, sc);
    }
    __device__ float fill(int c) const {
        if (BUF) return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rp, (int)((uint32_t)c * 4u), 0, 0));
        return phi[c];
    }
    __device__ int flag(int c) const {
        if (BUF) return (int)__builtin_amdgcn_raw_buffer_load_b8(rf, (int)c, 0, 0);
        return (int)fl[c];
    }
};

template <typename S, bool W, bool BUF>
__device__ __forceinline__ void sweep_boundary1(const Inst& I, int parity, int wg, int nwg) {
    const BndIO<S, BUF> io(I, parity);
    StepCounters& C = I.ctl->cnt[parity];
    const int nlist = min(C.n_bnd, I.list_cap);
    if (!active_workgroup(C, wg, nwg, nlist, 256)) return;
    const bool px = I.periodic & 1, py = I.periodic & 2, pz = I.periodic & 4;
    const int nx = I.nx, ny = I.ny, nz = I.nz, sxy = nx, sz = nx * ny;
    __shared__ ForceLDS fsum;
    force_begin(fsum);
    __shared__ double bpos[MAXB][3];
    __shared__ float bvel[MAXB][3], bom[MAXB][3];
    if ((int)threadIdx.x < I.nbodies * 3) {
        const int b = threadIdx.x / 3, a = threadIdx.x % 3;
        const DevBody& B = I.bodies[b];
        bpos[b][a] = B.pos[a];
        bvel[b][a] = (float)B.vel[a];
        bom[b][a] = (float)B.omega[a];
    }
    __syncthreads();

    for (int base = wg * 256; base < nlist; base += nwg * 256) {
        int cell_body = -1;
        float cv[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        const int k = base + (int)threadIdx.x;
        const bool active = k < nlist;
        const int id = I.bnd[active ? k : base];
        int x, y, z;
        cell_coords(I, id, x, y, z);
        const int fl = io.flag(id);
        const int type = fl & TYPE_MASK;
        const bool ifc = type == IFC;
        const bool face = x == 0 || x == nx - 1 || y == 0 || y == ny - 1 || z == 0 || z == nz - 1;
        // source s_i = x - c_i, or -1 beyond a wall
        auto source = [&](int i) -> int {
            if (!face) return id - (cx(i) + sxy * cy(i) + sz * cz(i));
            const int X = step_axis(x, -cx(i), nx, px), Y = step_axis(y, -cy(i), ny, py);
            const int Z = step_axis(z, -cz(i), nz, pz);
            return (X | Y | Z) >= 0 ? X + nx * (Y + ny * Z) : -1;
        };

        // the cell's own f_i(x, t); then, for the sources s_i (the cell
        // itself beyond a wall), their types, incoming populations
        // f_i(x - c_i) and fills: those of links 1..9 right away, those of
        // 10..18 when links 1..9 are done.  Each half is issued before any
        // of it is used (one round trip, not one per link), and only half
        // of the sources' values are live at a time.
        float dx[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) dx[i] = io.pop(i, id);
        const float phr = io.fill(id);
        const float mhr = I.m_hi[id], mlr = I.m_lo[id];
        int sq[Q], eq[Q];
        float pq[Q], fq[Q];
        auto fetch = [&](int i) {
            const int s = source(i);
            const int sa = s >= 0 ? s : id;
            sq[i] = s;
            eq[i] = io.flag(sa);
            pq[i] = io.pop(i, sa);
            fq[i] = io.fill(sa);
        };
        constexpr int H1 = 9;  // links of the first half
#pragma unroll
        for (int i = 1; i <= H1; ++i) fetch(i);
        float drx = 0.f, jx0 = 0.f, jx1 = 0.f, jx2 = 0.f;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            drx += dx[i];
            jx0 += cx(i) * dx[i];
            jx1 += cy(i) * dx[i];
            jx2 += cz(i) * dx[i];
        }
        const float rhox = 1.f + drx;
        const float ux0 = jx0 / rhox, ux1 = jx1 / rhox, ux2 = jx2 / rhox;
        const float uu = ux0 * ux0 + ux1 * ux1 + ux2 * ux2;
        const float phix = ifc ? phr : 1.f;
        const float mhi0 = ifc ? mhr : 0.f, mlo0 = ifc ? mlr : 0.f;

        // interface normal n = -grad(phi) from the sources of links 1..6
        // (wall / obstacle: own fill), FP64 sign test
        double n0 = 0.0, n1 = 0.0, n2 = 0.0, nthr = 0.0;
        if (ifc && I.recon_mode != LBM_RECON_GAS_ONLY) {
            double f[7];
#pragma unroll
            for (int i = 1; i <= 6; ++i) {
                const int e = sq[i] >= 0 ? eq[i] : -1;
                const int st = e & TYPE_MASK;
                double v = (double)phix;
                if (e >= 0 && st == LIQ) v = 1.0;
                else if (e >= 0 && st == GAS) v = 0.0;
                else if (e >= 0 && st == IFC) v = (double)fq[i];
                f[i] = v;
            }
            n0 = 0.5 * (f[2] - f[1]);
            n1 = 0.5 * (f[3] - f[4]);
            n2 = 0.5 * (f[5] - f[6]);
            nthr = NORMAL_TOL * ((fabs(n0) + fabs(n1)) + fabs(n2));
        }

        // gas density of this cell's reconstruction
        float rg = I.rho_g;
        if (I.lap != 0.f && ifc) rg += I.lap * I.kap[id];

        // per source s_i: mass exchange of link ibar (x + c_ibar = s_i),
        // liquid contact, incoming population f_i(x) and momentum exchange
        // with a body
        float pdm = 0.f;
        int liq = 0;
        float d[Q];
        d[0] = dx[0];
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f, a5 = 0.f;
        int abody = -1;
        const float xc0 = x + 0.5f, xc1 = y + 0.5f, xc2 = z + 0.5f;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            if (i == H1 + 1) {
#pragma unroll
                for (int i2 = H1 + 1; i2 < Q; ++i2) fetch(i2);
            }
            const int o = opp(i);
            const int e = sq[i] >= 0 ? eq[i] : -1;
            const float dri = pq[i];  // f_i(x - c_i)
            const float fs = fq[i];   // used only when the source is an interface cell
            const int st = e & TYPE_MASK;
            const float dxo = dx[o];
            if (e >= 0 && st == LIQ) liq = 1;
            if (ifc && e >= 0) {
                const float ex = dri - dxo;  // f_i(x + c_ibar) - f_ibar(x)
                if (st == LIQ) pdm += ex;
                else if (st == IFC) pdm += 0.5f * (phix + fs) * ex;
            }
            const float cxf = (float)cx(i), cyf = (float)cy(i), czf = (float)cz(i);
            const float wi = wgt(i);
            float di = dri;
            if (e < 0 || st == OBS) {
                float cu = 0.f;
                int bk = -1;
                float r0 = 0.f, r1 = 0.f, r2 = 0.f;
                if (e >= 0) {
                    bk = (e >> 2) & 15;
                    // body velocity at the link midpoint x_c - c_i/2
                    const float q0 = (float)wrap_rel(xc0 - 0.5f * cxf - bpos[bk][0], nx, px);
                    const float q1 = (float)wrap_rel(xc1 - 0.5f * cyf - bpos[bk][1], ny, py);
                    const float q2 = (float)wrap_rel(xc2 - 0.5f * czf - bpos[bk][2], nz, pz);
                    const float w0 = bom[bk][0], w1 = bom[bk][1], w2 = bom[bk][2];
                    const float u0 = bvel[bk][0] + (w1 * q2 - w2 * q1);
                    const float u1 = bvel[bk][1] + (w2 * q0 - w0 * q2);
                    const float u2 = bvel[bk][2] + (w0 * q1 - w1 * q0);
                    cu = cxf * u0 + cyf * u1 + czf * u2;
                    r0 = (float)wrap_rel(xc0 - bpos[bk][0], nx, px);
                    r1 = (float)wrap_rel(xc1 - bpos[bk][1], ny, py);
                    r2 = (float)wrap_rel(xc2 - bpos[bk][2], nz, pz);
                }
                if (W && e < 0) cu = cxf * I.wall_u[0] + cyf * I.wall_u[1] + czf * I.wall_u[2];  // a moving wall
                const float mw = 6.f * wi * rhox * cu;
                di = dxo + mw;
                if (bk >= 0 && active) {
                    // momentum the fluid gains on this link (deviation form);
                    // the body receives the opposite
                    const float phat = type == LIQ ? 1.f : phix;
                    const float amp = 2.f * phat * (dxo + wi * (1.f - I.rho_g) + 0.5f * mw);
                    const float j0 = amp * cxf, j1 = amp * cyf, j2 = amp * czf;
                    const float t3 = r1 * j2 - r2 * j1, t4 = r2 * j0 - r0 * j2, t5 = r0 * j1 - r1 * j0;
                    if (abody < 0) abody = bk;
                    if (bk == abody) {
                        a0 -= j0;
                        a1 -= j1;
                        a2 -= j2;
                        a3 -= t3;
                        a4 -= t4;
                        a5 -= t5;
                    } else {
                        const float tb[6] = {-j0, -j1, -j2, -t3, -t4, -t5};  // a second body
                        force_atomic(C, bk, tb);
                    }
                }
            } else {
                bool recon = st == GAS;
                if (!recon && ifc && I.recon_mode != LBM_RECON_GAS_ONLY) {
                    const double cn = cxf * n0 + cyf * n1 + czf * n2;
                    recon = I.recon_mode == LBM_RECON_GAS_SIDE ? (cn < -nthr) : (cn <= nthr);
                }
                if (recon) {
                    const float cu = cxf * ux0 + cyf * ux1 + czf * ux2;
                    di = 2.f * wi * (rg * (1.f + 4.5f * cu * cu - 1.5f * uu) - 1.f) - dxo;
                }
            }
            d[i] = di;
        }

        // moments after streaming, fill level and marks, collision
        float drho = 0.f, j0 = 0.f, j1 = 0.f, j2 = 0.f;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            drho += d[i];
            j0 += cx(i) * d[i];
            j1 += cy(i) * d[i];
            j2 += cz(i) * d[i];
        }
        const float rho = 1.f + drho;
        bool cand = false, strd = false;
        if (active && ifc) {
            float mhi = mhi0, mlo = mlo0;
            two_sum_add(mhi, mlo, pdm);
            const float ph = (float)(((double)mhi + (double)mlo) / (1.0 + (double)drho));
            const double phd = (double)ph;
            uint8_t mark = 0;
            if (phd >= 1.0 + I.eps) mark = MARK_FILL;
            else if (phd <= -I.eps) mark = MARK_EMPTY;
            I.m_hi[id] = mhi;
            I.m_lo[id] = mlo;
            phi_of(I, parity ^ 1)[id] = ph;
            I.aux[id] = drho;
            I.lnb[id] = (uint8_t)liq;
            if (mark) {
                I.flags[id] = (uint8_t)((fl & KEEP_MASK) | mark);
                cand = true;
            }
            strd = !mark && !liq;
        }
        wave_append(cand, id, I.cand, &C.n_cand, I.list_cap, &C.overflow);
        wave_append(strd, id, I.recv, &C.n_strd, I.list_cap, &C.overflow);
        if (active) {
            const float irho = 1.f / rho;
            const float u0 = j0 * irho, u1 = j1 * irho, u2 = j2 * irho;
            const float uq = 1.5f * (u0 * u0 + u1 * u1 + u2 * u2);
            const float ua = u0 * I.ax + u1 * I.ay + u2 * I.az;
            if (!(rho > 0.f && rho < 1e6f)) atomicOr(&I.ctl->nonfinite, 1);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const float cxf = (float)cx(i), cyf = (float)cy(i), czf = (float)cz(i);
                const float wi = wgt(i);
                const float cu = cxf * u0 + cyf * u1 + czf * u2;
                const float ca = cxf * I.ax + cyf * I.ay + czf * I.az;
                const float deq = wi * (drho + rho * (3.f * cu + 4.5f * cu * cu - uq));
                const float F = wi * rho * (3.f * (ca - ua) + 9.f * cu * ca);
                io.put(i, id, d[i] + I.omega * (deq - d[i]) + F);
            }
            if (abody >= 0) {
                cell_body = abody;
                cv[0] = a0;
                cv[1] = a1;
                cv[2] = a2;
                cv[3] = a3;
                cv[4] = a4;
                cv[5] = a5;
            }
        }
        force_flush(fsum, cell_body, cv);
    }
    force_record(I, wg, fsum);
}

// one thread per cell; LGS_BND1_WAVES wavefronts per SIMD (three: 168
// registers, with the sources loaded in two halves; all 18 at once take
// some 220, i.e. two wavefronts, too few slots for a long list in one round)
#ifndef LGS_BND1_WAVES
#define LGS_BND1_WAVES 3
#endif
template <typename S, bool W, bool BUF>
__global__ __launch_bounds__(256, LGS_BND1_WAVES) void k_sweep_boundary1(Inst I, int parity) {
    sweep_boundary1<S, W, BUF>(I, parity, blockIdx.x, gridDim.x);
}

// Batched boundary sweep on a persistent grid.  A work item is one active
// slot of one instance's boundary grid (slot s of instance k takes the list
// cells, and writes the force record, that workgroup s of the instance's
// own grid would); items are numbered in instance order and workgroup g
// takes items g, g + G, ...  The list lengths are known only on the
// device, so a grid of every instance's full boundary grid would launch
// mostly workgroups without cells; this grid is sized to what the chip
// holds at once and launches none.  body(k, s) runs one item; every thread
// of the workgroup calls it with the same arguments.
template <typename F>
__device__ __forceinline__ void batch_items(const Inst* __restrict__ tab, int n, int parity, int per, F&& body) {
    __shared__ int pre[256];
    const int t = threadIdx.x;
    int before = 0;  // items of the instances before this chunk of 256
    for (int k0 = 0; k0 < n; k0 += 256) {
        int a = 0;
        if (k0 + t < n) {
            const Inst& J = tab[k0 + t];
            const int nlist = min(J.ctl->cnt[parity].n_bnd, J.list_cap);
            a = min(boundary_blocks(J), (nlist + per - 1) / per);
        }
        __syncthreads();  // the last chunk's items have read pre
        pre[t] = a;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {  // inclusive scan
            const int v = t >= o ? pre[t - o] : 0;
            __syncthreads();
            pre[t] += v;
            __syncthreads();
        }
        const int total = __builtin_amdgcn_readfirstlane(pre[255]);
        const int G = (int)gridDim.x, g = (int)blockIdx.x;
        for (int i = before + (g - before % G + G) % G; i < before + total; i += G) {
            const int loc = i - before;
            int lo = 0, hi = 255;  // first instance j of the chunk with pre[j] > loc
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (pre[mid] > loc) hi = mid;
                else lo = mid + 1;
            }
            const int j = __builtin_amdgcn_readfirstlane(lo);
            const int sl = __builtin_amdgcn_readfirstlane(loc - (j ? pre[j - 1] : 0));
            __syncthreads();  // the last item's readers of the sweep's LDS are done
            body(k0 + j, sl);
        }
        before += total;
    }
}

// BUF: every instance of the batch addressable with 32-bit buffer offsets
template <typename S, bool BUF>
__global__ __launch_bounds__(256, LGS_BND1_WAVES) void kb_sweep_boundary1(const Inst* __restrict__ tab, int n, int parity) {
    batch_items(tab, n, parity, 256, [&](int k, int sl) {
        const Inst& I = tab[k];  // fields read from the table as needed
        sweep_boundary1<S, true, BUF>(I, parity, sl, boundary_blocks(I));
    });
}

template <typename S, bool W>
__global__ __launch_bounds__(256, 3) void k_sweep_boundary(Inst I, int parity) {
    sweep_boundary<S, W>(I, parity, blockIdx.x, gridDim.x);
}

template <typename S>
__global__ __launch_bounds__(256, 3) void kb_sweep_boundary(const Inst* __restrict__ tab, int n, int parity) {
    batch_items(tab, n, parity, BCELLS, [&](int k, int sl) {
        const Inst& I = tab[k];  // fields read from the table as needed
        sweep_boundary<S, true>(I, parity, sl, boundary_blocks(I));
    });
}

// The sweep kernels go through the extended launch, which records the
// optional start / stop events with the dispatch itself (the kernel's own
// execution, without separate marker packets).
// compute units of the current device (256 if the query fails)
int device_cus() {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        ncu <= 0)
        ncu = 256;
    return ncu;
}

int bulk_blocks(const Inst& I, int tile_x, int layers) {
    const int nz = layers > 0 && layers < I.nz ? layers : I.nz;
    int n;
    if (tile_x == 0) {
        n = ((I.nx * I.ny + 255) / 256) * nz;
    } else {
        const int ty = 256 / tile_x;
        n = ((I.nx + tile_x - 1) / tile_x) * ((I.ny + ty - 1) / ty) * nz;
    }
    return (n + 7) / 8 * 8;
}

namespace {
template <typename S, int TX, bool NT>
void bulk_one(const Inst& I, int parity, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int layers) {
    const dim3 g(bulk_blocks(I, TX, layers)), b(256);
    const bool px = I.periodic & 1;
    if (I.wall_moving && px)
        hipExtLaunchKernelGGL((k_sweep_bulk<S, TX, true, NT, true>), g, b, 0, s, e0, e1, 0, I, parity);
    else if (I.wall_moving)
        hipExtLaunchKernelGGL((k_sweep_bulk<S, TX, true, NT, false>), g, b, 0, s, e0, e1, 0, I, parity);
    else if (px)
        hipExtLaunchKernelGGL((k_sweep_bulk<S, TX, false, NT, true>), g, b, 0, s, e0, e1, 0, I, parity);
    else hipExtLaunchKernelGGL((k_sweep_bulk<S, TX, false, NT, false>), g, b, 0, s, e0, e1, 0, I, parity);
}
template <typename S, int TX, bool NT>
void bulk_batch(const BatchGrid& G, int parity, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (G.hoff)
        hipExtLaunchKernelGGL((kb_sweep_bulk_cut<S, TX, NT>), dim3(G.hoff->off[G.n]), dim3(256), 0, s, e0, e1, 0, G.tab,
                              *G.hoff, G.n, parity);
    else
        hipExtLaunchKernelGGL((kb_sweep_bulk<S, TX, NT>), dim3(G.blocks), dim3(256), 0, s, e0, e1, 0, G.tab, G.off, G.n,
                              parity);
}
template <typename S, int TX, bool NT>
void bulk_go(const Inst* I, const BatchGrid* G, int parity, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int layers) {
    if (I) bulk_one<S, TX, NT>(*I, parity, s, e0, e1, layers);
    else bulk_batch<S, TX, NT>(*G, parity, s, e0, e1);
}
template <typename S, bool NT>
void bulk_tx(int tile_x, const Inst* I, const BatchGrid* G, int parity, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
             int layers) {
    switch (tile_x) {
    case 32: bulk_go<S, 32, NT>(I, G, parity, s, e0, e1, layers); break;
    case 128: bulk_go<S, 128, NT>(I, G, parity, s, e0, e1, layers); break;
    case 0: bulk_go<S, 0, NT>(I, G, parity, s, e0, e1, layers); break;
    default: bulk_go<S, 64, NT>(I, G, parity, s, e0, e1, layers); break;
    }
}
template <typename S>
void bulk_nt(int tile_x, bool nt, const Inst* I, const BatchGrid* G, int parity, hipStream_t s, hipEvent_t e0,
             hipEvent_t e1, int layers) {
    if (nt) bulk_tx<S, true>(tile_x, I, G, parity, s, e0, e1, layers);
    else bulk_tx<S, false>(tile_x, I, G, parity, s, e0, e1, layers);
}
void bulk_dispatch(int storage, int tile_x, bool nt, const Inst* I, const BatchGrid* G, int parity, hipStream_t s,
                   hipEvent_t e0, hipEvent_t e1, int layers) {
    switch (storage) {
    case LBM_FP16_DEV: bulk_nt<__half>(tile_x, nt, I, G, parity, s, e0, e1, layers); break;
    case LBM_BF16_DEV: bulk_nt<__hip_bfloat16>(tile_x, nt, I, G, parity, s, e0, e1, layers); break;
    default: bulk_nt<float>(tile_x, nt, I, G, parity, s, e0, e1, layers); break;
    }
}
}  // namespace

void launch_sweep_bulk(const Inst& I, int parity, int tile_x, bool nt, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                       int layers) {
    bulk_dispatch(I.storage, tile_x, nt, &I, nullptr, parity, s, e0, e1, layers);
}

void launch_sweep_bulk_batch(const BatchGrid& G, int storage, int tile_x, bool nt, int parity, hipStream_t s,
                             hipEvent_t e0, hipEvent_t e1) {
    bulk_dispatch(storage, tile_x, nt, nullptr, &G, parity, s, e0, e1, 0);
}

namespace {
template <typename S, bool W>
void boundary_one(const Inst& I, int parity, int layout, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const dim3 g(boundary_blocks(I)), b(256);
    if (layout && bnd_buf_fits(I, sizeof(S)))
        hipExtLaunchKernelGGL((k_sweep_boundary1<S, W, true>), g, b, 0, s, e0, e1, 0, I, parity);
    else if (layout) hipExtLaunchKernelGGL((k_sweep_boundary1<S, W, false>), g, b, 0, s, e0, e1, 0, I, parity);
    else hipExtLaunchKernelGGL((k_sweep_boundary<S, W>), g, b, 0, s, e0, e1, 0, I, parity);
}

// workgroups of the persistent batch boundary grid: what the chip holds at
// once (one workgroup per CU per wavefront a SIMD keeps), at most one per
// slot of the instances' grids
int persistent_blocks(const BatchGrid& G, int per_cu) { return std::max(1, std::min(G.blocks, device_cus() * per_cu)); }

template <typename S>
void boundary_batch(const BatchGrid& G, int parity, int layout, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const dim3 b(256);
    if (layout && G.buf_fits)
        hipExtLaunchKernelGGL((kb_sweep_boundary1<S, true>), dim3(persistent_blocks(G, LGS_BND1_WAVES)), b, 0, s, e0, e1, 0, G.tab,
                              G.n, parity);
    else if (layout)
        hipExtLaunchKernelGGL((kb_sweep_boundary1<S, false>), dim3(persistent_blocks(G, LGS_BND1_WAVES)), b, 0, s, e0, e1, 0, G.tab,
                              G.n, parity);
    else hipExtLaunchKernelGGL(kb_sweep_boundary<S>, dim3(persistent_blocks(G, 3)), b, 0, s, e0, e1, 0, G.tab, G.n, parity);
}
}  // namespace

void launch_sweep_boundary(const Inst& I, int parity, int layout, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    const bool w = I.wall_moving != 0;
    switch (I.storage) {
    case LBM_FP16_DEV:
        w ? boundary_one<__half, true>(I, parity, layout, s, e0, e1) : boundary_one<__half, false>(I, parity, layout, s, e0, e1);
        break;
    case LBM_BF16_DEV:
        w ? boundary_one<__hip_bfloat16, true>(I, parity, layout, s, e0, e1)
          : boundary_one<__hip_bfloat16, false>(I, parity, layout, s, e0, e1);
        break;
    default:
        w ? boundary_one<float, true>(I, parity, layout, s, e0, e1) : boundary_one<float, false>(I, parity, layout, s, e0, e1);
        break;
    }
}

void launch_sweep_boundary_batch(const BatchGrid& G, int storage, int parity, int layout, hipStream_t s, hipEvent_t e0,
                                 hipEvent_t e1) {
    switch (storage) {
    case LBM_FP16_DEV: boundary_batch<__half>(G, parity, layout, s, e0, e1); break;
    case LBM_BF16_DEV: boundary_batch<__hip_bfloat16>(G, parity, layout, s, e0, e1); break;
    default: boundary_batch<float>(G, parity, layout, s, e0, e1); break;
    }
}

// Candidate scan without a sweep (conversion phase on injected fields).
__global__ __launch_bounds__(256) void k_mark(Inst I, int parity) {
    StepCounters& C = I.ctl->cnt[parity];
    const int id = blockIdx.x * 256 + threadIdx.x;
    bool cand = false, strd = false;
    if (id < I.N) {
        const uint8_t fl = I.flags[id];
        uint8_t mark = 0;
        if ((fl & TYPE_MASK) == IFC) {
            // rho - 1 for the conversion phase (as the sweep leaves it)
            float dr = 0.f;
            switch (I.storage) {
            case LBM_FP16_DEV:
                for (int i = 0; i < Q; ++i)
                    dr += Store<__half>::ld((const __half*)pop_of(I, parity ^ 1), (size_t)i * I.ps + id, I.inv_scale);
                break;
            case LBM_BF16_DEV:
                for (int i = 0; i < Q; ++i)
                    dr += Store<__hip_bfloat16>::ld((const __hip_bfloat16*)pop_of(I, parity ^ 1), (size_t)i * I.ps + id,
                                                    I.inv_scale);
                break;
            default:
                for (int i = 0; i < Q; ++i)
                    dr += Store<float>::ld((const float*)pop_of(I, parity ^ 1), (size_t)i * I.ps + id, I.inv_scale);
                break;
            }
            I.aux[id] = dr;
            int x, y, z;
            cell_coords(I, id, x, y, z);
            bool liq = false;
            for (int i = 1; i < Q; ++i) {
                const int nb = nbr_index(I, x, y, z, cx(i), cy(i), cz(i));
                if (nb >= 0 && (I.flags[nb] & TYPE_MASK) == LIQ) liq = true;
            }
            const double ph = (double)phi_of(I, parity ^ 1)[id];
            if (ph >= 1.0 + I.eps) mark = MARK_FILL;
            else if (ph <= -I.eps) mark = MARK_EMPTY;
            I.lnb[id] = (uint8_t)liq;
            strd = !mark && !liq;
        }
        cand = mark != 0;
        const uint8_t nf = (fl & KEEP_MASK) | mark;
        if (nf != fl) I.flags[id] = nf;
    }
    wave_append(cand, id, I.cand, &C.n_cand, I.list_cap, &C.overflow);
    wave_append(strd, id, I.recv, &C.n_strd, I.list_cap, &C.overflow);
}

void launch_mark(const Inst& I, int parity, hipStream_t s) {
    hipLaunchKernelGGL(k_mark, dim3((I.N + 255) / 256), dim3(256), 0, s, I, parity);
}

}  // namespace lgs
