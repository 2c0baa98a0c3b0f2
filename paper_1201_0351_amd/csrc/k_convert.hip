// k_convert.hip -- free-surface cell conversions (Sec. 2.2) on the state at
// t+1, driven by the candidate list the sweep built, plus the end of a step.
//
// One workgroup of 1024 threads runs the phases one after the other,
// separated by workgroup barriers (candidate lists are short: a few to a few
// thousand cells per step).  Per-cell work is spread over a 32-lane group
// (lane i looks at neighbour x + c_i, or population i), so a cell costs a
// few dependent memory round trips, not a serial walk over its neighbours.
// Each phase is a function of the state before it, so the result does not
// depend on the order of the (atomically appended) lists:
//   forces  the boundary sweep's per-workgroup momentum-exchange records are
//           summed per body in slot order (fixed-order FP64 reduction); the
//           records are loaded before the claims and summed after them
//   bodies  (last wavefront, beside new-gas) retire the step's body moves;
//           free bodies take the rigid-body update from the reduced force
//           and torque
//   claim   per candidate: a filled cell (phi >= 1+eps) records its excess
//           m - rho and claims its gas neighbours as new interface cells; an
//           emptied cell (phi <= -eps) touching a filled one stays interface
//           (filling wins), otherwise it records its excess m and claims its
//           liquid neighbours as new interface cells (m = rho).  Claims go
//           through a bitmap, so every new cell is listed once.
//   newgas  each new cell from gas: f = f_eq(mean rho, mean u) over its
//           neighbours that are liquid or interface and not emptying, m = 0
//   share   per converted cell: count the neighbours that are interface after
//           the conversion (a function of the flags, marks and claims), divide
//           the excess among them and list them as receivers; with none the
//           excess leaves the fluid (ledger).
//   commit  receivers add the shares of their converted neighbours in link
//           order i = 1..18 and recompute phi = m / rho; converted and new
//           cells take their new types.  Converted cells keep their mark until
//           the next sweep clears it.
//   finish  clear the other parity's counters.
#include <cstddef>

#include "lgs_internal.h"

namespace lgs {

namespace {

constexpr int CONV_THREADS = 1024;

__device__ __forceinline__ bool claim(uint32_t* bits, int id) {
    const uint32_t m = 1u << (id & 31);
    return (atomicOr(bits + (id >> 5), m) & m) == 0;
}
__device__ __forceinline__ bool claimed(const uint32_t* bits, int id) {
    return (__hip_atomic_load(bits + (id >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> (id & 31)) & 1u;
}
__device__ __forceinline__ int load_count(int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Clear the whole bitmap word of a claimed cell with a plain store: for use
// only where every bit set in the bitmap is being cleared in the same phase
// and none is read or set there.
__device__ __forceinline__ void unclaim_word(uint32_t* bits, int id) { bits[id >> 5] = 0u; }
// add the number of calling lanes with `on` set to *cnt (one atomic per
// wavefront)
__device__ __forceinline__ void wave_count(bool on, int* cnt) {
    const unsigned long long m = __ballot(on);
    if (m && (threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicAdd(cnt, __popcll(m));
}

__device__ __forceinline__ void push(int* list, int* cnt, int cap, int* overflow, int id) {
    const int p = atomicAdd(cnt, 1);
    if (p < cap) list[p] = id;
    else atomicOr(overflow, 1);
}

template <typename S>
__device__ __forceinline__ void moments(const Inst& I, const S* pop, int id, float& drho, float u[3]) {
    float dr = 0.f, j0 = 0.f, j1 = 0.f, j2 = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float v = Store<S>::ld(pop, (size_t)i * I.ps + id, I.inv_scale);
        dr += v;
        j0 += cx(i) * v;
        j1 += cy(i) * v;
        j2 += cz(i) * v;
    }
    drho = dr;
    const float r = 1.f + dr;
    u[0] = j0 / r;
    u[1] = j1 / r;
    u[2] = j2 / r;
}

template <typename S>
__device__ __forceinline__ float drho_of(const Inst& I, const S* pop, int id) {
    float dr = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) dr += Store<S>::ld(pop, (size_t)i * I.ps + id, I.inv_scale);
    return dr;
}

__device__ __forceinline__ void add_comp(float& hi, float& lo, float v) {
    const float s = hi + v;
    const float bp = s - hi;
    const float err = (hi - (s - bp)) + (v - bp);
    const float l = lo + err;
    const float h = s + l;
    lo = l - (h - s);
    hi = h;
}

__device__ __forceinline__ bool has_fill_neighbour(const Inst& I, int x, int y, int z) {
    for (int i = 1; i < Q; ++i) {
        const int nb = nbr_index(I, x, y, z, cx(i), cy(i), cz(i));
        if (nb >= 0 && (I.flags[nb] & MARK_FILL)) return true;
    }
    return false;
}

// an interface cell that will become gas in this conversion phase
__device__ __forceinline__ bool empties(const Inst& I, int id, uint8_t f) {
    if (!(f & MARK_EMPTY)) return false;
    int x, y, z;
    cell_coords(I, id, x, y, z);
    return !has_fill_neighbour(I, x, y, z);
}

// type of a neighbour after this conversion phase (flags, marks and claims
// are not modified while the share kernel runs)
__device__ __forceinline__ int post_type(const Inst& I, int id) {
    const uint8_t f = I.flags[id];
    const int t = f & TYPE_MASK;
    if (t == IFC) return (f & MARK_FILL) ? LIQ : ((f & MARK_EMPTY) ? GAS : IFC);
    if ((t == GAS || t == LIQ) && claimed(I.claim, id)) return IFC;
    return t;
}

#define BLOCK_LOOP(k, n) for (int k = threadIdx.x; k < (n); k += blockDim.x)

}  // namespace

// group-aggregated append (one atomic per group)
__device__ __forceinline__ void g_push(bool pred, int id, int* list, int* cnt, int cap, int* overflow) {
    const unsigned m = g_ballot(pred);
    if (m == 0) return;
    const int leader = __ffs(m) - 1;
    int base = 0;
    if (g_lane() == leader) base = atomicAdd(cnt, __popc(m));
    base = g_bcast(base, leader);
    if (pred) {
        const int pos = base + __popc(m & ((1u << g_lane()) - 1u));
        if (pos < cap) list[pos] = id;
        else atomicOr(overflow, 1);
    }
}

// neighbour x + c_i of the calling lane's link (lanes 1..18), else -1
__device__ __forceinline__ int lane_nbr(const Inst& I, int x, int y, int z) {
    const int i = g_lane();
    if (i < 1 || i >= Q) return -1;
    return nbr_index(I, x, y, z, lane_c(CXP, i), lane_c(CYP, i), lane_c(CZP, i));
}

// claim: one 32-lane group per candidate, lane i looks at neighbour x + c_i.
template <typename S>
__device__ __forceinline__ void phase_claim(const Inst& I, int parity, int g0, int ngroups) {
    StepCounters& C = I.ctl->cnt[parity];
    const int n = min(load_count(&C.n_cand), I.list_cap);
    const int i = g_lane();
    for (int k = g0; k < n; k += ngroups) {
        const int id = I.cand[k];
        const uint8_t fl = I.flags[id];
        int x, y, z;
        cell_coords(I, id, x, y, z);
        const int nb = lane_nbr(I, x, y, z);
        const uint8_t nf = nb >= 0 ? I.flags[nb] : 0;
        if (fl & MARK_FILL) {
            if (i == 0) {
                const float dr = I.aux[id];  // rho - 1 left by the sweep
                I.share[id] = (float)(((double)I.m_hi[id] - 1.0) + ((double)I.m_lo[id] - (double)dr));
            }
            const bool take = nb >= 0 && (nf & TYPE_MASK) == GAS && claim(I.claim, nb);
            g_push(take, nb, I.newg, &C.n_newg, I.list_cap, &C.overflow);
        } else if (fl & MARK_EMPTY) {
            if (g_ballot(nb >= 0 && (nf & MARK_FILL))) {
                if (i == 0) I.flags[id] = fl & (uint8_t)~MARK_EMPTY;  // filling wins: stays interface
                continue;
            }
            if (i == 0) I.share[id] = (float)((double)I.m_hi[id] + (double)I.m_lo[id]);
            const bool take = nb >= 0 && (nf & TYPE_MASK) == LIQ && claim(I.claim, nb);
            g_push(take, nb, I.newl, &C.n_newl, I.list_cap, &C.overflow);
        }
    }
}

// New interface cells from gas: equilibrium of the mean density and
// velocity of their liquid / interface neighbours that are not emptying
// (one group per new cell, lane j looks at neighbour j); m = 0.  New
// interface cells from liquid (one thread each): m = rho, phi = 1.
template <typename S>
__device__ __forceinline__ void phase_newgas(const Inst& I, int parity, int g0, int ngroups) {
    StepCounters& C = I.ctl->cnt[parity];
    const int n = min(load_count(&C.n_newg), I.list_cap);
    S* pop = (S*)pop_of(I, parity ^ 1);
    float* phi = phi_of(I, parity ^ 1);
    const int j = g_lane();
    for (int k = g0; k < n; k += ngroups) {
        const int g = I.newg[k];
        int gx, gy, gz;
        cell_coords(I, g, gx, gy, gz);
        const int nb = lane_nbr(I, gx, gy, gz);
        bool use = false;
        if (nb >= 0) {
            const uint8_t f = I.flags[nb];
            const int t = f & TYPE_MASK;
            use = (t == LIQ || t == IFC) && !empties(I, nb, f);
        }
        float d = 0.f, u0 = 0.f, u1 = 0.f, u2 = 0.f;
        if (use) {
            float u[3];
            moments<S>(I, pop, nb, d, u);
            u0 = u[0];
            u1 = u[1];
            u2 = u[2];
        }
        const int ns = __popc(g_ballot(use));
        const float rs = gsum(d), us0 = gsum(u0), us1 = gsum(u1), us2 = gsum(u2);
        const float inv = 1.f / (float)max(ns, 1);
        const float drb = ns > 0 ? rs * inv : I.rho_g - 1.f, rb = 1.f + drb;
        const float v0 = us0 * inv, v1 = us1 * inv, v2 = us2 * inv;
        const float uu = v0 * v0 + v1 * v1 + v2 * v2;
        if (j < Q) {
            const float cu = lane_c(CXP, j) * v0 + lane_c(CYP, j) * v1 + lane_c(CZP, j) * v2;
            const float deq = lane_w(j) * (drb + rb * (3.f * cu + 4.5f * cu * cu - 1.5f * uu));
            Store<S>::st(pop, (size_t)j * I.ps + g, deq, I.scale);
        }
        if (j == 0) {
            I.m_hi[g] = 0.f;
            I.m_lo[g] = 0.f;
            I.aux[g] = drb;
            phi[g] = 0.f;
        }
    }
    const int nl = min(load_count(&C.n_newl), I.list_cap);
    for (int k = g0 * 32 + g_lane(); k < nl; k += ngroups * 32) {
        const int id = I.newl[k];
        const float dr = drho_of<S>(I, pop, id);
        I.m_hi[id] = 1.f;
        I.m_lo[id] = dr;
        I.aux[id] = dr;
        phi[id] = 1.f;
    }
}

// share: one group per converted cell; lane i counts neighbour x + c_i if it
// is interface after the conversions (flags, marks and claims are not
// modified in this phase).
__device__ __forceinline__ void phase_share(const Inst& I, int parity) {
    StepCounters& C = I.ctl->cnt[parity];
    const int nc = min(load_count(&C.n_cand), I.list_cap);
    const int grp = threadIdx.x >> 5, ngrp = blockDim.x >> 5;
    for (int k = grp; k < nc; k += ngrp) {
        const int id = I.cand[k];
        const uint8_t fl = I.flags[id];
        if (!(fl & (MARK_FILL | MARK_EMPTY))) continue;
        int x, y, z;
        cell_coords(I, id, x, y, z);
        const int nb = lane_nbr(I, x, y, z);
        const bool rcv = nb >= 0 && post_type(I, nb) == IFC;
        const int nr = __popc(g_ballot(rcv));
        if (nr == 0) {
            if (g_lane() == 0) {
                atomicAdd(&I.ctl->ledger, -(double)I.share[id]);
                I.share[id] = 0.f;
            }
            continue;
        }
        if (g_lane() == 0) I.share[id] = (float)((double)I.share[id] / nr);
        // the receiver notes this converted neighbour (its link opp(i));
        // the first note puts it on the list
        const bool first = rcv && atomicOr(&I.cmask[nb], 1u << lane_opp(g_lane())) == 0u;
        g_push(first, nb, I.recv, &C.n_recv, I.list_cap, &C.overflow);
    }
}

// commit: converted and new cells take their new types; receivers add the
// shares of their converted neighbours in link order i = 1..18 and
// recompute phi = m / rho.
template <typename S>
__device__ __forceinline__ void phase_commit(const Inst& I, int parity) {
    StepCounters& C = I.ctl->cnt[parity];
    const int nc = min(load_count(&C.n_cand), I.list_cap), ng = min(load_count(&C.n_newg), I.list_cap);
    const int nl = min(load_count(&C.n_newl), I.list_cap), nr = min(load_count(&C.n_recv), I.list_cap);
    float* phi = phi_of(I, parity ^ 1);
    // single-thread items; the claim bits of the new cells are the only
    // bits set in I.claim, and all of them are cleared here
    for (int k0 = 0; k0 < nc + ng + nl; k0 += blockDim.x) {
        const int k = k0 + (int)threadIdx.x;
        bool f = false, e = false, g = false, l = false;
        if (k < nc) {
            const int id = I.cand[k];
            const uint8_t fl = I.flags[id];
            if (fl & MARK_FILL) {
                I.flags[id] = LIQ | MARK_FILL;
                I.m_hi[id] = 0.f;
                I.m_lo[id] = 0.f;
                phi[id] = 1.f;
                f = true;
            } else if (fl & MARK_EMPTY) {
                I.flags[id] = GAS | MARK_EMPTY;
                I.m_hi[id] = 0.f;
                I.m_lo[id] = 0.f;
                phi[id] = 0.f;
                e = true;
            }
        } else if (k < nc + ng + nl) {
            g = k < nc + ng;
            l = !g;
            const int id = g ? I.newg[k - nc] : I.newl[k - nc - ng];
            I.flags[id] = IFC;
            unclaim_word(I.claim, id);
        }
        wave_count(f, &C.filled);
        wave_count(e, &C.emptied);
        wave_count(g, &C.newg);
        wave_count(l, &C.newl);
    }
    // receivers, one thread each: the note mask names the converted
    // neighbours, whose shares are added in link order; rho - 1 of every
    // receiver is in I.aux (left by the sweep for interface cells, by the
    // claim and new-gas phases for new ones)
    BLOCK_LOOP(k, nr) {
        const int id = I.recv[k];
        const uint32_t m = I.cmask[id];
        int x, y, z;
        cell_coords(I, id, x, y, z);
        float sh[Q];
#pragma unroll
        for (int l = 1; l < Q; ++l) {
            sh[l] = 0.f;
            if ((m >> l) & 1u) sh[l] = I.share[nbr_index(I, x, y, z, cx(l), cy(l), cz(l))];
        }
        float hi = I.m_hi[id], lo = I.m_lo[id];
        const float dr = I.aux[id];
#pragma unroll
        for (int l = 1; l < Q; ++l)
            if ((m >> l) & 1u) add_comp(hi, lo, sh[l]);
        I.m_hi[id] = hi;
        I.m_lo[id] = lo;
        phi[id] = (float)(((double)hi + (double)lo) / (1.0 + (double)dr));
        I.cmask[id] = 0u;
    }
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Fixed-order FP64 sum of the boundary sweep's force records, per body, in
// three parts so that its memory round trip overlaps the claim phase:
//   load     every thread loads its records (slots tid + j * CONV_THREADS)
//            and threads t < 6 nbodies the accumulator entry they finish
//   partial  per body: the thread's records in slot order, wavefront
//            butterflies, one partial per wavefront in LDS
//   final    (after a barrier) acc = loaded entry + partials in wavefront order
struct ForceLoad {
    static constexpr int PER = BND_BLOCKS_MAX / CONV_THREADS;
    int rb[PER];
    double rv[PER][6];
    double acc0;
};
static_assert(ForceLoad::PER * CONV_THREADS == BND_BLOCKS_MAX, "force records per thread");
constexpr int CONV_WAVES = CONV_THREADS / 64;

__device__ __forceinline__ void forces_load(const Inst& I, int parity, ForceLoad& F) {
    const int nrec = boundary_blocks(I);
#pragma unroll
    for (int j = 0; j < ForceLoad::PER; ++j) {
        const int k = threadIdx.x + j * CONV_THREADS;
        F.rb[j] = k < nrec ? I.frec_body[k] : -1;
#pragma unroll
        for (int q = 0; q < 6; ++q) F.rv[j][q] = k < nrec ? I.frec_v[q * BND_BLOCKS_MAX + k] : 0.0;
    }
    const int t = threadIdx.x;
    F.acc0 = t < 6 * I.nbodies ? I.ctl->cnt[parity].acc[t / 6][t % 6] : 0.0;
}

__device__ __forceinline__ void forces_partial(const Inst& I, const ForceLoad& F, double (*part)[MAXB][6]) {
    for (int b = 0; b < I.nbodies; ++b) {
        double v[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < ForceLoad::PER; ++j)
            if (F.rb[j] == b)
#pragma unroll
                for (int q = 0; q < 6; ++q) v[q] += F.rv[j][q];
#pragma unroll
        for (int q = 0; q < 6; ++q) v[q] = wave_sum_d(v[q]);
        if ((threadIdx.x & 63) == 0)
#pragma unroll
            for (int q = 0; q < 6; ++q) part[threadIdx.x >> 6][b][q] = v[q];
    }
}

__device__ __forceinline__ void forces_final(const Inst& I, int parity, const ForceLoad& F,
                                             const double (*part)[MAXB][6], double (*sacc)[6]) {
    const int t = threadIdx.x;
    if (t < 6 * I.nbodies) {
        double s = F.acc0;
#pragma unroll
        for (int w = 0; w < CONV_WAVES; ++w) s += part[w][t / 6][t % 6];
        I.ctl->cnt[parity].acc[t / 6][t % 6] = s;
        sacc[t / 6][t % 6] = s;  // the body update reads it from here
    }
}

// the whole sum at once (phase-isolated calls)
__device__ __forceinline__ void phase_forces(const Inst& I, int parity, double (*sacc)[6]) {
    __shared__ double part[CONV_WAVES][MAXB][6];
    ForceLoad F;
    forces_load(I, parity, F);
    forces_partial(I, F, part);
    __syncthreads();
    forces_final(I, parity, F, part, sacc);
    __syncthreads();
}

// Copy of the body records in LDS, written by one wavefront (32-bit words),
// so that the body update does not wait on global memory after the force
// reduction.
__device__ __forceinline__ void stage_bodies(const Inst& I, DevBody* sb) {
    static_assert(sizeof(DevBody) % 4 == 0, "body record in 32-bit words");
    const int nw = I.nbodies * (int)(sizeof(DevBody) / 4);
    const uint32_t* src = (const uint32_t*)I.bodies;
    uint32_t* dst = (uint32_t*)sb;
    for (int w = threadIdx.x & 63; w < nw; w += 64) dst[w] = src[w];
}

// clear the other parity's counters
__device__ __forceinline__ void phase_finish(const Inst& I, int parity) {
    StepCounters& O = I.ctl->cnt[parity ^ 1];
    int* ci = (int*)&O;
    const int nint = (int)(offsetof(StepCounters, acc) / sizeof(int));
    for (int q = threadIdx.x; q < nint; q += blockDim.x) ci[q] = 0;
    for (int q = threadIdx.x; q < MAXB * 6; q += blockDim.x) (&O.acc[0][0])[q] = 0.0;
}

// Bodies after the force reduction of a full step, run by one wavefront
// (lane b owns body b).  A body remapped at the start of the step now has
// its obstacle cells at its pose (retire the move).  Free bodies then take
// the rigid-body update driven by the mean of this and the previous step's
// force and torque; the new pose is mapped by the next step's remap.  An
// update that would leave the domain's interior, reach one cell per step at
// the surface, jump a cell from the mapped pose or bring two bodies closer
// than three cells is rejected: the body keeps its pose and Ctl::body_err
// records why.
// The inputs come from the LDS copies of the body records (sb, staged at the
// kernel's start) and of the reduced force and torque (sacc); the results go
// to the records in global memory.
__device__ __forceinline__ void bodies_wave(const Inst& I, bool retire_moves, bool integrate, const DevBody* sb,
                                            const double (*sacc)[6]) {
    const int b = threadIdx.x & 63;
    const bool mine = b < I.nbodies;
    double pos[3] = {0, 0, 0}, quat[4] = {1, 0, 0, 0}, vel[3] = {0, 0, 0}, om[3] = {0, 0, 0}, ext[3] = {0, 0, 0};
    double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    double prev[3] = {0, 0, 0};
    bool upd = false, act = false, mapped = false;
    if (mine) {
        const DevBody& S = sb[b];
        DevBody& B = I.bodies[b];
        act = S.active != 0;
        mapped = S.mapped != 0;
        for (int a = 0; a < 3; ++a) prev[a] = S.prev_pos[a];
        if (retire_moves && S.moved) {
            B.moved = 0;
            B.mapped = 1;
            mapped = true;
            for (int a = 0; a < 3; ++a) {
                B.prev_pos[a] = S.pos[a];
                B.prev_ext[a] = S.ext[a];
                prev[a] = S.pos[a];
            }
        }
        for (int a = 0; a < 3; ++a) {
            pos[a] = S.pos[a];
            ext[a] = S.ext[a];
        }
        if (integrate && S.active && S.free_body && S.dof) {
            const double* acc = sacc[b];
            double F[3], T[3];
            for (int a = 0; a < 3; ++a) {
                F[a] = S.have_prev ? 0.5 * (acc[a] + S.fprev[a]) : acc[a];
                T[a] = S.have_prev ? 0.5 * (acc[3 + a] + S.fprev[3 + a]) : acc[3 + a];
            }
            for (int a = 0; a < 6; ++a) B.fprev[a] = acc[a];
            B.have_prev = 1;
            const double accel[3] = {(double)I.ax, (double)I.ay, (double)I.az};
            upd = integrate_rigid(S.shape, S.half, S.pos, S.quat, S.vel, S.omega, S.density, F, T, accel, S.dof, pos,
                                  quat, vel, om);
            if (upd) {
                const double n[3] = {(double)I.nx, (double)I.ny, (double)I.nz};
                for (int a = 0; a < 3; ++a)
                    if (I.periodic & (1u << a)) pos[a] = pos[a] - n[a] * floor(pos[a] / n[a]);
                quat_to_R(quat, R);
                box_extent(S.shape, R, S.half, ext);
            }
        }
    }
    // separation from every other body at its (new) pose
    const double n[3] = {(double)I.nx, (double)I.ny, (double)I.nz};
    bool close = false;
    for (int j = 0; j < I.nbodies; ++j) {
        const bool aj = __shfl((int)act, j) != 0;
        bool sep = false;
        for (int a = 0; a < 3; ++a) {
            const double pj = __shfl(pos[a], j), ej = __shfl(ext[a], j);
            const double dd = wrap_rel(pos[a] - pj, n[a], I.periodic & (1u << a));
            if (fabs(dd) >= ext[a] + ej + 3.0) sep = true;
        }
        if (j != b && aj && !sep) close = true;
    }
    if (upd) {
        const DevBody& S = sb[b];
        DevBody& B = I.bodies[b];
        int err = close ? BODY_ERR_CLOSE : 0;
        const double Rc = sqrt(S.half[0] * S.half[0] + S.half[1] * S.half[1] + S.half[2] * S.half[2]);
        const double speed = sqrt(vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2]) +
                             sqrt(om[0] * om[0] + om[1] * om[1] + om[2] * om[2]) * Rc;
        if (!(speed < 1.0)) err |= BODY_ERR_SPEED;
        for (int a = 0; a < 3; ++a) {
            const bool per = I.periodic & (1u << a);
            if (per) {
                if (2.0 * ext[a] >= n[a] && !(S.half[a] >= 0.5 * n[a] && ext[a] == S.half[a])) err |= BODY_ERR_WALL;
            } else if (!(pos[a] - ext[a] >= 1.0 && pos[a] + ext[a] <= n[a] - 1.0)) {
                err |= BODY_ERR_WALL;
            }
            if (mapped && !(fabs(wrap_rel(pos[a] - prev[a], n[a], per)) < 1.0)) err |= BODY_ERR_JUMP;
        }
        if (err) {
            atomicOr(&I.ctl->body_err, err);
        } else {
            for (int a = 0; a < 3; ++a) {
                B.pos[a] = pos[a];
                B.vel[a] = vel[a];
                B.omega[a] = om[a];
                B.ext[a] = ext[a];
            }
            for (int a = 0; a < 4; ++a) B.quat[a] = quat[a];
            for (int a = 0; a < 9; ++a) B.R[a] = R[a];
            B.moved = 1;
        }
    }
}

// One step's conversions.  The last wavefront updates the bodies while the
// others claim; the later phases use all groups.
// The force records are loaded first and reduced after the claims, so their
// round trip overlaps the claim phase; the body update (last wavefront)
// overlaps the new-gas phase (the other wavefronts).
template <typename S>
__device__ __forceinline__ void convert(const Inst& I, int parity, bool retire_moves, bool integrate) {
    __shared__ double part[CONV_WAVES][MAXB][6];
    __shared__ double sacc[MAXB][6];
    __shared__ DevBody sb[MAXB];
    const bool last = (int)(threadIdx.x >> 6) == CONV_WAVES - 1;
    constexpr int WORK_GROUPS = CONV_THREADS / 32 - 2;  // the 32-lane groups of all but the last wavefront
    ForceLoad F;
    forces_load(I, parity, F);
    if (!last) phase_claim<S>(I, parity, threadIdx.x >> 5, WORK_GROUPS);
    else stage_bodies(I, sb);
    forces_partial(I, F, part);
    __syncthreads();
    forces_final(I, parity, F, part, sacc);
    __syncthreads();
    if (last) bodies_wave(I, retire_moves, integrate, sb, sacc);
    else phase_newgas<S>(I, parity, threadIdx.x >> 5, WORK_GROUPS);
    __syncthreads();
    phase_share(I, parity);
    __syncthreads();
    phase_commit<S>(I, parity);
    __syncthreads();
    phase_finish(I, parity);
}

template <typename S>
__global__ __launch_bounds__(CONV_THREADS) void k_convert(Inst I, int parity, int retire_moves, int integrate) {
    convert<S>(I, parity, retire_moves != 0, integrate != 0);
}

// one workgroup per instance of a batch (at most 64: bit k of the masks
// belongs to instance k)
template <typename S>
__global__ __launch_bounds__(CONV_THREADS) void kb_convert(const Inst* __restrict__ tab, int parity,
                                                          unsigned long long retire_mask,
                                                          unsigned long long integrate_mask) {
    const int k = blockIdx.x;
    const Inst I = tab[k];
    convert<S>(I, parity, (retire_mask >> k) & 1ull, (integrate_mask >> k) & 1ull);
}

// End of a step without conversions (phase-isolated calls).
__global__ __launch_bounds__(CONV_THREADS) void k_finish(Inst I, int parity, int reduce, int zero_other,
                                                         int retire_moves) {
    __shared__ double sacc[MAXB][6];
    __shared__ DevBody sb[MAXB];
    if (threadIdx.x < 64) stage_bodies(I, sb);
    if (reduce) phase_forces(I, parity, sacc);
    __syncthreads();
    if (threadIdx.x < 64) bodies_wave(I, retire_moves != 0, false, sb, sacc);
    if (zero_other) phase_finish(I, parity);
}

void launch_convert_batch(const Inst* tab, int n, int storage, int parity, unsigned long long retire_mask,
                          unsigned long long integrate_mask, hipStream_t s) {
    const dim3 g(n), b(CONV_THREADS);
    switch (storage) {
    case LBM_FP16_DEV: hipLaunchKernelGGL(kb_convert<__half>, g, b, 0, s, tab, parity, retire_mask, integrate_mask); break;
    case LBM_BF16_DEV:
        hipLaunchKernelGGL(kb_convert<__hip_bfloat16>, g, b, 0, s, tab, parity, retire_mask, integrate_mask);
        break;
    default: hipLaunchKernelGGL(kb_convert<float>, g, b, 0, s, tab, parity, retire_mask, integrate_mask); break;
    }
}

void launch_convert(const Inst& I, int parity, bool retire_moves, bool integrate, hipStream_t s) {
    const dim3 g(1), b(CONV_THREADS);
    const int r = (int)retire_moves, n = (int)integrate;
    switch (I.storage) {
    case LBM_FP16_DEV: hipLaunchKernelGGL(k_convert<__half>, g, b, 0, s, I, parity, r, n); break;
    case LBM_BF16_DEV: hipLaunchKernelGGL(k_convert<__hip_bfloat16>, g, b, 0, s, I, parity, r, n); break;
    default: hipLaunchKernelGGL(k_convert<float>, g, b, 0, s, I, parity, r, n); break;
    }
}

void launch_finish(const Inst& I, int parity, bool reduce, bool zero_other, bool retire_moves, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(CONV_THREADS), 0, s, I, parity, (int)reduce, (int)zero_other,
                       (int)retire_moves);
}

}  // namespace lgs
