// k_convert.hip -- free-surface cell conversions (Sec. 2.2) on the state at
// t+1, driven by the candidate list the sweep built, plus the end of a step.
//
// Three launches over the whole chip, each a pure function of the state the
// launch before it left, so the result does not depend on the order of the
// (atomically appended) lists or on scheduling.  Per-cell work is spread
// over a 32-lane group (lane i looks at neighbour x + c_i, or population i):
//   claim   (one group per candidate) a filled cell (phi >= 1+eps) records
//           its excess m - rho and claims its gas neighbours as new
//           interface cells; an emptied cell (phi <= -eps) touching a filled
//           one stays interface (filling wins: its empty mark is dropped),
//           otherwise it records its excess m and claims its liquid
//           neighbours as new interface cells (m = rho).  Claims go through a
//           bitmap, so every new cell is listed once.  A stranded interface
//           cell (no liquid neighbour, and no interface neighbour that has
//           one) empties as well, unless a neighbour fills.
//   middle  (one group per new cell from gas) f = f_eq(mean rho, mean u) over
//           its neighbours that are liquid or interface and not emptying,
//           m = 0; (one thread per new cell from liquid) m = rho, phi = 1;
//           (one group per converted cell) count the neighbours that are
//           interface after the conversion (a function of the flags, marks
//           and claims), divide the excess among them and note this cell in
//           each receiver's link mask; with none the excess leaves the fluid
//           (ledger).  The last workgroup of the grid instead sums the
//           boundary sweep's momentum-exchange records per body (fixed-point
//           integer sums), retires the step's body moves and gives free
//           bodies the rigid-body update; no conversion reads the bodies.
//   commit  converted and new cells take their new types; receivers add the
//           shares of their converted neighbours in link order i = 1..18 and
//           recompute phi = m / rho.  Converted cells keep their mark until
//           the next sweep clears it.  The other parity's counters are
//           cleared for the next step.
#include <cstddef>

#include "lgs_internal.h"

namespace lgs {

namespace {

constexpr int CT = 256;      // threads per workgroup of the conversion kernels
constexpr int CG = CT / 32;  // 32-lane groups per workgroup
constexpr int CW = CT / 64;  // wavefronts per workgroup

__device__ __forceinline__ bool claim(uint32_t* bits, int id) {
    const uint32_t m = 1u << (id & 31);
    return (atomicOr(bits + (id >> 5), m) & m) == 0;
}
__device__ __forceinline__ bool claimed(const uint32_t* bits, int id) {
    return (bits[id >> 5] >> (id & 31)) & 1u;
}
// Clear the whole bitmap word of a claimed cell with a plain store: for use
// only where every bit set in the bitmap is being cleared in the same launch
// and none is read or set there.
__device__ __forceinline__ void unclaim_word(uint32_t* bits, int id) { bits[id >> 5] = 0u; }
// add the number of calling lanes with `on` set to *cnt (one atomic per
// wavefront; every lane of the wavefront calls it)
__device__ __forceinline__ void wave_count(bool on, int* cnt) {
    const unsigned long long m = __ballot(on);
    if (m && (threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicAdd(cnt, __popcll(m));
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

// Type of a cell after this conversion phase, read between the claim and
// the commit launches: the claim launch has dropped the empty mark of every
// emptied cell that filling overrides, so the marks name exactly the cells
// that convert, and the claim bitmap the new interface cells.
__device__ __forceinline__ int post_type(const Inst& I, int id) {
    const uint8_t f = I.flags[id];
    const int t = f & TYPE_MASK;
    if (t == IFC) return (f & MARK_FILL) ? LIQ : ((f & MARK_EMPTY) ? GAS : IFC);
    if ((t == GAS || t == LIQ) && claimed(I.claim, id)) return IFC;
    return t;
}

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

__device__ __forceinline__ int list_len(const int* cnt, int cap) { return min(*cnt, cap); }
// converted cells after the claim launch: the sweep's candidates, then the
// stranded cells that empty
__device__ __forceinline__ int cand_len(const StepCounters& C, int cap) { return min(C.n_cand + C.n_se, cap); }

}  // namespace

// ---------------------------------------------------------------------------
// force reduction and body update (one workgroup of CT threads)
// ---------------------------------------------------------------------------
namespace {

// Sum of the boundary sweep's force records per body, in fixed point
// (fx_split): thread t takes records t + j CT, then wavefront butterflies,
// then the wavefronts, then the atomics' sums; all integer sums, so the
// result does not depend on their order.  F and T (FP64, formed once from
// the totals) go to the accumulators and to sacc.
__device__ __forceinline__ long long wave_sum_i(long long v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ void reduce_forces(const Inst& I, int parity, double (*sacc)[6]) {
    constexpr int PER = BND_BLOCKS_MAX / CT;
    static_assert(PER * CT == BND_BLOCKS_MAX, "force records per thread");
    __shared__ long long part[CW][MAXB][FXW];
    StepCounters& C = I.ctl->cnt[parity];
    const int nrec = min(boundary_blocks(I), C.n_frec);
    uint32_t mk[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int k = threadIdx.x + j * CT;
        mk[j] = k < nrec ? I.frec_mask[k] : 0u;
    }
    for (int b = 0; b < I.nbodies; ++b) {
        long long v[FXW];
#pragma unroll
        for (int q = 0; q < FXW; ++q) v[q] = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j)
            if ((mk[j] >> b) & 1u) {
                const int k = threadIdx.x + j * CT;
#pragma unroll
                for (int q = 0; q < FXW; ++q) v[q] += I.frec_v[(b * FXW + q) * BND_BLOCKS_MAX + k];
            }
#pragma unroll
        for (int q = 0; q < FXW; ++q) v[q] = wave_sum_i(v[q]);
        if ((threadIdx.x & 63) == 0)
#pragma unroll
            for (int q = 0; q < FXW; ++q) part[threadIdx.x >> 6][b][q] = v[q];
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < 6 * I.nbodies) {
        const int b = t / 6, q = t % 6;
        long long h = C.facc[b][q], l = C.facc[b][6 + q];
#pragma unroll
        for (int w = 0; w < CW; ++w) {
            h += part[w][b][q];
            l += part[w][b][6 + q];
        }
        const double s = fx_value(h, l);
        C.acc[b][q] = s;
        sacc[b][q] = s;
    }
    __syncthreads();
}

// Copy of the body records in LDS (32-bit words, one wavefront), so that the
// body update reads them without a global round trip after the reduction.
__device__ __forceinline__ void stage_bodies(const Inst& I, DevBody* sb) {
    static_assert(sizeof(DevBody) % 4 == 0, "body record in 32-bit words");
    const int nw = I.nbodies * (int)(sizeof(DevBody) / 4);
    const uint32_t* src = (const uint32_t*)I.bodies;
    uint32_t* dst = (uint32_t*)sb;
    for (int w = threadIdx.x & 63; w < nw; w += 64) dst[w] = src[w];
}

// clear the other parity's counters (the next step's)
__device__ __forceinline__ void clear_other(const Inst& I, int parity, int tid, int nthr) {
    StepCounters& O = I.ctl->cnt[parity ^ 1];
    int* ci = (int*)&O;
    const int nint = (int)(offsetof(StepCounters, acc) / sizeof(int));
    for (int q = tid; q < nint; q += nthr) ci[q] = 0;
    for (int q = tid; q < MAXB * 6; q += nthr) (&O.acc[0][0])[q] = 0.0;
    for (int q = tid; q < MAXB * FXW; q += nthr) (&O.facc[0][0])[q] = 0;
}

// Bodies after the force reduction of a full step, run by one wavefront
// (lane b owns body b).  A body remapped at the start of the step now has
// its obstacle cells at its pose (retire the move).  Free bodies then take
// the rigid-body update driven by the mean of this and the previous step's
// force and torque; the new pose is mapped by the next step's remap.  An
// update that would leave the domain's interior, reach one cell per step at
// the surface, jump a cell from the mapped pose or bring two bodies closer
// than three cells is rejected: the body keeps its pose and Ctl::body_err
// records why.  Inputs from the LDS copies of the body records (sb) and of
// the reduced force and torque (sacc); results to the records in global
// memory.
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

// The end of a step's body work in one workgroup: optional fixed-order force
// reduction, then the body update by wavefront 0.
__device__ __forceinline__ void forces_and_bodies(const Inst& I, int parity, bool reduce, bool retire_moves,
                                                  bool integrate) {
    __shared__ double sacc[MAXB][6];
    __shared__ DevBody sb[MAXB];
    if ((int)(threadIdx.x >> 6) == CW - 1) stage_bodies(I, sb);
    if (reduce) reduce_forces(I, parity, sacc);
    __syncthreads();
    if (threadIdx.x < 64) bodies_wave(I, retire_moves, integrate, sb, sacc);
}

// ---------------------------------------------------------------------------
// the three conversion launches; blk of nblk is the workgroup's place in the
// instance's grid
// ---------------------------------------------------------------------------
template <typename S>
__device__ __forceinline__ void conv_claim(const Inst& I, int parity, int blk, int nblk, int bulk_layers = 0) {
    // a bulk grid cut to bulk_layers layers must have covered every layer up
    // to ztop (the sweeps raise no layer; the remap before them already did)
    if (blk == 0 && threadIdx.x == 0 && bulk_layers > 0 && I.ctl->ztop >= bulk_layers)
        atomicOr(&I.ctl->nonfinite, NONFINITE_LAYERS);
    StepCounters& C = I.ctl->cnt[parity];
    const int n = list_len(&C.n_cand, I.list_cap);
    const int ns = list_len(&C.n_strd, I.list_cap);
    const int i = g_lane();
    const int ng = nblk * CG;
    for (int k = blk * CG + (int)(threadIdx.x >> 5); k < n + ns; k += ng) {
        if (k >= n) {
            // a stranded candidate (no liquid neighbour, no mark): it empties
            // unless an interface neighbour has a liquid neighbour (it is an
            // outer cell of a surface two cells thick) or a neighbour fills
            // (filling wins); emptying cells are listed after the sweep's
            // candidates, which this loop does not reach
            const int id = I.recv[k - n];
            int x, y, z;
            cell_coords(I, id, x, y, z);
            const int nb = lane_nbr(I, x, y, z);
            const uint8_t nf = nb >= 0 ? I.flags[nb] : 0;
            const bool keep = nb >= 0 && ((nf & MARK_FILL) || ((nf & TYPE_MASK) == IFC && I.lnb[nb]));
            if (g_ballot(keep)) continue;
            if (i == 0) {
                I.flags[id] = I.flags[id] | MARK_EMPTY;
                I.share[id] = (float)((double)I.m_hi[id] + (double)I.m_lo[id]);
                const int p = n + atomicAdd(&C.n_se, 1);
                if (p < I.list_cap) I.cand[p] = id;
                else atomicOr(&C.overflow, 1);
            }
            continue;
        }
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

// The last workgroup of the middle launch sums the boundary sweep's force
// records and updates the bodies (nothing in this launch or the next reads
// them); the others share the conversions.
template <typename S>
__device__ __forceinline__ void conv_middle(const Inst& I, int parity, int blk, int nblk_all, bool retire_moves,
                                            bool integrate) {
    if (blk == nblk_all - 1) {
        forces_and_bodies(I, parity, true, retire_moves, integrate);
        return;
    }
    const int nblk = nblk_all - 1;
    StepCounters& C = I.ctl->cnt[parity];
    S* pop = (S*)pop_of(I, parity ^ 1);
    float* phi = phi_of(I, parity ^ 1);
    const int j = g_lane();
    // The new cells from gas and the excess shares are independent chains of
    // dependent loads: the first half of the workgroups takes the one, the
    // second half the other, so that they run side by side.
    const int half = max(1, nblk / 2);
    const bool gas_part = blk < half;
    const int pb = gas_part ? blk : blk - half, pn = gas_part ? half : nblk - half;
    const int g0 = pb * CG + (int)(threadIdx.x >> 5), ng = pn * CG;
    // new interface cells from gas, one group each (lane j: neighbour j)
    const int nng = gas_part ? list_len(&C.n_newg, I.list_cap) : 0;
    for (int k = g0; k < nng; k += ng) {
        const int g = I.newg[k];
        int gx, gy, gz;
        cell_coords(I, g, gx, gy, gz);
        const int nb = lane_nbr(I, gx, gy, gz);
        bool use = false;
        if (nb >= 0) {
            const uint8_t f = I.flags[nb];
            const int t = f & TYPE_MASK;
            use = (t == LIQ || t == IFC) && !(f & MARK_EMPTY);
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
    // new interface cells from liquid, one thread each: m = rho, phi = 1
    const int nnl = list_len(&C.n_newl, I.list_cap);
    for (int k = blk * CT + (int)threadIdx.x; k < nnl; k += nblk * CT) {
        const int id = I.newl[k];
        const float dr = drho_of<S>(I, pop, id);
        I.m_hi[id] = 1.f;
        I.m_lo[id] = dr;
        I.aux[id] = dr;
        phi[id] = 1.f;
    }
    // excess shares, one group per converted cell (lane i: neighbour x + c_i)
    const int nc = gas_part && nblk > 1 ? 0 : cand_len(C, I.list_cap);
    for (int k = g0; k < nc; k += ng) {
        const int id = I.cand[k];
        const uint8_t fl = I.flags[id];
        if (!(fl & (MARK_FILL | MARK_EMPTY))) continue;
        int x, y, z;
        cell_coords(I, id, x, y, z);
        const int nb = lane_nbr(I, x, y, z);
        const bool rcv = nb >= 0 && post_type(I, nb) == IFC;
        const int nr = __popc(g_ballot(rcv));
        if (nr == 0) {
            if (j == 0) {
                atomicAdd(&I.ctl->ledger, -(double)I.share[id]);
                I.share[id] = 0.f;
            }
            continue;
        }
        if (j == 0) I.share[id] = (float)((double)I.share[id] / nr);
        // the receiver notes this converted neighbour (its link opp(i)); the
        // first note puts it on the list
        const bool first = rcv && atomicOr(&I.cmask[nb], 1u << lane_opp(j)) == 0u;
        g_push(first, nb, I.recv, &C.n_recv, I.list_cap, &C.overflow);
    }
}

template <typename S>
__device__ __forceinline__ void conv_commit(const Inst& I, int parity, int blk, int nblk, unsigned step_tag) {
    StepCounters& C = I.ctl->cnt[parity];
    const int nc = cand_len(C, I.list_cap), ng = list_len(&C.n_newg, I.list_cap);
    const int nl = list_len(&C.n_newl, I.list_cap), nr = list_len(&C.n_recv, I.list_cap);
    float* phi = phi_of(I, parity ^ 1);
    const int t0 = blk * CT, step = nblk * CT;
    // converted and new cells, one thread each (the claim bits of the new
    // cells are the only bits set in the bitmap, and all are cleared here)
    const int items = nc + ng + nl;
    for (int k0 = t0; k0 < items; k0 += step) {
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
        } else if (k < items) {
            g = k < nc + ng;
            l = !g;
            const int id = g ? I.newg[k - nc] : I.newl[k - nc - ng];
            I.flags[id] = IFC;
            unclaim_word(I.claim, id);
            if (g) atomicMax(&I.ctl->ztop, id / (I.nx * I.ny));  // gas turned fluid
        }
        wave_count(f, &C.filled);
        wave_count(e, &C.emptied);
        wave_count(g, &C.newg);
        wave_count(l, &C.newl);
    }
    // receivers, one thread each: the note mask names the converted
    // neighbours, whose shares are added in link order; rho - 1 of every
    // receiver is in I.aux (left by the sweep for interface cells, by the
    // middle launch for new ones)
    for (int k = t0 + (int)threadIdx.x; k < nr; k += step) {
        const int id = I.recv[k];
        const uint32_t m = I.cmask[id];
        int x, y, z;
        cell_coords(I, id, x, y, z);
        float sh[Q];
#pragma unroll
        for (int q = 1; q < Q; ++q) {
            sh[q] = 0.f;
            if ((m >> q) & 1u) sh[q] = I.share[nbr_index(I, x, y, z, cx(q), cy(q), cz(q))];
        }
        float hi = I.m_hi[id], lo = I.m_lo[id];
        const float dr = I.aux[id];
#pragma unroll
        for (int q = 1; q < Q; ++q)
            if ((m >> q) & 1u) add_comp(hi, lo, sh[q]);
        I.m_hi[id] = hi;
        I.m_lo[id] = lo;
        phi[id] = (float)(((double)hi + (double)lo) / (1.0 + (double)dr));
        I.cmask[id] = 0u;
    }
    if (blk == 0) clear_other(I, parity, threadIdx.x, CT);
    // report the layer bound with the step's index (one 64-bit store to the
    // pinned host word; read in this launch, the bound may miss this launch's
    // own raises, which later steps' bounds allow for)
    if (blk == 0 && threadIdx.x == 0 && step_tag != NO_STEP_TAG && I.zpin) {
        const unsigned zt = (unsigned)__atomic_load_n(&I.ctl->ztop, __ATOMIC_RELAXED);
        *(volatile unsigned long long*)I.zpin = ((unsigned long long)step_tag << 32) | zt;
    }
}

}  // namespace

// one instance
template <typename S>
__global__ __launch_bounds__(CT) void k_conv_claim(Inst I, int parity, int bulk_layers) {
    conv_claim<S>(I, parity, blockIdx.x, gridDim.x, bulk_layers);
}
template <typename S>
__global__ __launch_bounds__(CT) void k_conv_middle(Inst I, int parity, int retire_moves, int integrate) {
    conv_middle<S>(I, parity, blockIdx.x, gridDim.x, retire_moves != 0, integrate != 0);
}
template <typename S>
__global__ __launch_bounds__(CT) void k_conv_commit(Inst I, int parity, unsigned step_tag) {
    conv_commit<S>(I, parity, blockIdx.x, gridDim.x, step_tag);
}

// a batch of at most 64 instances: blockIdx.y is the instance (bit y of the
// masks), blockIdx.x the workgroup of its grid (grids of other sizes: the
// extra workgroups return)
template <typename S>
__global__ __launch_bounds__(CT) void kb_conv_claim(const Inst* __restrict__ tab, int parity, const GroupLayers L) {
    const Inst I = tab[blockIdx.y];
    const int nb = conv_blocks(I);
    if ((int)blockIdx.x >= nb) return;
    conv_claim<S>(I, parity, blockIdx.x, nb, L.v[blockIdx.y]);
}
template <typename S>
__global__ __launch_bounds__(CT) void kb_conv_middle(const Inst* __restrict__ tab, int parity,
                                                     unsigned long long retire_mask, unsigned long long integrate_mask) {
    const int k = blockIdx.y;
    const Inst I = tab[k];
    const int nb = conv_blocks(I);
    if ((int)blockIdx.x >= nb) return;
    conv_middle<S>(I, parity, blockIdx.x, nb, (retire_mask >> k) & 1ull, (integrate_mask >> k) & 1ull);
}
template <typename S>
__global__ __launch_bounds__(CT) void kb_conv_commit(const Inst* __restrict__ tab, int parity, unsigned step_tag) {
    const Inst I = tab[blockIdx.y];
    const int nb = conv_blocks(I);
    if ((int)blockIdx.x >= nb) return;
    conv_commit<S>(I, parity, blockIdx.x, nb, step_tag);
}

// End of a step without conversions (phase-isolated calls).
__global__ __launch_bounds__(CT) void k_finish(Inst I, int parity, int reduce, int zero_other, int retire_moves) {
    forces_and_bodies(I, parity, reduce != 0, retire_moves != 0, false);
    if (zero_other) clear_other(I, parity, threadIdx.x, CT);
}

namespace {
template <typename S>
void convert_one(const Inst& I, int parity, int r, int n, hipStream_t s, unsigned step_tag, int bulk_layers) {
    const dim3 g(conv_blocks(I)), b(CT);
    hipLaunchKernelGGL(k_conv_claim<S>, g, b, 0, s, I, parity, bulk_layers);
    hipLaunchKernelGGL(k_conv_middle<S>, g, b, 0, s, I, parity, r, n);
    hipLaunchKernelGGL(k_conv_commit<S>, g, b, 0, s, I, parity, step_tag);
}
template <typename S>
void convert_batch(const Inst* tab, int n, int blocks, int parity, unsigned long long rm, unsigned long long im,
                   hipStream_t s, unsigned step_tag, const GroupLayers& L) {
    const dim3 g(blocks, n), b(CT);
    hipLaunchKernelGGL(kb_conv_claim<S>, g, b, 0, s, tab, parity, L);
    hipLaunchKernelGGL(kb_conv_middle<S>, g, b, 0, s, tab, parity, rm, im);
    hipLaunchKernelGGL(kb_conv_commit<S>, g, b, 0, s, tab, parity, step_tag);
}
}  // namespace

void launch_convert_batch(const Inst* tab, int n, int blocks, int storage, int parity, unsigned long long retire_mask,
                          unsigned long long integrate_mask, hipStream_t s, unsigned step_tag, const int* bulk_layers) {
    GroupLayers L{};
    for (int k = 0; k < n && k < 64; ++k) L.v[k] = bulk_layers ? bulk_layers[k] : 0;
    switch (storage) {
    case LBM_FP16_DEV: convert_batch<__half>(tab, n, blocks, parity, retire_mask, integrate_mask, s, step_tag, L); break;
    case LBM_BF16_DEV:
        convert_batch<__hip_bfloat16>(tab, n, blocks, parity, retire_mask, integrate_mask, s, step_tag, L);
        break;
    default: convert_batch<float>(tab, n, blocks, parity, retire_mask, integrate_mask, s, step_tag, L); break;
    }
}

void launch_convert(const Inst& I, int parity, bool retire_moves, bool integrate, hipStream_t s, unsigned step_tag,
                    int bulk_layers) {
    const int r = (int)retire_moves, n = (int)integrate;
    switch (I.storage) {
    case LBM_FP16_DEV: convert_one<__half>(I, parity, r, n, s, step_tag, bulk_layers); break;
    case LBM_BF16_DEV: convert_one<__hip_bfloat16>(I, parity, r, n, s, step_tag, bulk_layers); break;
    default: convert_one<float>(I, parity, r, n, s, step_tag, bulk_layers); break;
    }
}

void launch_finish(const Inst& I, int parity, bool reduce, bool zero_other, bool retire_moves, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(CT), 0, s, I, parity, (int)reduce, (int)zero_other,
                       (int)retire_moves);
}

}  // namespace lgs
