// k_convert.hip -- free-surface cell conversions (Sec. 2.2) on the state at
// t+1, driven by the candidate list the sweep built, plus the end of a step.
//
// One workgroup of 1024 threads runs the phases one after the other,
// separated by workgroup barriers (candidate lists are short: a few to a few
// thousand cells per step).  Each phase is a function of the state before
// it, so the result does not depend on the order of the (atomically
// appended) lists:
//   forces  the boundary sweep's per-wavefront momentum-exchange records are
//           summed per body in slot order (fixed-order FP64 reduction)
//   claim   per candidate: a filled cell (phi >= 1+eps) records its excess
//           m - rho and claims its gas neighbours as new interface cells,
//           initialising each with f = f_eq(mean rho, mean u) over its
//           neighbours that are liquid or interface and not emptying, m = 0;
//           an emptied cell (phi <= -eps) touching a filled one stays
//           interface (filling wins), otherwise it records its excess m and
//           claims its liquid neighbours as new interface cells (m = rho).
//           Claims go through a bitmap, so every new cell is initialised once.
//   share   per converted cell: count the neighbours that are interface after
//           the conversion (a function of the flags, marks and claims), divide
//           the excess among them and list them as receivers; with none the
//           excess leaves the fluid (ledger).
//   commit  receivers add the shares of their converted neighbours in link
//           order i = 1..18 and recompute phi = m / rho; converted and new
//           cells take their new types.  Converted cells keep their mark until
//           the next sweep clears it.
//   finish  clear the other parity's counters, retire body moves.
#include <cstddef>

#include "lgs_internal.h"

namespace lgs {

namespace {

constexpr int CONV_THREADS = 512;

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
__device__ __forceinline__ void unclaim(uint32_t* bits, int id) { atomicAnd(bits + (id >> 5), ~(1u << (id & 31))); }

__device__ __forceinline__ void push(int* list, int* cnt, int cap, int* overflow, int id) {
    const int p = atomicAdd(cnt, 1);
    if (p < cap) list[p] = id;
    else atomicOr(overflow, 1);
}

template <typename S>
__device__ __forceinline__ void moments(const Inst& I, const S* pop, int id, float& drho, float u[3]) {
    const size_t N = (size_t)I.N;
    float dr = 0.f, j0 = 0.f, j1 = 0.f, j2 = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float v = Store<S>::ld(pop, (size_t)i * N + id, I.inv_scale);
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
    const size_t N = (size_t)I.N;
    float dr = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) dr += Store<S>::ld(pop, (size_t)i * N + id, I.inv_scale);
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

template <typename S>
__device__ __forceinline__ void phase_claim(const Inst& I, int parity) {
    StepCounters& C = I.ctl->cnt[parity];
    const int n = min(load_count(&C.n_cand), I.list_cap);
    S* pop = (S*)I.pop[parity ^ 1];
    const size_t N = (size_t)I.N;
    float* phi = I.phi[parity ^ 1];
    BLOCK_LOOP(k, n) {
        const int id = I.cand[k];
        const uint8_t fl = I.flags[id];
        int x, y, z;
        cell_coords(I, id, x, y, z);
        if (fl & MARK_FILL) {
            const float dr = drho_of<S>(I, pop, id);
            I.share[id] = (float)(((double)I.m_hi[id] - 1.0) + ((double)I.m_lo[id] - (double)dr));
            for (int i = 1; i < Q; ++i) {
                const int g = nbr_index(I, x, y, z, cx(i), cy(i), cz(i));
                if (g < 0 || (I.flags[g] & TYPE_MASK) != GAS || !claim(I.claim, g)) continue;
                push(I.newg, &C.n_newg, I.list_cap, &C.overflow, g);
                // new interface cell from gas: equilibrium of its liquid /
                // interface neighbours that are not emptying
                int gx, gy, gz;
                cell_coords(I, g, gx, gy, gz);
                float rs = 0.f, us0 = 0.f, us1 = 0.f, us2 = 0.f;
                int ns = 0;
                for (int j = 1; j < Q; ++j) {
                    const int nb = nbr_index(I, gx, gy, gz, cx(j), cy(j), cz(j));
                    if (nb < 0) continue;
                    const uint8_t f = I.flags[nb];
                    const int t = f & TYPE_MASK;
                    if ((t != LIQ && t != IFC) || empties(I, nb, f)) continue;
                    float d, u[3];
                    moments<S>(I, pop, nb, d, u);
                    rs += d;
                    us0 += u[0];
                    us1 += u[1];
                    us2 += u[2];
                    ++ns;
                }
                const float inv = 1.f / (float)max(ns, 1);
                const float drb = ns > 0 ? rs * inv : I.rho_g - 1.f, rb = 1.f + drb;
                const float u0 = us0 * inv, u1 = us1 * inv, u2 = us2 * inv;
                const float uu = u0 * u0 + u1 * u1 + u2 * u2;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const float cu = cx(q) * u0 + cy(q) * u1 + cz(q) * u2;
                    const float deq = wgt(q) * (drb + rb * (3.f * cu + 4.5f * cu * cu - 1.5f * uu));
                    Store<S>::st(pop, (size_t)q * N + g, deq, I.scale);
                }
                I.m_hi[g] = 0.f;
                I.m_lo[g] = 0.f;
                phi[g] = 0.f;
            }
        } else if (fl & MARK_EMPTY) {
            if (has_fill_neighbour(I, x, y, z)) {
                I.flags[id] = fl & (uint8_t)~MARK_EMPTY;  // filling wins: stays interface
                continue;
            }
            I.share[id] = (float)((double)I.m_hi[id] + (double)I.m_lo[id]);
            for (int i = 1; i < Q; ++i) {
                const int l = nbr_index(I, x, y, z, cx(i), cy(i), cz(i));
                if (l < 0 || (I.flags[l] & TYPE_MASK) != LIQ || !claim(I.claim, l)) continue;
                push(I.newl, &C.n_newl, I.list_cap, &C.overflow, l);
                I.m_hi[l] = 1.f;
                I.m_lo[l] = drho_of<S>(I, pop, l);
                phi[l] = 1.f;
            }
        }
    }
}

__device__ __forceinline__ void phase_share(const Inst& I, int parity) {
    StepCounters& C = I.ctl->cnt[parity];
    const int nc = min(load_count(&C.n_cand), I.list_cap);
    BLOCK_LOOP(k, nc) {
        const int id = I.cand[k];
        const uint8_t fl = I.flags[id];
        if (!(fl & (MARK_FILL | MARK_EMPTY))) continue;
        int x, y, z;
        cell_coords(I, id, x, y, z);
        int nr = 0;
        for (int i = 1; i < Q; ++i) {
            const int nb = nbr_index(I, x, y, z, cx(i), cy(i), cz(i));
            if (nb >= 0 && post_type(I, nb) == IFC) ++nr;
        }
        if (nr == 0) {
            atomicAdd(&I.ctl->ledger, -(double)I.share[id]);
            I.share[id] = 0.f;
            continue;
        }
        I.share[id] = (float)((double)I.share[id] / nr);
        for (int i = 1; i < Q; ++i) {
            const int nb = nbr_index(I, x, y, z, cx(i), cy(i), cz(i));
            if (nb >= 0 && post_type(I, nb) == IFC && claim(I.claim2, nb))
                push(I.recv, &C.n_recv, I.list_cap, &C.overflow, nb);
        }
    }
}

template <typename S>
__device__ __forceinline__ void phase_commit(const Inst& I, int parity) {
    StepCounters& C = I.ctl->cnt[parity];
    const int nc = min(load_count(&C.n_cand), I.list_cap), ng = min(load_count(&C.n_newg), I.list_cap);
    const int nl = min(load_count(&C.n_newl), I.list_cap), nr = min(load_count(&C.n_recv), I.list_cap);
    S* pop = (S*)I.pop[parity ^ 1];
    float* phi = I.phi[parity ^ 1];
    BLOCK_LOOP(k, nc + ng + nl + nr) {
        if (k < nc) {
            const int id = I.cand[k];
            const uint8_t fl = I.flags[id];
            if (fl & MARK_FILL) {
                I.flags[id] = LIQ | MARK_FILL;
                I.m_hi[id] = 0.f;
                I.m_lo[id] = 0.f;
                phi[id] = 1.f;
                atomicAdd(&C.filled, 1);
            } else if (fl & MARK_EMPTY) {
                I.flags[id] = GAS | MARK_EMPTY;
                I.m_hi[id] = 0.f;
                I.m_lo[id] = 0.f;
                phi[id] = 0.f;
                atomicAdd(&C.emptied, 1);
            }
        } else if (k < nc + ng + nl) {
            const bool g = k < nc + ng;
            const int id = g ? I.newg[k - nc] : I.newl[k - nc - ng];
            I.flags[id] = IFC;
            unclaim(I.claim, id);
            atomicAdd(g ? &C.newg : &C.newl, 1);
        } else {
            const int id = I.recv[k - nc - ng - nl];
            int x, y, z;
            cell_coords(I, id, x, y, z);
            float hi = I.m_hi[id], lo = I.m_lo[id];
            for (int i = 1; i < Q; ++i) {
                const int nb = nbr_index(I, x, y, z, cx(i), cy(i), cz(i));
                if (nb >= 0 && (I.flags[nb] & (MARK_FILL | MARK_EMPTY))) add_comp(hi, lo, I.share[nb]);
            }
            I.m_hi[id] = hi;
            I.m_lo[id] = lo;
            const float dr = drho_of<S>(I, pop, id);
            phi[id] = (float)(((double)hi + (double)lo) / (1.0 + (double)dr));
            unclaim(I.claim2, id);
        }
    }
}

// fixed-order FP64 sum of the boundary sweep's force records, per body
__device__ __forceinline__ void phase_forces(const Inst& I, int parity) {
    __shared__ double red[6][CONV_THREADS];
    StepCounters& C = I.ctl->cnt[parity];
    const int nrec = boundary_blocks(I) * 4;  // one record per wavefront of the boundary grid
    for (int b = 0; b < I.nbodies; ++b) {
        double v[6] = {0, 0, 0, 0, 0, 0};
        for (int k = threadIdx.x; k < nrec; k += blockDim.x) {
            const ForceRec& r = I.frec[k];
            if (r.body != b) continue;
#pragma unroll
            for (int q = 0; q < 6; ++q) v[q] += r.v[q];
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) red[q][threadIdx.x] = v[q];
        __syncthreads();
        for (int o = blockDim.x >> 1; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o)
#pragma unroll
                for (int q = 0; q < 6; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x < 6) C.acc[b][threadIdx.x] += red[threadIdx.x][0];
        __syncthreads();
    }
}

// clear the other parity's counters and / or retire body moves
__device__ __forceinline__ void phase_finish(const Inst& I, int parity, bool zero_other, bool retire_moves) {
    if (zero_other) {
        StepCounters& O = I.ctl->cnt[parity ^ 1];
        int* ci = (int*)&O;
        const int nint = (int)(offsetof(StepCounters, acc) / sizeof(int));
        for (int q = threadIdx.x; q < nint; q += blockDim.x) ci[q] = 0;
        for (int q = threadIdx.x; q < MAXB * 6; q += blockDim.x) (&O.acc[0][0])[q] = 0.0;
    }
    if (retire_moves && (int)threadIdx.x < I.nbodies) {
        DevBody& b = I.bodies[threadIdx.x];
        if (b.moved) {
            b.moved = 0;
            b.prev_pos[0] = b.pos[0];
            b.prev_pos[1] = b.pos[1];
            b.prev_pos[2] = b.pos[2];
        }
    }
}

template <typename S>
__global__ __launch_bounds__(CONV_THREADS) void k_convert(Inst I, int parity, int retire_moves,
                                                          unsigned long long seq) {
    phase_forces(I, parity);
    if (I.hout && seq) {
        // hand the forces to the host early: the conversions do not change them
        StepCounters& C = I.ctl->cnt[parity];
        for (int q = threadIdx.x; q < I.nbodies * 6; q += blockDim.x) I.hout->acc[q / 6][q % 6] = C.acc[q / 6][q % 6];
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence_system();
            I.hout->seq = seq;
        }
    }
    phase_claim<S>(I, parity);
    __syncthreads();
    phase_share(I, parity);
    __syncthreads();
    phase_commit<S>(I, parity);
    __syncthreads();
    phase_finish(I, parity, true, retire_moves != 0);
}

// End of a step without conversions (phase-isolated calls).
__global__ __launch_bounds__(CONV_THREADS) void k_finish(Inst I, int parity, int reduce, int zero_other,
                                                         int retire_moves) {
    if (reduce) phase_forces(I, parity);
    phase_finish(I, parity, zero_other != 0, retire_moves != 0);
}

void launch_convert(const Inst& I, int parity, bool retire_moves, unsigned long long seq, hipStream_t s) {
    const dim3 g(1), b(CONV_THREADS);
    const int r = (int)retire_moves;
    switch (I.storage) {
    case LBM_FP16_DEV: hipLaunchKernelGGL(k_convert<__half>, g, b, 0, s, I, parity, r, seq); break;
    case LBM_BF16_DEV: hipLaunchKernelGGL(k_convert<__hip_bfloat16>, g, b, 0, s, I, parity, r, seq); break;
    default: hipLaunchKernelGGL(k_convert<float>, g, b, 0, s, I, parity, r, seq); break;
    }
}

void launch_finish(const Inst& I, int parity, bool reduce, bool zero_other, bool retire_moves, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(CONV_THREADS), 0, s, I, parity, (int)reduce, (int)zero_other,
                       (int)retire_moves);
}

}  // namespace lgs
