// k_sweep.hip -- the fused per-cell time step of liquid and interface cells.
//
// Pull form of Sec. 2.1 Eq. stream: cell x takes f'_i from s = x - c_i.
//   s liquid/interface : f'_i = f_i(s)
//   s wall / obstacle  : moving-wall bounce-back, Eq. noslip,
//                        f'_i = f_ibar(x) + 6 w_i rho_x c_i.u_w
//   s gas              : Eq. reconstruct with this cell's own outgoing
//                        f_ibar(x): f'_i = f_eq,i + f_eq,ibar - f_ibar(x) at
//                        (rho_G, u_x)
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
//                     are appended to a boundary list (wavefront ballot +
//                     prefix sum).  Gas and obstacle cells cost a flag byte.
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

#include "lgs_internal.h"

namespace lgs {

namespace {

constexpr double NORMAL_TOL = 1e-3;
constexpr int BND_BLOCKS = 1024;

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

// BGK collision with the force term on pulled deviations d[], written to dst
template <typename S>
__device__ __forceinline__ void collide_store(const Inst& I, float (&d)[Q], S* __restrict__ dst, size_t N, int id) {
    float drho = 0.f, j0 = 0.f, j1 = 0.f, j2 = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        drho += d[i];
        j0 += cx(i) * d[i];
        j1 += cy(i) * d[i];
        j2 += cz(i) * d[i];
    }
    const float rho = 1.f + drho;
    const float irho = 1.f / rho;
    const float u0 = j0 * irho, u1 = j1 * irho, u2 = j2 * irho;
    const float uu = u0 * u0 + u1 * u1 + u2 * u2;
    const float ua = u0 * I.ax + u1 * I.ay + u2 * I.az;
    const float om = I.omega;
    if (!(rho > 0.f && rho < 1e6f)) atomicOr(&I.ctl->nonfinite, 1);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float cu = cx(i) * u0 + cy(i) * u1 + cz(i) * u2;
        const float ca = cx(i) * I.ax + cy(i) * I.ay + cz(i) * I.az;
        const float w = wgt(i);
        const float deq = w * (drho + rho * (3.f * cu + 4.5f * cu * cu - 1.5f * uu));
        const float F = w * rho * (3.f * (ca - ua) + 9.f * cu * ca);
        const float dn = d[i] + om * (deq - d[i]) + F;
        Store<S>::store(dst, (size_t)i * N + id, dn, I.scale);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// bulk sweep
// ---------------------------------------------------------------------------
template <typename S, int TX>
__global__ __launch_bounds__(256) void k_sweep_bulk(Inst I, int parity, int tiles_x, int tiles_y) {
    constexpr int TY = 256 / TX;
    // XCD-aware tile order: workgroup b runs on XCD b % 8; give each XCD a
    // contiguous range of tiles so that halo rows are shared inside one L2.
    const int nb = gridDim.x, b = blockIdx.x;
    const int q8 = nb >> 3, r8 = nb & 7, xcd = b & 7, kk = b >> 3;
    const int t = (xcd < r8 ? xcd * (q8 + 1) : r8 * (q8 + 1) + (xcd - r8) * q8) + kk;
    const int tx = t % tiles_x;
    const int rest = t / tiles_x;
    const int ty = rest % tiles_y;
    const int z = rest / tiles_y;
    const int x = tx * TX + (threadIdx.x % TX);
    const int y = ty * TY + (threadIdx.x / TX);

    const size_t N = (size_t)I.N;
    const S* __restrict__ src = (const S*)I.pop[parity];
    S* __restrict__ dst = (S*)I.pop[parity ^ 1];
    StepCounters& C = I.ctl->cnt[parity];

    const bool inb = (x < I.nx) && (y < I.ny);
    const int id = inb ? x + I.nx * (y + I.ny * z) : 0;
    const uint8_t fl = inb ? I.flags[id] : (uint8_t)GAS;
    const int type = fl & TYPE_MASK;
    // drop the marks a previous conversion phase left on this cell
    if (inb && (fl & ~KEEP_MASK)) I.flags[id] = fl & KEEP_MASK;

    bool defer = (type == IFC);
    if (type == LIQ) {
        const bool px = I.periodic & 1, py = I.periodic & 2, pz = I.periodic & 4;
        const int xm = step_axis(x, -1, I.nx, px), xp = step_axis(x, 1, I.nx, px);
        const int ym = step_axis(y, -1, I.ny, py), yp = step_axis(y, 1, I.ny, py);
        const int zm = step_axis(z, -1, I.nz, pz), zp = step_axis(z, 1, I.nz, pz);
        float d[Q];
        bool bad = false;
        d[0] = Store<S>::load(src, id, I.inv_scale);
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const int X = cx(i) == 1 ? xm : (cx(i) == -1 ? xp : x);
            const int Y = cy(i) == 1 ? ym : (cy(i) == -1 ? yp : y);
            const int Z = cz(i) == 1 ? zm : (cz(i) == -1 ? zp : z);
            const bool ok = (X | Y | Z) >= 0;
            const int s = X + I.nx * (Y + I.ny * Z);
            // static wall: halfway bounce-back takes this cell's own f_ibar
            const size_t a = ok ? (size_t)i * N + s : (size_t)opp(i) * N + id;
            d[i] = Store<S>::load(src, a, I.inv_scale);
            if (ok) {
                const int st = I.flags[s] & TYPE_MASK;
                bad |= (st == GAS) || (st == OBS);
            }
        }
        if (bad) defer = true;
        else collide_store<S>(I, d, dst, N, id);
    }
    wave_append(defer, id, I.bnd, &C.n_bnd, I.list_cap, &C.overflow);
}

// ---------------------------------------------------------------------------
// boundary sweep: interface cells, liquid cells next to gas or a body
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(256) void k_sweep_boundary(Inst I, int parity) {
    const size_t N = (size_t)I.N;
    const S* __restrict__ src = (const S*)I.pop[parity];
    S* __restrict__ dst = (S*)I.pop[parity ^ 1];
    const float isc = I.inv_scale;
    StepCounters& C = I.ctl->cnt[parity];
    const int nlist = min(C.n_bnd, I.list_cap);
    const bool px = I.periodic & 1, py = I.periodic & 2, pz = I.periodic & 4;

    for (int base = blockIdx.x * blockDim.x; base < nlist; base += gridDim.x * blockDim.x) {
        const int k = base + threadIdx.x;
        const bool active = k < nlist;
        const int id = active ? I.bnd[k] : 0;
        float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        int accb = -1;
        uint8_t mark = 0;
        if (active) {
            int x, y, z;
            cell_coords(I, id, x, y, z);
            const uint8_t fl = I.flags[id];
            const int type = fl & TYPE_MASK;
            const int xm = step_axis(x, -1, I.nx, px), xp = step_axis(x, 1, I.nx, px);
            const int ym = step_axis(y, -1, I.ny, py), yp = step_axis(y, 1, I.ny, py);
            const int zm = step_axis(z, -1, I.nz, pz), zp = step_axis(z, 1, I.nz, pz);
            int sidx[Q];
            uint8_t sfl[Q];
            float d[Q];   // pulled deviations (raw, then replaced where a rule applies)
            float dx[Q];  // this cell's own f(x, t)
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int X = cx(i) == 1 ? xm : (cx(i) == -1 ? xp : x);
                const int Y = cy(i) == 1 ? ym : (cy(i) == -1 ? yp : y);
                const int Z = cz(i) == 1 ? zm : (cz(i) == -1 ? zp : z);
                const bool ok = (X | Y | Z) >= 0;
                sidx[i] = ok ? X + I.nx * (Y + I.ny * Z) : -1;
                sfl[i] = ok ? I.flags[sidx[i]] : (uint8_t)OBS;
                d[i] = Store<S>::ld(src, (size_t)i * N + (ok ? sidx[i] : id), isc);
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) dx[i] = Store<S>::ld(src, (size_t)i * N + id, isc);
            d[0] = dx[0];
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
            const float phix = type == IFC ? I.phi[parity][id] : 1.f;

            // interface normal n = -grad(phi) on the 6 axis neighbours; the
            // sign test is made in FP64 on the stored fill levels
            double n0 = 0.0, n1 = 0.0, n2 = 0.0, nthr = 0.0;
            if (type == IFC && I.recon_mode != LBM_RECON_GAS_ONLY) {
                auto fillv = [&](int sid, uint8_t f) -> double {
                    const int st = f & TYPE_MASK;
                    if (sid < 0 || st == OBS) return (double)phix;
                    if (st == LIQ) return 1.0;
                    if (st == GAS) return 0.0;
                    return (double)I.phi[parity][sid];
                };
                // the source of link E (c = +x) is x-1, of W (c = -x) is x+1
                n0 = 0.5 * (fillv(sidx[2], sfl[2]) - fillv(sidx[1], sfl[1]));
                n1 = 0.5 * (fillv(sidx[3], sfl[3]) - fillv(sidx[4], sfl[4]));
                n2 = 0.5 * (fillv(sidx[5], sfl[5]) - fillv(sidx[6], sfl[6]));
                nthr = NORMAL_TOL * ((fabs(n0) + fabs(n1)) + fabs(n2));
            }

            // mass exchange (interface cells), on the raw pulled values:
            // neighbour y = x + c_i is the source of link ibar; f_ibar(y) = d[ibar]
            float dm = 0.f;
            if (type == IFC) {
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    const int ib = opp(i);
                    const int st = sfl[ib] & TYPE_MASK;
                    if (sidx[ib] < 0) continue;
                    const float ex = d[ib] - dx[i];
                    if (st == LIQ) dm += ex;
                    else if (st == IFC) dm += 0.5f * (phix + I.phi[parity][sidx[ib]]) * ex;
                }
            }

            const float xc0 = x + 0.5f, xc1 = y + 0.5f, xc2 = z + 0.5f;
            const float uu = ux0 * ux0 + ux1 * ux1 + ux2 * ux2;
            const float phat = type == LIQ ? 1.f : phix;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int ib = opp(i);
                const int st = sfl[i] & TYPE_MASK;
                if (sidx[i] < 0 || st == OBS) {
                    float cu = 0.f;
                    int bk = -1;
                    float r0 = 0.f, r1 = 0.f, r2 = 0.f;
                    if (sidx[i] >= 0) {
                        bk = (sfl[i] >> 2) & 15;
                        const DevBody& B = I.bodies[bk];
                        // body velocity at the link midpoint x_c - c_i/2
                        const float p0 = (float)wrap_rel(xc0 - 0.5f * cx(i) - B.pos[0], I.nx, px);
                        const float p1 = (float)wrap_rel(xc1 - 0.5f * cy(i) - B.pos[1], I.ny, py);
                        const float p2 = (float)wrap_rel(xc2 - 0.5f * cz(i) - B.pos[2], I.nz, pz);
                        const float w0 = (float)B.omega[0], w1 = (float)B.omega[1], w2 = (float)B.omega[2];
                        const float u0 = (float)B.vel[0] + (w1 * p2 - w2 * p1);
                        const float u1 = (float)B.vel[1] + (w2 * p0 - w0 * p2);
                        const float u2 = (float)B.vel[2] + (w0 * p1 - w1 * p0);
                        cu = cx(i) * u0 + cy(i) * u1 + cz(i) * u2;
                        r0 = (float)wrap_rel(xc0 - B.pos[0], I.nx, px);
                        r1 = (float)wrap_rel(xc1 - B.pos[1], I.ny, py);
                        r2 = (float)wrap_rel(xc2 - B.pos[2], I.nz, pz);
                    }
                    const float mw = 6.f * wgt(i) * rhox * cu;
                    d[i] = dx[ib] + mw;
                    if (bk >= 0) {
                        // momentum the fluid gains on this link (deviation form)
                        const float amp = 2.f * phat * (dx[ib] + wgt(i) * (1.f - I.rho_g) + 0.5f * mw);
                        const float j0 = amp * cx(i), j1 = amp * cy(i), j2 = amp * cz(i);
                        const float t0 = r1 * j2 - r2 * j1, t1 = r2 * j0 - r0 * j2, t2 = r0 * j1 - r1 * j0;
                        if (accb < 0) accb = bk;
                        if (bk == accb) {
                            acc[0] -= j0; acc[1] -= j1; acc[2] -= j2;
                            acc[3] -= t0; acc[4] -= t1; acc[5] -= t2;
                        } else {
                            double* a = C.acc[bk];
                            atomicAdd(a + 0, -(double)j0); atomicAdd(a + 1, -(double)j1); atomicAdd(a + 2, -(double)j2);
                            atomicAdd(a + 3, -(double)t0); atomicAdd(a + 4, -(double)t1); atomicAdd(a + 5, -(double)t2);
                        }
                    }
                    continue;
                }
                bool recon = (st == GAS);
                if (!recon && type == IFC && I.recon_mode != LBM_RECON_GAS_ONLY) {
                    const double cn = cx(i) * n0 + cy(i) * n1 + cz(i) * n2;
                    recon = I.recon_mode == LBM_RECON_GAS_SIDE ? (cn < -nthr) : (cn <= nthr);
                }
                if (recon) {
                    const float cu = cx(i) * ux0 + cy(i) * ux1 + cz(i) * ux2;
                    // (f_eq,i + f_eq,ibar)(rho_G, u_x) - 2 w_i, minus d_ibar(x)
                    d[i] = 2.f * wgt(i) * (I.rho_g * (1.f + 4.5f * cu * cu - 1.5f * uu) - 1.f) - dx[ib];
                }
            }

            if (type == IFC) {
                // fill level from the density after streaming
                float dr = 0.f;
#pragma unroll
                for (int i = 0; i < Q; ++i) dr += d[i];
                float hi = I.m_hi[id], lo = I.m_lo[id];
                two_sum_add(hi, lo, dm);
                I.m_hi[id] = hi;
                I.m_lo[id] = lo;
                const double mm = (double)hi + (double)lo;
                const float ph = (float)(mm / (1.0 + (double)dr));
                I.phi[parity ^ 1][id] = ph;
                const double phd = (double)ph;
                if (phd >= 1.0 + I.eps) mark = MARK_FILL;
                else if (phd <= -I.eps) mark = MARK_EMPTY;
                if (mark) I.flags[id] = (fl & KEEP_MASK) | mark;
            }
            collide_store<S>(I, d, dst, N, id);
        }

        // candidates for the conversion phase
        wave_append(mark != 0, id, I.cand, &C.n_cand, I.list_cap, &C.overflow);

        // momentum exchange: wavefront reduction in FP64, one atomic per body
        const bool has = accb >= 0;
        unsigned long long m = __ballot(has);
        while (m) {
            const int leader = __ffsll((long long)m) - 1;
            const int bk = __shfl(accb, leader);
            const bool mine = has && accb == bk;
            double v[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) v[q] = wave_sum(mine ? (double)acc[q] : 0.0);
            if (lane_id() == leader) {
#pragma unroll
                for (int q = 0; q < 6; ++q) atomicAdd(&C.acc[bk][q], v[q]);
            }
            m &= ~__ballot(mine);
        }
    }
}

template <typename S, int TX>
static void launch_bulk_t(const Inst& I, int parity, hipStream_t s) {
    constexpr int TY = 256 / TX;
    const int tiles_x = (I.nx + TX - 1) / TX;
    const int tiles_y = (I.ny + TY - 1) / TY;
    const int nblk = tiles_x * tiles_y * I.nz;
    hipLaunchKernelGGL((k_sweep_bulk<S, TX>), dim3(nblk), dim3(256), 0, s, I, parity, tiles_x, tiles_y);
}

void launch_sweep_bulk(const Inst& I, int parity, hipStream_t s) {
    const bool wide = I.nx >= 64;
    switch (I.storage) {
    case LBM_FP16_DEV:
        if (wide) launch_bulk_t<__half, 64>(I, parity, s);
        else launch_bulk_t<__half, 32>(I, parity, s);
        break;
    case LBM_BF16_DEV:
        if (wide) launch_bulk_t<__hip_bfloat16, 64>(I, parity, s);
        else launch_bulk_t<__hip_bfloat16, 32>(I, parity, s);
        break;
    default:
        if (wide) launch_bulk_t<float, 64>(I, parity, s);
        else launch_bulk_t<float, 32>(I, parity, s);
        break;
    }
}

void launch_sweep_boundary(const Inst& I, int parity, hipStream_t s) {
    const dim3 g(std::min(BND_BLOCKS, (I.N + 255) / 256)), b(256);
    switch (I.storage) {
    case LBM_FP16_DEV: hipLaunchKernelGGL(k_sweep_boundary<__half>, g, b, 0, s, I, parity); break;
    case LBM_BF16_DEV: hipLaunchKernelGGL(k_sweep_boundary<__hip_bfloat16>, g, b, 0, s, I, parity); break;
    default: hipLaunchKernelGGL(k_sweep_boundary<float>, g, b, 0, s, I, parity); break;
    }
}

// Candidate scan without a sweep (conversion phase on injected fields).
__global__ __launch_bounds__(256) void k_mark(Inst I, int parity) {
    StepCounters& C = I.ctl->cnt[parity];
    const int id = blockIdx.x * 256 + threadIdx.x;
    bool cand = false;
    if (id < I.N) {
        const uint8_t fl = I.flags[id];
        uint8_t mark = 0;
        if ((fl & TYPE_MASK) == IFC) {
            const double ph = (double)I.phi[parity ^ 1][id];
            if (ph >= 1.0 + I.eps) mark = MARK_FILL;
            else if (ph <= -I.eps) mark = MARK_EMPTY;
        }
        cand = mark != 0;
        const uint8_t nf = (fl & KEEP_MASK) | mark;
        if (nf != fl) I.flags[id] = nf;
    }
    wave_append(cand, id, I.cand, &C.n_cand, I.list_cap, &C.overflow);
}

void launch_mark(const Inst& I, int parity, hipStream_t s) {
    hipLaunchKernelGGL(k_mark, dim3((I.N + 255) / 256), dim3(256), 0, s, I, parity);
}

}  // namespace lgs
