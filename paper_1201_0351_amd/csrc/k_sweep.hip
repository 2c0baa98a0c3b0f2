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

// The nine pairs (i, ibar) of opposite D3Q19 links, primary member first.
__device__ constexpr int PAIR_P[9] = {2, 3, 5, 8, 9, 10, 12, 14, 16};

// BGK collision with the force term on pulled deviations d[], written to dst.
// Evaluated per pair of opposite links: the equilibrium and the force term
// split into a part even in c_i (shared) and a part odd in c_i (sign flips).
template <typename S>
__device__ __forceinline__ void collide_store(const Inst& I, float (&d)[Q], S* __restrict__ dst, size_t N, int id) {
    float drho = d[0], j0 = 0.f, j1 = 0.f, j2 = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int p = PAIR_P[k], q = opp(p);
        drho += d[p] + d[q];
        const float od = d[p] - d[q];
        j0 += cx(p) * od;
        j1 += cy(p) * od;
        j2 += cz(p) * od;
    }
    const float rho = 1.f + drho;
    const float irho = 1.f / rho;
    const float u0 = j0 * irho, u1 = j1 * irho, u2 = j2 * irho;
    const float uu15 = 1.5f * (u0 * u0 + u1 * u1 + u2 * u2);
    const float ua3 = 3.f * (u0 * I.ax + u1 * I.ay + u2 * I.az);
    const float om = I.omega;
    if (!(rho > 0.f && rho < 1e6f)) atomicOr(&I.ctl->nonfinite, 1);
    {
        const float w = wgt(0);
        const float deq = w * (drho - rho * uu15);
        const float F = -w * rho * ua3;
        Store<S>::store(dst, id, d[0] + om * (deq - d[0]) + F, I.scale);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int p = PAIR_P[k], q = opp(p);
        const float w = wgt(p);
        const float cu = cx(p) * u0 + cy(p) * u1 + cz(p) * u2;
        const float ca = cx(p) * I.ax + cy(p) * I.ay + cz(p) * I.az;
        const float wr = w * rho;
        const float even = w * drho + wr * (4.5f * cu * cu - uu15);
        const float odd = 3.f * wr * cu;
        const float Fe = wr * (9.f * cu * ca - ua3);
        const float Fo = 3.f * wr * ca;
        const float dp = d[p] + om * (even + odd - d[p]) + (Fe + Fo);
        const float dq = d[q] + om * (even - odd - d[q]) + (Fe - Fo);
        Store<S>::store(dst, (size_t)p * N + id, dp, I.scale);
        Store<S>::store(dst, (size_t)q * N + id, dq, I.scale);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// bulk sweep
// ---------------------------------------------------------------------------
template <typename S, int TX>
__global__ __launch_bounds__(256) void k_sweep_bulk(Inst I, int parity, int tiles_x, int tiles_y) {
    constexpr int TY = 256 / TX;
    // XCD-aware tile order: workgroup b runs on XCD b % 8.  Whole z-layers
    // (chunks of tiles_x * tiles_y tiles) go round-robin to the XCDs, so a
    // layer's y-halo rows and flags stay in one L2 while liquid and gas layers
    // spread evenly over all eight XCDs.
    const int nb = gridDim.x, b = blockIdx.x;
    const int CH = tiles_x * tiles_y;
    const int full = nb / (8 * CH) * (8 * CH);
    int t = b;
    if (b < full) {
        const int xcd = b & 7, kk = b >> 3;
        t = ((kk / CH) * 8 + xcd) * CH + kk % CH;
    }
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
        // all 37 loads are issued without branches; per-link array bases are
        // wavefront-uniform and the per-cell offset is 32-bit
        float d[Q];
        uint8_t sf[Q];
        d[0] = Store<S>::load(src, id, I.inv_scale);
        const bool interior = x > 0 && x < I.nx - 1 && y > 0 && y < I.ny - 1 && z > 0 && z < I.nz - 1;
        if (interior) {
            const int sxy = I.nx, sz = I.nx * I.ny;
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int s = id - (cx(i) + sxy * cy(i) + sz * cz(i));
                d[i] = Store<S>::load(src + (size_t)i * N, (unsigned)s, I.inv_scale);
                sf[i] = I.flags[(unsigned)s];
            }
        } else {
            const bool px = I.periodic & 1, py = I.periodic & 2, pz = I.periodic & 4;
            const int xm = step_axis(x, -1, I.nx, px), xp = step_axis(x, 1, I.nx, px);
            const int ym = step_axis(y, -1, I.ny, py), yp = step_axis(y, 1, I.ny, py);
            const int zm = step_axis(z, -1, I.nz, pz), zp = step_axis(z, 1, I.nz, pz);
            // a wall source reads this cell's own flag (liquid) and, for the
            // halfway bounce-back, its own f_ibar
#pragma unroll
            for (int i = 1; i < Q; ++i) {
                const int X = cx(i) == 1 ? xm : (cx(i) == -1 ? xp : x);
                const int Y = cy(i) == 1 ? ym : (cy(i) == -1 ? yp : y);
                const int Z = cz(i) == 1 ? zm : (cz(i) == -1 ? zp : z);
                const bool ok = (X | Y | Z) >= 0;
                const int s = ok ? X + I.nx * (Y + I.ny * Z) : id;
                const int arr = ok ? i : opp(i);
                d[i] = Store<S>::load(src + (size_t)arr * N, (unsigned)s, I.inv_scale);
                sf[i] = I.flags[(unsigned)s];
            }
        }
        uint32_t bad = 0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const uint32_t st = sf[i] & TYPE_MASK;
            bad |= (uint32_t)(st == GAS) | (uint32_t)(st == OBS);
        }
        if (bad) defer = true;
        else collide_store<S>(I, d, dst, N, id);
    }
    wave_append(defer, id, I.bnd, &C.n_bnd, I.list_cap, &C.overflow);
}

// ---------------------------------------------------------------------------
// boundary sweep: interface cells, liquid cells next to gas or a body.
// One group of 32 lanes per cell: lane i (< 19) owns link i; moments, the
// mass exchange and the momentum exchange are butterfly reductions over the
// group, values of the opposite link come from lane ibar by a shuffle.
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

    const int i = threadIdx.x & 31;          // link of this lane
    const int gbase = threadIdx.x & 32;      // first lane of this group in the wavefront
    const bool link = i < Q;
    const int cxi = link ? lane_c(CXP, i) : 0, cyi = link ? lane_c(CYP, i) : 0, czi = link ? lane_c(CZP, i) : 0;
    const int oi = link ? lane_opp(i) : i;
    const float wi = lane_w(i);
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    // this wavefront's momentum-exchange partial sum (first body it meets)
    int rec_body = -1;
    double rv[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};

    for (int k0 = 2 * wave; k0 < nlist; k0 += 2 * nwaves) {
        const int k = k0 + (gbase >> 5);
        const bool active = k < nlist;
        const int id = active ? I.bnd[k] : I.bnd[k0];
        int x, y, z;
        cell_coords(I, id, x, y, z);
        const uint8_t fl = I.flags[id];
        const int type = fl & TYPE_MASK;

        // source of this lane's link and everything read from it
        const int X = step_axis(x, -cxi, I.nx, px), Y = step_axis(y, -cyi, I.ny, py), Z = step_axis(z, -czi, I.nz, pz);
        const bool ok = link && (X | Y | Z) >= 0;
        const int s = ok ? X + I.nx * (Y + I.ny * Z) : id;
        const uint8_t sf = ok ? I.flags[s] : (uint8_t)OBS;  // wall: obstacle at rest
        const int st = sf & TYPE_MASK;
        const float sph = I.phi[parity][s];
        const float draw = link ? Store<S>::ld(src, (size_t)i * N + s, isc) : 0.f;
        const float dxi = link ? Store<S>::ld(src, (size_t)i * N + id, isc) : 0.f;
        const float phix = type == IFC ? I.phi[parity][id] : 1.f;
        float mhi = 0.f, mlo = 0.f;
        if (type == IFC) {
            mhi = I.m_hi[id];
            mlo = I.m_lo[id];
        }
        // the opposite link's lane: own f_ibar(x); raw f_ibar(x + c_i) and
        // its type / fill (x + c_i is the source of link ibar)
        const float dxo = __shfl(dxi, gbase + oi);
        const float drawo = __shfl(draw, gbase + oi);
        const int sto = __shfl(ok ? st : -1, gbase + oi);
        const float spho = __shfl(sph, gbase + oi);

        // moments of f(x, t)
        const float drx = gsum(dxi);
        const float jx0 = gsum(cxi * dxi), jx1 = gsum(cyi * dxi), jx2 = gsum(czi * dxi);
        const float rhox = 1.f + drx;
        const float ux0 = jx0 / rhox, ux1 = jx1 / rhox, ux2 = jx2 / rhox;
        const float uu = ux0 * ux0 + ux1 * ux1 + ux2 * ux2;

        // interface normal n = -grad(phi): fill of the sources of links 1..6
        // (FP64 sign test, same operations on every lane)
        double n0 = 0.0, n1 = 0.0, n2 = 0.0, nthr = 0.0;
        if (type == IFC && I.recon_mode != LBM_RECON_GAS_ONLY) {
            double fv = (double)phix;  // wall / obstacle: own fill
            if (ok && st == LIQ) fv = 1.0;
            else if (ok && st == GAS) fv = 0.0;
            else if (ok && st == IFC) fv = (double)sph;
            const double f1 = __shfl(fv, gbase + 1), f2 = __shfl(fv, gbase + 2), f3 = __shfl(fv, gbase + 3);
            const double f4 = __shfl(fv, gbase + 4), f5 = __shfl(fv, gbase + 5), f6 = __shfl(fv, gbase + 6);
            // the source of link E (c = +x) is x-1, of W (c = -x) is x+1
            n0 = 0.5 * (f2 - f1);
            n1 = 0.5 * (f3 - f4);
            n2 = 0.5 * (f5 - f6);
            nthr = NORMAL_TOL * ((fabs(n0) + fabs(n1)) + fabs(n2));
        }

        // mass exchange with neighbour x + c_i (interface cells)
        float dmi = 0.f;
        if (type == IFC && link && i > 0) {
            const float ex = drawo - dxi;
            if (sto == LIQ) dmi = ex;
            else if (sto == IFC) dmi = 0.5f * (phix + spho) * ex;
        }
        const float dm = gsum(dmi);

        // this lane's incoming population
        float dpi = draw;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f, a5 = 0.f;
        int bk = -1;
        if (i == 0) {
            dpi = dxi;
        } else if (link && (!ok || st == OBS)) {
            float cu = 0.f;
            float r0 = 0.f, r1 = 0.f, r2 = 0.f;
            const float xc0 = x + 0.5f, xc1 = y + 0.5f, xc2 = z + 0.5f;
            if (ok) {
                bk = (sf >> 2) & 15;
                const DevBody& B = I.bodies[bk];
                // body velocity at the link midpoint x_c - c_i/2
                const float p0 = (float)wrap_rel(xc0 - 0.5f * cxi - B.pos[0], I.nx, px);
                const float p1 = (float)wrap_rel(xc1 - 0.5f * cyi - B.pos[1], I.ny, py);
                const float p2 = (float)wrap_rel(xc2 - 0.5f * czi - B.pos[2], I.nz, pz);
                const float w0 = (float)B.omega[0], w1 = (float)B.omega[1], w2 = (float)B.omega[2];
                const float u0 = (float)B.vel[0] + (w1 * p2 - w2 * p1);
                const float u1 = (float)B.vel[1] + (w2 * p0 - w0 * p2);
                const float u2 = (float)B.vel[2] + (w0 * p1 - w1 * p0);
                cu = cxi * u0 + cyi * u1 + czi * u2;
                r0 = (float)wrap_rel(xc0 - B.pos[0], I.nx, px);
                r1 = (float)wrap_rel(xc1 - B.pos[1], I.ny, py);
                r2 = (float)wrap_rel(xc2 - B.pos[2], I.nz, pz);
            }
            const float mw = 6.f * wi * rhox * cu;
            dpi = dxo + mw;
            if (bk >= 0) {
                // momentum the fluid gains on this link (deviation form); the
                // body receives the opposite
                const float phat = type == LIQ ? 1.f : phix;
                const float amp = 2.f * phat * (dxo + wi * (1.f - I.rho_g) + 0.5f * mw);
                const float j0 = amp * cxi, j1 = amp * cyi, j2 = amp * czi;
                a0 = -j0;
                a1 = -j1;
                a2 = -j2;
                a3 = -(r1 * j2 - r2 * j1);
                a4 = -(r2 * j0 - r0 * j2);
                a5 = -(r0 * j1 - r1 * j0);
            }
        } else if (link) {
            bool recon = (st == GAS);
            if (!recon && type == IFC && I.recon_mode != LBM_RECON_GAS_ONLY) {
                const double cn = cxi * n0 + cyi * n1 + czi * n2;
                recon = I.recon_mode == LBM_RECON_GAS_SIDE ? (cn < -nthr) : (cn <= nthr);
            }
            if (recon) {
                const float cu = cxi * ux0 + cyi * ux1 + czi * ux2;
                // (f_eq,i + f_eq,ibar)(rho_G, u_x) - 2 w_i, minus d_ibar(x)
                dpi = 2.f * wi * (I.rho_g * (1.f + 4.5f * cu * cu - 1.5f * uu) - 1.f) - dxo;
            }
        }
        if (!active || !link) dpi = 0.f;

        // moments after streaming, collide
        const float drho = gsum(dpi);
        const float j0 = gsum(cxi * dpi), j1 = gsum(cyi * dpi), j2 = gsum(czi * dpi);
        const float rho = 1.f + drho;
        uint8_t mark = 0;
        if (type == IFC) {
            two_sum_add(mhi, mlo, dm);
            const float ph = (float)(((double)mhi + (double)mlo) / (1.0 + (double)drho));
            const double phd = (double)ph;
            if (phd >= 1.0 + I.eps) mark = MARK_FILL;
            else if (phd <= -I.eps) mark = MARK_EMPTY;
            if (active && i == 0) {
                I.m_hi[id] = mhi;
                I.m_lo[id] = mlo;
                I.phi[parity ^ 1][id] = ph;
                if (mark) I.flags[id] = (fl & KEEP_MASK) | mark;
            }
        }
        if (active && link) {
            const float irho = 1.f / rho;
            const float u0 = j0 * irho, u1 = j1 * irho, u2 = j2 * irho;
            const float cu = cxi * u0 + cyi * u1 + czi * u2;
            const float ca = cxi * I.ax + cyi * I.ay + czi * I.az;
            const float ua = u0 * I.ax + u1 * I.ay + u2 * I.az;
            const float deq = wi * (drho + rho * (3.f * cu + 4.5f * cu * cu - 1.5f * (u0 * u0 + u1 * u1 + u2 * u2)));
            const float F = wi * rho * (3.f * (ca - ua) + 9.f * cu * ca);
            Store<S>::store(dst, (size_t)i * N + id, dpi + I.omega * (deq - dpi) + F, I.scale);
            if (i == 0 && !(rho > 0.f && rho < 1e6f)) atomicOr(&I.ctl->nonfinite, 1);
        }

        // candidates for the conversion phase (one lane per group)
        wave_append(active && i == 0 && mark != 0, id, I.cand, &C.n_cand, I.list_cap, &C.overflow);

        // momentum exchange: wavefront reduction in FP64 into this wavefront's
        // record (first body it meets), FP64 atomics for any other body
        const bool has = active && bk >= 0;
        unsigned long long m = __ballot(has);
        while (m) {
            const int leader = __ffsll((long long)m) - 1;
            const int b = __shfl(bk, leader);
            const bool mine = has && bk == b;
            double v[6];
            v[0] = wave_sum(mine ? (double)a0 : 0.0);
            v[1] = wave_sum(mine ? (double)a1 : 0.0);
            v[2] = wave_sum(mine ? (double)a2 : 0.0);
            v[3] = wave_sum(mine ? (double)a3 : 0.0);
            v[4] = wave_sum(mine ? (double)a4 : 0.0);
            v[5] = wave_sum(mine ? (double)a5 : 0.0);
            if (rec_body < 0) rec_body = b;
            if (b == rec_body) {
#pragma unroll
                for (int q = 0; q < 6; ++q) rv[q] += v[q];
            } else if (lane_id() == leader) {
#pragma unroll
                for (int q = 0; q < 6; ++q) atomicAdd(&C.acc[b][q], v[q]);
            }
            m &= ~__ballot(mine);
        }
    }
    // the workgroup's record: its wavefronts' records in wavefront order
    __shared__ int sb[4];
    __shared__ double sv[4][6];
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0) {
        sb[wv] = rec_body;
#pragma unroll
        for (int q = 0; q < 6; ++q) sv[wv][q] = rv[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int body = -1;
        double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int w = 0; w < 4; ++w) {
            const int b = sb[w];
            if (b < 0) continue;
            if (body < 0) body = b;
            if (b == body) {
#pragma unroll
                for (int q = 0; q < 6; ++q) acc[q] += sv[w][q];
            } else {
#pragma unroll
                for (int q = 0; q < 6; ++q) atomicAdd(&C.acc[b][q], sv[w][q]);
            }
        }
        I.frec_body[blockIdx.x] = body;
#pragma unroll
        for (int q = 0; q < 6; ++q) I.frec_v[q * BND_BLOCKS_MAX + blockIdx.x] = acc[q];
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
    const dim3 g(boundary_blocks(I)), b(256);
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
