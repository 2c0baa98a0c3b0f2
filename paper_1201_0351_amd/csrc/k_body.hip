// k_body.hip -- basin initialisation, body upload, body remap (Sec. 2.3 cell
// mapping, Sec. 2.4 conversions into and out of obstacle), and reductions.
//
// Remap of a moved body k works on a box of cells around the union of its
// last mapped and its new pose (computed on the device from the body record,
// so the launch does not depend on the pose) and runs in two kernels:
//   eval    every cell of the region that is an obstacle cell no longer
//           inside its body's new pose ("uncovered") gets its rule from the
//           pre-remap state: B(x) = neighbours that are not obstacle and not
//           inside any body's new pose;
//             no LIQ in B      -> GAS           (rule 1)
//             no GAS in B      -> LIQ           (rule 2)
//             both             -> IF            (rule 3)
//           rho = mean rho over the non-gas members, phi = mean phi over the
//           interface members (else #LIQ/(#LIQ+#GAS), or 1 for rule 2).
//           All other cells of the region get rule 0.  Overlapping regions
//           compute identical values.
//   commit  cover: fluid cells inside the new pose become OBS(k); their mass
//           leaves the fluid (ledger).  Uncover: apply the rule, a rule-2 cell
//           touching a rule-1 cell becomes IF (fix-up); f = f_eq(rho,
//           u_w(closest surface point)); the new mass enters the ledger.
#include <cstddef>

#include "lgs_internal.h"

namespace lgs {

namespace {

__device__ __forceinline__ double splitmix64_unit(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ double fill0(double H, int z) {
    double p = H - z;
    return p < 0.0 ? 0.0 : (p > 1.0 ? 1.0 : p);
}

template <typename S>
__device__ __forceinline__ void write_feq(const Inst& I, S* pop, int id, double rho, const double u[3]) {
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double cu = cx(i) * u[0] + cy(i) * u[1] + cz(i) * u[2];
        const double w = wgtd(i);
        const double dev = w * ((rho - 1.0) + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
        Store<S>::st(pop, (size_t)i * I.ps + id, (float)dev, I.scale);
    }
}

template <typename S>
__device__ __forceinline__ float cell_drho(const Inst& I, const S* pop, int id) {
    float dr = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) dr += Store<S>::ld(pop, (size_t)i * I.ps + id, I.inv_scale);
    return dr;
}

__device__ __forceinline__ void split_mass(double m, float& hi, float& lo) {
    hi = (float)m;
    lo = (float)(m - (double)hi);
}

}  // namespace

// ---------------------------------------------------------------------------
// initialisation: flat basin of fill height H (hydrostatic, optional shear)
// ---------------------------------------------------------------------------
struct InitParams {
    double H, us, rho_g, az, noise;
    uint64_t seed;
};

template <typename S>
__global__ __launch_bounds__(256) void k_init(Inst I, InitParams P) {
    const int id = blockIdx.x * 256 + threadIdx.x;
    if (id >= I.N) return;
    int x, y, z;
    cell_coords(I, id, x, y, z);
    const double ph = fill0(P.H, z);
    int t = ph >= 1.0 ? LIQ : (ph > 0.0 ? IFC : GAS);
    if (t == LIQ) {
        for (int i = 1; i < Q; ++i) {
            const int nb = nbr_index(I, x, y, z, cx(i), cy(i), cz(i));
            if (nb < 0) continue;
            int zx, zy, zz;
            cell_coords(I, nb, zx, zy, zz);
            if (fill0(P.H, zz) <= 0.0) {
                t = IFC;
                break;
            }
        }
    }
    S* p0 = (S*)pop_of(I, 0);
    S* p1 = (S*)pop_of(I, 1);
    I.flags[id] = (uint8_t)t;
    if (t == GAS) {
        for (int i = 0; i < Q; ++i) {
            Store<S>::st(p0, (size_t)i * I.ps + id, 0.f, I.scale);
            Store<S>::st(p1, (size_t)i * I.ps + id, 0.f, I.scale);
        }
        I.m_hi[id] = I.m_lo[id] = 0.f;
        phi_of(I, 0)[id] = phi_of(I, 1)[id] = 0.f;
        return;
    }
    const double zc = z + 0.5;
    double rho = P.rho_g - 3.0 * P.az * (P.H - zc);
    if (P.noise != 0.0) rho += P.noise * (2.0 * splitmix64_unit(P.seed ^ (uint64_t)id) - 1.0);
    double u[3] = {0.0, 0.0, 0.0};
    if (P.us != 0.0 && P.H > 0.0) u[0] = P.us * zc * (2.0 * P.H - zc) / (P.H * P.H);
    write_feq<S>(I, p0, id, rho, u);
    for (int i = 0; i < Q; ++i) Store<S>::st(p1, (size_t)i * I.ps + id, 0.f, I.scale);
    float hi, lo;
    split_mass(ph * rho, hi, lo);
    I.m_hi[id] = hi;
    I.m_lo[id] = lo;
    phi_of(I, 0)[id] = phi_of(I, 1)[id] = (float)ph;
}

// Highest layer with a liquid or interface cell or a mark: each workgroup
// scans a contiguous chunk of cells and adds one atomicMax.
constexpr int ZTOP_CHUNK = 1 << 12;
__global__ __launch_bounds__(256) void k_ztop(Inst I) {
    const size_t c0 = (size_t)blockIdx.x * ZTOP_CHUNK;
    const size_t c1 = c0 + ZTOP_CHUNK < (size_t)I.N ? c0 + ZTOP_CHUNK : (size_t)I.N;
    const size_t layer = (size_t)I.nx * I.ny;
    int top = -1;
    for (size_t id = c0 + threadIdx.x; id < c1; id += 256) {
        const uint8_t f = I.flags[id];
        const int t = f & TYPE_MASK;
        if (t == LIQ || t == IFC || (f & ~KEEP_MASK)) top = (int)(id / layer);  // ids ascend: the last is the highest
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) top = max(top, __shfl_xor(top, o));
    __shared__ int wm[4];
    if (__lane_id() == 0) wm[threadIdx.x >> 6] = top;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int m = max(max(wm[0], wm[1]), max(wm[2], wm[3]));
        if (m >= 0) atomicMax(&I.ctl->ztop, m);
    }
}

void launch_ztop(const Inst& I, hipStream_t s) {
    const dim3 g((unsigned)(((size_t)I.N + ZTOP_CHUNK - 1) / ZTOP_CHUNK)), b(256);
    hipLaunchKernelGGL(k_ztop, g, b, 0, s, I);
}

void launch_init(const Inst& I, const lbm_config& c, hipStream_t s) {
    InitParams P{c.fill_height, c.init_ux_surface, c.rho_gas, c.accel[2], c.noise_amp, c.seed};
    const dim3 g((I.N + 255) / 256), b(256);
    switch (I.storage) {
    case LBM_FP16_DEV: hipLaunchKernelGGL(k_init<__half>, g, b, 0, s, I, P); break;
    case LBM_BF16_DEV: hipLaunchKernelGGL(k_init<__hip_bfloat16>, g, b, 0, s, I, P); break;
    default: hipLaunchKernelGGL(k_init<float>, g, b, 0, s, I, P); break;
    }
}

// ---------------------------------------------------------------------------
// body upload (parameters travel as kernel arguments: no host staging buffer)
// ---------------------------------------------------------------------------
__global__ void k_set_body(DevBody* dst, DevBody v) {
    if (threadIdx.x == 0) *dst = v;
}

void launch_set_body(const Inst& I, int slot, const DevBody& b, hipStream_t s) {
    hipLaunchKernelGGL(k_set_body, dim3(1), dim3(64), 0, s, I.bodies + slot, b);
}

// ---------------------------------------------------------------------------
// remap
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool region_cell(const Inst& I, const Region& R, int local, int& x, int& y, int& z) {
    const int d0 = R.dim[0], d1 = R.dim[1];
    const int l[3] = {local % d0, (local / d0) % d1, local / (d0 * d1)};
    const int n[3] = {I.nx, I.ny, I.nz};
    int c[3];
    for (int a = 0; a < 3; ++a) {
        int v = R.lo[a] + l[a];
        if (I.periodic & (1 << a)) v = ((v % n[a]) + n[a]) % n[a];
        else if (v < 0 || v >= n[a]) return false;
        c[a] = v;
    }
    x = c[0];
    y = c[1];
    z = c[2];
    return true;
}

// remap rule of one cell of body k's region (pre-remap state only)
template <typename S>
__device__ __forceinline__ void remap_eval_cell(const Inst& I, int parity, const Region& R, int local) {
    int x, y, z;
    if (!region_cell(I, R, local, x, y, z)) return;
    const int id = x + I.nx * (y + I.ny * z);
    const uint8_t fl = I.flags[id];
    uint8_t r = 0;
    if ((fl & TYPE_MASK) == OBS) {
        const int owner = (fl >> 2) & 15;
        if (!inside_body(I, I.bodies[owner], x, y, z) && body_at(I, x, y, z) < 0) {
            const S* pop = (const S*)pop_of(I, parity);
            int nL = 0, nG = 0, nI = 0;
            float rs = 0.f, ps = 0.f;
            for (int i = 1; i < Q; ++i) {
                const int X = step_axis(x, cx(i), I.nx, I.periodic & 1);
                const int Y = step_axis(y, cy(i), I.ny, I.periodic & 2);
                const int Z = step_axis(z, cz(i), I.nz, I.periodic & 4);
                if ((X | Y | Z) < 0) continue;
                const int nb = X + I.nx * (Y + I.ny * Z);
                const int t = I.flags[nb] & TYPE_MASK;
                if (t == OBS || body_at(I, X, Y, Z) >= 0) continue;
                if (t == GAS) {
                    ++nG;
                } else {
                    rs += cell_drho<S>(I, pop, nb);
                    if (t == LIQ) {
                        ++nL;
                    } else {
                        ++nI;
                        ps += phi_of(I, parity)[nb];
                    }
                }
            }
            if (nL == 0) {
                r = 1;
            } else {
                r = nG == 0 ? 2 : 3;
                I.share[id] = rs / (float)(nL + nI);  // mean (rho - 1)
                float pb;
                if (nI > 0) pb = ps / (float)nI;
                else pb = nG == 0 ? 1.f : (float)nL / (float)(nL + nG);
                I.aux[id] = pb;
            }
        }
    }
    I.rule[id] = r;
}

// cover / uncover one cell of body k's region
template <typename S>
__device__ __forceinline__ void remap_commit_cell(const Inst& I, int parity, int k, const DevBody& B,
                                                  const Region& R, int local) {
    int x, y, z;
    if (!region_cell(I, R, local, x, y, z)) return;
    const int id = x + I.nx * (y + I.ny * z);
    const uint8_t fl = I.flags[id];
    const int t = fl & TYPE_MASK;
    S* pop = (S*)pop_of(I, parity);
    if (t != OBS) {
        if (!inside_body(I, B, x, y, z)) return;
        double lost = 0.0;
        if (t == LIQ) lost = 1.0 + (double)cell_drho<S>(I, pop, id);
        else if (t == IFC) lost = (double)I.m_hi[id] + (double)I.m_lo[id];
        if (lost != 0.0) atomicAdd(&I.ctl->ledger, -lost);
        I.flags[id] = (uint8_t)(OBS | (k << 2));
        I.m_hi[id] = I.m_lo[id] = 0.f;
        phi_of(I, parity)[id] = 0.f;
        // every neighbour now has an obstacle neighbour
        for (int i = 1; i < Q; ++i) {
            const int nb = nbr_index(I, x, y, z, cx(i), cy(i), cz(i));
            if (nb >= 0) I.nearo[nb] = 1;
        }
        return;
    }
    if (((fl >> 2) & 15) != k) return;
    int r = I.rule[id];
    if (r == 0) return;
    I.nearo[id] = 1;  // an uncovered cell borders the body (the bulk sweep clears it otherwise)
    if (r == 2) {
        for (int i = 1; i < Q; ++i) {
            const int nb = nbr_index(I, x, y, z, cx(i), cy(i), cz(i));
            if (nb >= 0 && I.rule[nb] == 1) {
                r = 4;
                break;
            }
        }
    }
    if (r == 1) {
        I.flags[id] = GAS;
        I.m_hi[id] = I.m_lo[id] = 0.f;
        phi_of(I, parity)[id] = 0.f;
        return;
    }
    // velocity of the closest point of the body surface
    double u[3];
    {
#pragma clang fp contract(off)
        double d0 = wrap_rel((x + 0.5) - B.pos[0], (double)I.nx, I.periodic & 1);
        double d1 = wrap_rel((y + 0.5) - B.pos[1], (double)I.ny, I.periodic & 2);
        double d2 = wrap_rel((z + 0.5) - B.pos[2], (double)I.nz, I.periodic & 4);
        double p[3];
        if (B.shape == LBM_SHAPE_SPHERE) {
            // the centre's offset scaled to the radius
            const double dn = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            const double sc = dn > B.half[0] ? B.half[0] / dn : 1.0;
            p[0] = d0 * sc;
            p[1] = d1 * sc;
            p[2] = d2 * sc;
        } else {
            // clamped to the cuboid in the body frame
            double rb[3] = {B.R[0] * d0 + B.R[3] * d1 + B.R[6] * d2, B.R[1] * d0 + B.R[4] * d1 + B.R[7] * d2,
                            B.R[2] * d0 + B.R[5] * d1 + B.R[8] * d2};
            for (int a = 0; a < 3; ++a)
                rb[a] = rb[a] < -B.half[a] ? -B.half[a] : (rb[a] > B.half[a] ? B.half[a] : rb[a]);
            for (int a = 0; a < 3; ++a)
                p[a] = B.R[a * 3 + 0] * rb[0] + B.R[a * 3 + 1] * rb[1] + B.R[a * 3 + 2] * rb[2];
        }
        u[0] = B.vel[0] + (B.omega[1] * p[2] - B.omega[2] * p[1]);
        u[1] = B.vel[1] + (B.omega[2] * p[0] - B.omega[0] * p[2]);
        u[2] = B.vel[2] + (B.omega[0] * p[1] - B.omega[1] * p[0]);
    }
    const double drb = (double)I.share[id];
    const double rho = 1.0 + drb;
    write_feq<S>(I, pop, id, rho, u);
    float hi, lo;
    double m;
    atomicMax(&I.ctl->ztop, z);  // a fluid cell again
    if (r == 2) {
        I.flags[id] = LIQ;
        hi = 1.f;
        lo = (float)drb;
        m = rho;
        phi_of(I, parity)[id] = 1.f;
    } else {
        const double ph = (double)I.aux[id];
        I.flags[id] = IFC;
        m = ph * rho;
        split_mass(m, hi, lo);
        phi_of(I, parity)[id] = (float)ph;
    }
    I.m_hi[id] = hi;
    I.m_lo[id] = lo;
    atomicAdd(&I.ctl->ledger, m);
}

// workgroup b of nb working on body k's region
template <typename S>
__device__ __forceinline__ void remap_eval(const Inst& I, int parity, int k, int b, int nb) {
    if (k >= I.nbodies) return;
    const DevBody& B = I.bodies[k];
    if (!B.active || !B.moved) return;
    const Region R = body_region(B, I.nx, I.ny, I.nz, I.periodic);
    for (int local = b * 256 + threadIdx.x; local < R.cells; local += nb * 256) remap_eval_cell<S>(I, parity, R, local);
}

template <typename S>
__device__ __forceinline__ void remap_commit(const Inst& I, int parity, int k, int b, int nb) {
    if (k >= I.nbodies) return;
    const DevBody& B = I.bodies[k];
    if (!B.active || !B.moved) return;
    const Region R = body_region(B, I.nx, I.ny, I.nz, I.periodic);
    for (int local = b * 256 + threadIdx.x; local < R.cells; local += nb * 256)
        remap_commit_cell<S>(I, parity, k, B, R, local);
}

template <typename S>
__global__ __launch_bounds__(256) void k_remap_eval(Inst I, int parity) {
    remap_eval<S>(I, parity, blockIdx.y, blockIdx.x, gridDim.x);
}
template <typename S>
__global__ __launch_bounds__(256) void k_remap_commit(Inst I, int parity) {
    remap_commit<S>(I, parity, blockIdx.y, blockIdx.x, gridDim.x);
}
// a batch: instance blockIdx.z
template <typename S>
__global__ __launch_bounds__(256) void kb_remap_eval(const Inst* __restrict__ tab, int parity) {
    const Inst I = tab[blockIdx.z];
    remap_eval<S>(I, parity, blockIdx.y, blockIdx.x, gridDim.x);
}
template <typename S>
__global__ __launch_bounds__(256) void kb_remap_commit(const Inst* __restrict__ tab, int parity) {
    const Inst I = tab[blockIdx.z];
    remap_commit<S>(I, parity, blockIdx.y, blockIdx.x, gridDim.x);
}

void launch_remap(const Inst& I, int parity, int blocks_per_body, hipStream_t s) {
    if (I.nbodies == 0 || blocks_per_body <= 0) return;
    const dim3 g(blocks_per_body, I.nbodies), b(256);
    switch (I.storage) {
    case LBM_FP16_DEV:
        hipLaunchKernelGGL(k_remap_eval<__half>, g, b, 0, s, I, parity);
        hipLaunchKernelGGL(k_remap_commit<__half>, g, b, 0, s, I, parity);
        break;
    case LBM_BF16_DEV:
        hipLaunchKernelGGL(k_remap_eval<__hip_bfloat16>, g, b, 0, s, I, parity);
        hipLaunchKernelGGL(k_remap_commit<__hip_bfloat16>, g, b, 0, s, I, parity);
        break;
    default:
        hipLaunchKernelGGL(k_remap_eval<float>, g, b, 0, s, I, parity);
        hipLaunchKernelGGL(k_remap_commit<float>, g, b, 0, s, I, parity);
        break;
    }
}

void launch_remap_batch(const Inst* tab, int n, int max_bodies, int storage, int parity, int blocks_per_body,
                        hipStream_t s) {
    if (n == 0 || max_bodies == 0 || blocks_per_body <= 0) return;
    const dim3 g(blocks_per_body, max_bodies, n), b(256);
    switch (storage) {
    case LBM_FP16_DEV:
        hipLaunchKernelGGL(kb_remap_eval<__half>, g, b, 0, s, tab, parity);
        hipLaunchKernelGGL(kb_remap_commit<__half>, g, b, 0, s, tab, parity);
        break;
    case LBM_BF16_DEV:
        hipLaunchKernelGGL(kb_remap_eval<__hip_bfloat16>, g, b, 0, s, tab, parity);
        hipLaunchKernelGGL(kb_remap_commit<__hip_bfloat16>, g, b, 0, s, tab, parity);
        break;
    default:
        hipLaunchKernelGGL(kb_remap_eval<float>, g, b, 0, s, tab, parity);
        hipLaunchKernelGGL(kb_remap_commit<float>, g, b, 0, s, tab, parity);
        break;
    }
}

// ---------------------------------------------------------------------------
// diagnostics
// ---------------------------------------------------------------------------
__global__ void k_zero_diag(Ctl* c) {
    if (threadIdx.x == 0) c->contacts = 0ull;
}

// Partial liquid mass of chunk blockIdx.x (cells [b MASS_CHUNK, (b+1)
// MASS_CHUNK)): every thread sums its cells in index order, then a fixed
// tree over the workgroup.
template <typename S>
__global__ __launch_bounds__(256) void k_mass_part(Inst I, int parity, double* __restrict__ part) {
    __shared__ double red[256];
    double acc = 0.0;
    const S* pop = (const S*)pop_of(I, parity);
    const int lo = blockIdx.x * MASS_CHUNK, hi = min(I.N, lo + MASS_CHUNK);
    for (int id = lo + (int)threadIdx.x; id < hi; id += 256) {
        const int t = I.flags[id] & TYPE_MASK;
        if (t == LIQ) acc += 1.0 + (double)cell_drho<S>(I, pop, id);
        else if (t == IFC) acc += (double)I.m_hi[id] + (double)I.m_lo[id];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Sum of the n partials in a fixed order (one workgroup).
__global__ __launch_bounds__(256) void k_mass_sum(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) acc += part[k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

void launch_mass_total(const Inst& I, int parity, double* part, double* out, hipStream_t s) {
    const int n = mass_parts(I.N);
    const dim3 g(n), b(256);
    switch (I.storage) {
    case LBM_FP16_DEV: hipLaunchKernelGGL(k_mass_part<__half>, g, b, 0, s, I, parity, part); break;
    case LBM_BF16_DEV: hipLaunchKernelGGL(k_mass_part<__hip_bfloat16>, g, b, 0, s, I, parity, part); break;
    default: hipLaunchKernelGGL(k_mass_part<float>, g, b, 0, s, I, parity, part); break;
    }
    hipLaunchKernelGGL(k_mass_sum, dim3(1), b, 0, s, part, n, out);
}

__global__ __launch_bounds__(256) void k_contacts(Inst I) {
    for (int id = blockIdx.x * 256 + threadIdx.x; id < I.N; id += gridDim.x * 256) {
        if ((I.flags[id] & TYPE_MASK) != LIQ) continue;
        int x, y, z;
        cell_coords(I, id, x, y, z);
        for (int i = 1; i < Q; ++i) {
            const int nb = nbr_index(I, x, y, z, cx(i), cy(i), cz(i));
            if (nb >= 0 && (I.flags[nb] & TYPE_MASK) == GAS) {
                atomicAdd(&I.ctl->contacts, 1ull);
                break;
            }
        }
    }
}

void launch_contacts(const Inst& I, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_diag, dim3(1), dim3(64), 0, s, I.ctl);
    hipLaunchKernelGGL(k_contacts, dim3(min(1024, (I.N + 255) / 256)), dim3(256), 0, s, I);
}

}  // namespace lgs
