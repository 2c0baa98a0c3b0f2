// k_tension.hip -- surface tension (Sec. 2.2, Laplace pressure).
//
// With a surface tension sigma the gas pressure that an interface cell
// rebuilds its gas-side populations with is p_G + 2 sigma kappa, kappa the
// local mean curvature of the free surface.  The paper leaves the stencil
// open (it names deriving kappa from the surface normals of a neighbourhood
// as a second step after the normals).  Here:
//   n_hat(y)  = n(y) / |n(y)|, n the central-difference normal -grad(phi)
//               of the reconstruction (liquid 1, gas 0, interface phi; an
//               obstacle or wall neighbour lends the cell's own fill);
//               zero where the fill is flat
//   kappa(x)  = 1/2 div(n_hat) at an interface cell x, the divergence by
//               central differences over the six axis neighbours; an
//               obstacle neighbour or one beyond a wall lends n_hat(x)
// n points from the liquid to the gas, so a droplet of radius R has
// kappa = 1/R and a gas bubble -1/R.  The boundary sweep adds
// 2 sigma kappa / cs^2 = 6 sigma kappa to rho_G at interface cells.
//
// One pass over the step's boundary list between the bulk and the boundary
// sweep.  Eight lanes per list entry: lane 0 takes the cell's own normal,
// lanes 1-6 the normal of neighbour +x, -x, +y, -y, +z, -z.  Every load of a
// lane depends only on the list entry, so the chain is two loads deep (the
// entry, then the cell's, its neighbour's and that neighbour's six
// neighbours' flags and fills together); lane 0 gathers the six components by
// shuffles.  Double precision, like the reconstruction's normal sign test.
#include "lgs_internal.h"

namespace lgs {

namespace {
__device__ __forceinline__ int axis_step(const Inst& I, int& X, int& Y, int& Z, int a, int d) {
    if (a == 0) X = step_axis(X, d, I.nx, I.periodic & 1);
    else if (a == 1) Y = step_axis(Y, d, I.ny, I.periodic & 2);
    else Z = step_axis(Z, d, I.nz, I.periodic & 4);
    return (X | Y | Z) >= 0 ? X + I.nx * (Y + I.ny * Z) : -1;
}

// Workgroup wg of nwg over the list, 32 entries per pass.
__device__ void curvature_list(const Inst& I, int parity, int wg, int nwg) {
    const int nlist = min(I.ctl->cnt[parity].n_bnd, I.list_cap);
    const float* __restrict__ phi_t = phi_of(I, parity);
    const int l = threadIdx.x & 7;
    const int cell = threadIdx.x >> 3;
    for (int base = wg * 32; base < nlist; base += nwg * 32) {
        const int k = base + cell;
        const int id = I.bnd[k < nlist ? k : base];
        int x, y, z;
        cell_coords(I, id, x, y, z);
        // this lane's cell: the listed cell itself or one axis neighbour
        // (inl = 0 beyond a wall)
        int c = id;
        bool inl = true;
        if (l >= 1 && l <= 6) {
            int X = x, Y = y, Z = z;
            c = axis_step(I, X, Y, Z, (l - 1) >> 1, (l & 1) ? 1 : -1);
            inl = c >= 0;
            if (inl) {
                x = X;
                y = Y;
                z = Z;
            } else {
                c = id;
            }
        }
        // all loads at once: the listed cell's flag, this lane's cell and its
        // six neighbours
        const uint8_t fid = I.flags[id];
        const uint8_t fc = I.flags[c];
        const float pc = phi_t[c];
        int tn[6];
        float pn[6];
        bool hn[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            int X = x, Y = y, Z = z;
            const int s = inl && l <= 6 ? axis_step(I, X, Y, Z, j >> 1, (j & 1) ? 1 : -1) : -1;
            hn[j] = s >= 0;
            const int sc = hn[j] ? s : c;
            tn[j] = I.flags[sc] & TYPE_MASK;
            pn[j] = phi_t[sc];
        }
        const bool act = k < nlist && (fid & TYPE_MASK) == IFC;
        const int tc = fc & TYPE_MASK;
        const bool ok = inl && tc != OBS && l <= 6;
        const double own = tc == LIQ ? 1.0 : tc == IFC ? (double)pc : 0.0;
        double f[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const int t = tn[j];
            f[j] = !hn[j] ? own : t == LIQ ? 1.0 : t == GAS ? 0.0 : t == IFC ? (double)pn[j] : own;
        }
        // f[2a] is the fill at -1 along axis a, f[2a+1] at +1
        double n[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) n[a] = 0.5 * (f[2 * a] - f[2 * a + 1]);
        const double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (len > 0.0) {
#pragma unroll
            for (int a = 0; a < 3; ++a) n[a] /= len;
        }
        // lane 1 + 2a + j (j = 0: the +1 neighbour, j = 1: the -1 one)
        // offers component a of its normal
        const int my_a = l >= 1 && l <= 6 ? (l - 1) >> 1 : 0;
        const double mine = my_a == 0 ? n[0] : my_a == 1 ? n[1] : n[2];
        const int g0 = __lane_id() & ~7;
        double div = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double vp = __shfl(mine, g0 + 1 + 2 * a);
            const int op = __shfl((int)ok, g0 + 1 + 2 * a);
            const double vm = __shfl(mine, g0 + 2 + 2 * a);
            const int om = __shfl((int)ok, g0 + 2 + 2 * a);
            const double sp = op ? vp : n[a], sm = om ? vm : n[a];
            div += 0.5 * (sp - sm);
        }
        if (act && l == 0) I.kap[id] = (float)(0.5 * div);
    }
}
}  // namespace

__global__ __launch_bounds__(256) void k_curvature(Inst I, int parity) {
    curvature_list(I, parity, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(256) void kb_curvature(const Inst* __restrict__ tab, const int* __restrict__ off, int n,
                                                    int parity) {
    const int k = batch_instance(off, n, blockIdx.x);
    const Inst I = tab[k];
    const int b = blockIdx.x - off[k];
    if (I.lap == 0.f || b >= boundary_blocks(I)) return;
    curvature_list(I, parity, b, boundary_blocks(I));
}

void launch_curvature(const Inst& I, int parity, hipStream_t s) {
    hipLaunchKernelGGL(k_curvature, dim3(boundary_blocks(I)), dim3(256), 0, s, I, parity);
}

void launch_curvature_batch(const BatchGrid& G, int parity, hipStream_t s) {
    hipLaunchKernelGGL(kb_curvature, dim3(G.blocks), dim3(256), 0, s, G.tab, G.off, G.n, parity);
}

}  // namespace lgs
