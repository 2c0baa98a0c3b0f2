/*
 * lgs_oracle.c -- FP64 CPU oracle for the liquid-gas-solid lattice Boltzmann
 * time step of Bogner & Ruede, "Liquid-gas-solid flows with lattice Boltzmann:
 * Simulation of floating bodies".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * Everything is double precision, cells are visited in linear index order
 * (x fastest), reductions are sequential in that order.  The only parallel
 * loop (OpenMP, optional) is the per-cell sweep, where every cell writes only
 * its own outputs.  Compile with -ffp-contract=off.
 *
 * Paper passages followed (section / equation labels of the paper):
 *   Sec. 2.1  D3Q19 velocities and weights (Fig. d3q19, Eq. links),
 *             equilibrium (Eq. equilibrium), force term (Eq. forceterm),
 *             moments (Eqs. density, momentum), stream (Eq. stream),
 *             collide (the split form of Eq. lbgk).
 *   Sec. 2.2  fill level and mass m = phi*rho, mass exchange (Delta m cases),
 *             gas-side reconstruction (Eq. reconstruct), normal from the
 *             fill-level gradient, interface conversions at -eps / 1+eps.
 *   Sec. 2.3  moving-wall bounce-back (Eq. noslip), momentum exchange
 *             (Eq. momentumexchange), cell-centre mapping of bodies,
 *             net force and torque sums (Eqs. netforce, torque).
 *   Sec. 2.4  obstacle->fluid rules on the non-obstacle neighbourhood B(x),
 *             gas-pressure momentum exchange (Eq. momentuminterface).
 *
 * Where the paper is silent, garbled or self-contradictory, the reading taken
 * is stated next to the code that implements it (and listed in the design
 * notes of the repository).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19
#define OB_MAXB 16

enum { T_GAS = 0, T_LIQ = 1, T_IF = 2, T_OBS = 3 };

/* ---------------------------------------------------------------------------
 * Sec. 2.1, Fig. d3q19 caption order: C, W, E, N, S, T, B, TW, TE, TN, TS,
 * NW, NE, SW, SE, BW, BE, BN, BS with E = +x, N = +y, T = +z.  Weights:
 * 1/3 for C, 1/18 for the six axis links, 1/36 for the twelve diagonals.
 * ------------------------------------------------------------------------- */
static const int CX[Q] = {0, -1, 1, 0, 0, 0, 0, -1, 1, 0, 0, -1, 1, -1, 1, -1, 1, 0, 0};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, 1, -1, -1, 0, 0, 1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 1, 1, 1, 1, 0, 0, 0, 0, -1, -1, -1, -1};
static double W[Q];
static int OPP[Q];
static int lattice_ready = 0;

static void lattice_setup(void) {
    if (lattice_ready) return;
    for (int i = 0; i < Q; ++i) {
        int nz = (CX[i] != 0) + (CY[i] != 0) + (CZ[i] != 0);
        W[i] = nz == 0 ? 1.0 / 3.0 : (nz == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        for (int j = 0; j < Q; ++j)
            if (CX[j] == -CX[i] && CY[j] == -CY[i] && CZ[j] == -CZ[i]) OPP[i] = j;
    }
    lattice_ready = 1;
}

/* c_s^2 = 1/3 (Sec. 2.1). */
/* relative tolerance of the c_i.n sign test in interface cells (a reading:
 * the paper does not say how the sign of a near-tangential link is taken) */
static const double NORMAL_TOL = 1e-3;
static const double CS2 = 1.0 / 3.0;

/* Eq. equilibrium:  rho w_i [1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)]. */
static double feq(int i, double rho, const double u[3]) {
    double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return rho * W[i] * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

/* Eq. forceterm, read as Luo's first-order term (the printed form is garbled:
 * the second part must be (c.u) c / cs^4, without the 1/2, for the term to
 * carry zero mass and momentum rho*a):
 *   F_i = w_i rho [ (c_i - u)/cs2 + (c_i.u) c_i / cs2^2 ] . a                  */
static double fterm(int i, double rho, const double u[3], const double a[3]) {
    double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
    double ca = CX[i] * a[0] + CY[i] * a[1] + CZ[i] * a[2];
    double ua = u[0] * a[0] + u[1] * a[1] + u[2] * a[2];
    return W[i] * rho * ((ca - ua) / CS2 + cu * ca / (CS2 * CS2));
}

/* ---------------------------------------------------------------------------
 * State
 * ------------------------------------------------------------------------- */
/* body shapes: a cuboid of half extents half[0..2], or a sphere of radius
 * half[0] */
enum { OB_CUBOID = 0, OB_SPHERE = 1 };
static const double OB_PI = 3.14159265358979323846;

typedef struct {
    int active, moved;
    int shape; /* OB_CUBOID or OB_SPHERE; kept when the pose is set again */
    double half[3], pos[3], quat[4], vel[3], omega[3], density;
    int fixed;
    double R[9]; /* body -> world rotation, row major */
    double force[3], torque[3];
    double fprev[3], tprev[3]; /* previous step's force / torque (coupled steps) */
    int have_prev;
} ob_body;

typedef struct {
    int nx, ny, nz;
    long N;
    double tau, a[3], rho_g, eps;
    double wall_u[3]; /* velocity of the non-periodic faces (moving no-slip walls) */
    double sigma;     /* surface tension; 0 = none */
    int per[3];
    int recon_mode;
    double *f, *fn;          /* [Q][N] absolute PDFs: current and next */
    unsigned char *type;     /* T_GAS .. T_OBS */
    signed char *bid;        /* owning body of OBS cells, -1 otherwise */
    double *m, *phi;         /* liquid mass and fill level (current) */
    double *mn, *phin;       /* next-step copies written by the sweep */
    double ledger;           /* mass added to the fluid minus mass removed */
    int nb;
    ob_body b[OB_MAXB];
    int nthreads;
    int stranded_rule;       /* 1: stranded interface cells empty at the conversions (default) */
    long last_conv[4];       /* counts of the last conversion pass: F, E, NEW_G, NEW_L */
} ob_state;

static inline long IDX(const ob_state *s, int x, int y, int z) {
    return (long)x + (long)s->nx * ((long)y + (long)s->ny * (long)z);
}

/* Neighbour of (x,y,z) along (dx,dy,dz).  Returns 0 if it lies outside a
 * non-periodic face (a static wall), else 1 with its index. */
static int nbr(const ob_state *s, int x, int y, int z, int dx, int dy, int dz, long *out) {
    int p[3] = {x + dx, y + dy, z + dz};
    int n[3] = {s->nx, s->ny, s->nz};
    for (int k = 0; k < 3; ++k) {
        if (p[k] < 0 || p[k] >= n[k]) {
            if (!s->per[k]) return 0;
            p[k] = (p[k] + n[k]) % n[k];
        }
    }
    *out = IDX(s, p[0], p[1], p[2]);
    return 1;
}

static void coords(const ob_state *s, long id, int *x, int *y, int *z) {
    *x = (int)(id % s->nx);
    *y = (int)((id / s->nx) % s->ny);
    *z = (int)(id / ((long)s->nx * s->ny));
}

static double cell_rho(const ob_state *s, const double *f, long id) {
    double r = 0.0;
    for (int i = 0; i < Q; ++i) r += f[(long)i * s->N + id];
    return r;
}

static void cell_u(const ob_state *s, const double *f, long id, double rho, double u[3]) {
    double j[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        double v = f[(long)i * s->N + id];
        j[0] += CX[i] * v;
        j[1] += CY[i] * v;
        j[2] += CZ[i] * v;
    }
    for (int k = 0; k < 3; ++k) u[k] = j[k] / rho;
}

/* ---------------------------------------------------------------------------
 * Body geometry (Sec. 2.3: a cell is an obstacle cell of a body iff its cell
 * centre (x+.5, y+.5, z+.5) lies inside the body volume).  Cuboid bodies with
 * half extents h in the body frame; the test is closed: |R^T (x_c - o)|_k <= h_k.
 * Spheres of radius r: |x_c - o|^2 <= r^2, the squares summed in axis order.
 * Periodic axes use the minimum image of x_c - o.
 * ------------------------------------------------------------------------- */
static void quat_to_R(const double q[4], double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
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

static double wrapd(double d, double L, int periodic) {
    if (!periodic) return d;
    if (d >= 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

/* world offset p - o (minimum image), for a point p */
static void rel(const ob_state *s, const ob_body *b, const double p[3], double d[3]) {
    double L[3] = {s->nx, s->ny, s->nz};
    for (int k = 0; k < 3; ++k) d[k] = wrapd(p[k] - b->pos[k], L[k], s->per[k]);
}

static void to_body(const ob_body *b, const double d[3], double r[3]) {
    for (int k = 0; k < 3; ++k) r[k] = b->R[0 * 3 + k] * d[0] + b->R[1 * 3 + k] * d[1] + b->R[2 * 3 + k] * d[2];
}

static int inside(const ob_state *s, const ob_body *b, int x, int y, int z) {
    double p[3] = {x + 0.5, y + 0.5, z + 0.5}, d[3], r[3];
    rel(s, b, p, d);
    if (b->shape == OB_SPHERE) return d[0] * d[0] + d[1] * d[1] + d[2] * d[2] <= b->half[0] * b->half[0];
    to_body(b, d, r);
    return fabs(r[0]) <= b->half[0] && fabs(r[1]) <= b->half[1] && fabs(r[2]) <= b->half[2];
}

/* Velocity of the rigid body at world offset d from its centre: V + Omega x d. */
static void body_vel(const ob_body *b, const double d[3], double u[3]) {
    u[0] = b->vel[0] + (b->omega[1] * d[2] - b->omega[2] * d[1]);
    u[1] = b->vel[1] + (b->omega[2] * d[0] - b->omega[0] * d[2]);
    u[2] = b->vel[2] + (b->omega[0] * d[1] - b->omega[1] * d[0]);
}

/* Sec. 2.4: velocity of the point of the body surface closest to the cell
 * centre (for a cuboid and a centre outside it: clamp in the body frame; for
 * a sphere: the centre's offset scaled to the radius). */
static void closest_surface_vel(const ob_state *s, const ob_body *b, int x, int y, int z, double u[3]) {
    double p[3] = {x + 0.5, y + 0.5, z + 0.5}, d[3], r[3], c[3], dw[3];
    rel(s, b, p, d);
    if (b->shape == OB_SPHERE) {
        double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double sc = dn > b->half[0] ? b->half[0] / dn : 1.0;
        for (int k = 0; k < 3; ++k) dw[k] = d[k] * sc;
        body_vel(b, dw, u);
        return;
    }
    to_body(b, d, r);
    for (int k = 0; k < 3; ++k) c[k] = r[k] < -b->half[k] ? -b->half[k] : (r[k] > b->half[k] ? b->half[k] : r[k]);
    for (int k = 0; k < 3; ++k) dw[k] = b->R[k * 3 + 0] * c[0] + b->R[k * 3 + 1] * c[1] + b->R[k * 3 + 2] * c[2];
    body_vel(b, dw, u);
}

/* ---------------------------------------------------------------------------
 * Public API (ctypes)
 * ------------------------------------------------------------------------- */
void ob_lattice(int *c /* [Q*3] */, double *w /* [Q] */, int *opp /* [Q] */) {
    lattice_setup();
    for (int i = 0; i < Q; ++i) {
        c[3 * i] = CX[i];
        c[3 * i + 1] = CY[i];
        c[3 * i + 2] = CZ[i];
        w[i] = W[i];
        opp[i] = OPP[i];
    }
}

void ob_feq(double rho, const double *u, double *out) {
    lattice_setup();
    for (int i = 0; i < Q; ++i) out[i] = feq(i, rho, u);
}

void ob_force(double rho, const double *u, const double *a, double *out) {
    lattice_setup();
    for (int i = 0; i < Q; ++i) out[i] = fterm(i, rho, u, a);
}

ob_state *ob_create(int nx, int ny, int nz, double tau, const double *a, double rho_g, double eps,
                    int periodic_mask, int recon_mode) {
    lattice_setup();
    if (nx <= 0 || ny <= 0 || nz <= 0) return NULL;
    ob_state *s = (ob_state *)calloc(1, sizeof(ob_state));
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->N = (long)nx * ny * nz;
    s->tau = tau;
    for (int k = 0; k < 3; ++k) s->a[k] = a[k];
    s->rho_g = rho_g;
    s->eps = eps;
    s->per[0] = (periodic_mask & 1) != 0;
    s->per[1] = (periodic_mask & 2) != 0;
    s->per[2] = (periodic_mask & 4) != 0;
    s->recon_mode = recon_mode;
    s->f = (double *)calloc((size_t)Q * s->N, sizeof(double));
    s->fn = (double *)calloc((size_t)Q * s->N, sizeof(double));
    s->type = (unsigned char *)calloc(s->N, 1);
    s->bid = (signed char *)malloc(s->N);
    memset(s->bid, -1, s->N);
    s->m = (double *)calloc(s->N, sizeof(double));
    s->phi = (double *)calloc(s->N, sizeof(double));
    s->mn = (double *)calloc(s->N, sizeof(double));
    s->phin = (double *)calloc(s->N, sizeof(double));
    s->nthreads = 1;
    s->stranded_rule = 1;
    if (!s->f || !s->fn || !s->type || !s->bid || !s->m || !s->phi || !s->mn || !s->phin) return NULL;
    return s;
}

void ob_destroy(ob_state *s) {
    if (!s) return;
    free(s->f);
    free(s->fn);
    free(s->type);
    free(s->bid);
    free(s->m);
    free(s->phi);
    free(s->mn);
    free(s->phin);
    free(s);
}

void ob_set_threads(ob_state *s, int n) { s->nthreads = n > 0 ? n : 1; }

/* Switch the stranded-interface rule of the conversions (on by default);
 * off keeps only the fill-level thresholds. */
void ob_set_stranded_rule(ob_state *s, int on) { s->stranded_rule = on != 0; }

/* Velocity of the lattice's non-periodic faces: moving no-slip walls
 * (Eq. noslip with u_w; the paper's channel is driven by its long sides). */
void ob_set_wall_velocity(ob_state *s, const double *u) {
    for (int k = 0; k < 3; ++k) s->wall_u[k] = u[k];
}

/* Surface tension sigma (Sec. 2.2, Laplace pressure): the gas pressure
 * that an interface cell rebuilds its populations with becomes
 * p_G + 2 sigma kappa, i.e. the gas density rho_G + 2 sigma kappa / cs^2. */
void ob_set_surface_tension(ob_state *s, double sigma) { s->sigma = sigma; }

long ob_num_cells(const ob_state *s) { return s->N; }

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), used as a counter-based
 * generator: one output per cell from state seed ^ index. */
static uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Basin initialisation.  Fill level phi0 = clamp(H - z, 0, 1) per cell layer;
 * phi0 = 1 -> liquid, 0 < phi0 < 1 -> interface, 0 -> gas; then every liquid
 * cell touching gas becomes interface (phi = 1), closing the interface layer
 * (Sec. 2.2).  Liquid and interface cells start in hydrostatic equilibrium
 * (Sec. 3.3 initialises the basin with a hydrostatic pressure gradient):
 * p = cs2 rho and dp/dz = rho a_z, linearised about the gas density:
 * rho = rho_G - 3 a_z (H - z_c), plus seeded uniform noise A(2U-1), and an
 * optional half-Poiseuille velocity u_x(z_c) = u_s z_c (2H - z_c)/H^2.
 * Populations are set to the equilibrium. */
void ob_init_basin(ob_state *s, double H, double u_surface, uint64_t seed, double noise_amp) {
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = IDX(s, x, y, z);
                double p = H - z;
                p = p < 0.0 ? 0.0 : (p > 1.0 ? 1.0 : p);
                s->phi[id] = p;
                s->type[id] = p >= 1.0 ? T_LIQ : (p > 0.0 ? T_IF : T_GAS);
                s->bid[id] = -1;
            }
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = IDX(s, x, y, z);
                if (s->type[id] != T_LIQ) continue;
                for (int i = 1; i < Q; ++i) {
                    long n;
                    if (nbr(s, x, y, z, CX[i], CY[i], CZ[i], &n) && s->type[n] == T_GAS) {
                        s->type[id] = T_IF; /* phi stays 1 */
                        break;
                    }
                }
            }
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = IDX(s, x, y, z);
                if (s->type[id] == T_GAS) {
                    for (int i = 0; i < Q; ++i) s->f[(long)i * s->N + id] = 0.0;
                    s->m[id] = 0.0;
                    s->phi[id] = 0.0;
                    continue;
                }
                double zc = z + 0.5;
                double rho = s->rho_g - 3.0 * s->a[2] * (H - zc);
                if (noise_amp != 0.0) {
                    uint64_t r = splitmix64(seed ^ (uint64_t)id);
                    double U = (double)(r >> 11) * (1.0 / 9007199254740992.0);
                    rho += noise_amp * (2.0 * U - 1.0);
                }
                double u[3] = {0, 0, 0};
                if (u_surface != 0.0 && H > 0.0) u[0] = u_surface * zc * (2.0 * H - zc) / (H * H);
                for (int i = 0; i < Q; ++i) s->f[(long)i * s->N + id] = feq(i, rho, u);
                s->m[id] = s->phi[id] * rho;
            }
    s->ledger = 0.0;
}

int ob_set_body(ob_state *s, int k, const double *half, const double *pos, const double *quat,
                const double *vel, const double *omega, double density, int fixed) {
    if (k < 0 || k >= OB_MAXB) return -1;
    ob_body *b = &s->b[k];
    double L[3] = {s->nx, s->ny, s->nz};
    for (int j = 0; j < 3; ++j) {
        b->half[j] = half[j];
        double p = pos[j];
        if (s->per[j]) p = p - L[j] * floor(p / L[j]);
        b->pos[j] = p;
        b->vel[j] = vel[j];
        b->omega[j] = omega[j];
    }
    for (int j = 0; j < 4; ++j) b->quat[j] = quat[j];
    b->density = density;
    b->fixed = fixed;
    quat_to_R(b->quat, b->R);
    b->active = 1;
    b->moved = 1;
    b->have_prev = 0;
    if (k + 1 > s->nb) s->nb = k + 1;
    return 0;
}

/* Shape of body k (OB_CUBOID, OB_SPHERE with radius half[0]); kept by later
 * ob_set_body calls. */
int ob_set_body_shape(ob_state *s, int k, int shape) {
    if (k < 0 || k >= OB_MAXB || (shape != OB_CUBOID && shape != OB_SPHERE)) return -1;
    s->b[k].shape = shape;
    s->b[k].moved = 1;
    return 0;
}

int ob_get_body(const ob_state *s, int k, double *pos, double *quat, double *vel, double *omega) {
    if (k < 0 || k >= s->nb || !s->b[k].active) return -1;
    const ob_body *b = &s->b[k];
    for (int j = 0; j < 3; ++j) {
        pos[j] = b->pos[j];
        vel[j] = b->vel[j];
        omega[j] = b->omega[j];
    }
    for (int j = 0; j < 4; ++j) quat[j] = b->quat[j];
    return 0;
}

/* ---------------------------------------------------------------------------
 * S1: body remap (Sec. 2.3 mapping, Sec. 2.4 conversions into and out of
 * obstacle).  Evaluated against the pre-remap state:
 *   cover    fluid cell whose centre is inside a body -> OBS(b); its liquid
 *            mass (LIQ: rho, IF: m) leaves the fluid (ledger).
 *   uncover  OBS cell no longer inside its body.  B(x) = neighbours that are
 *            neither obstacle before the remap nor covered by it (cells being
 *            uncovered themselves count as obstacle).
 *              no LIQ in B          -> GAS
 *              LIQ, no GAS in B     -> LIQ, rho = mean rho over B,
 *                                      f = f_eq(rho, u_w(closest surface point))
 *              LIQ and GAS in B     -> IF, rho = mean rho over non-gas members,
 *                                      phi = mean phi over IF members (if none:
 *                                      #LIQ/(#LIQ+#GAS)), f as above
 *   fix-up   a cell made LIQ that now touches a cell made GAS becomes IF
 *            (phi = mean phi over IF members of B, else 1).
 *   The new mass enters the fluid (ledger).
 * "Liquid" in the rules is read as the LIQ cell type only.
 * ------------------------------------------------------------------------- */
static void remap(ob_state *s) {
    int any = 0;
    for (int k = 0; k < s->nb; ++k)
        if (s->b[k].active && s->b[k].moved) any = 1;
    if (!any) return;
    long N = s->N;
    signed char *inb = (signed char *)malloc(N);
    unsigned char *rule = (unsigned char *)calloc(N, 1); /* 1 R1, 2 R2, 3 R3 */
    double *rbar = (double *)calloc(N, sizeof(double));
    double *pbar = (double *)calloc(N, sizeof(double));
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = IDX(s, x, y, z);
                inb[id] = -1;
                for (int k = 0; k < s->nb; ++k)
                    if (s->b[k].active && inside(s, &s->b[k], x, y, z)) {
                        inb[id] = (signed char)k;
                        break;
                    }
            }
    /* uncover: evaluate the rules from the pre-remap state */
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = IDX(s, x, y, z);
                if (s->type[id] != T_OBS || inb[id] >= 0) continue;
                int nL = 0, nG = 0, nI = 0;
                double rsum = 0.0, psum = 0.0;
                for (int i = 1; i < Q; ++i) {
                    long n;
                    if (!nbr(s, x, y, z, CX[i], CY[i], CZ[i], &n)) continue;
                    if (s->type[n] == T_OBS || inb[n] >= 0) continue;
                    if (s->type[n] == T_GAS) {
                        nG++;
                    } else {
                        rsum += cell_rho(s, s->f, n);
                        if (s->type[n] == T_LIQ) {
                            nL++;
                        } else {
                            nI++;
                            psum += s->phi[n];
                        }
                    }
                }
                if (nL == 0) {
                    rule[id] = 1;
                } else if (nG == 0) {
                    rule[id] = 2;
                    rbar[id] = rsum / (nL + nI);
                    pbar[id] = nI > 0 ? psum / nI : 1.0;
                } else {
                    rule[id] = 3;
                    rbar[id] = rsum / (nL + nI);
                    pbar[id] = nI > 0 ? psum / nI : (double)nL / (double)(nL + nG);
                }
            }
    /* fix-up: new LIQ next to new GAS -> IF */
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = IDX(s, x, y, z);
                if (rule[id] != 2) continue;
                for (int i = 1; i < Q; ++i) {
                    long n;
                    if (nbr(s, x, y, z, CX[i], CY[i], CZ[i], &n) && rule[n] == 1) {
                        rule[id] = 4; /* R2 turned interface */
                        break;
                    }
                }
            }
    /* commit (cover, uncover) in index order */
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = IDX(s, x, y, z);
                int t = s->type[id];
                if (t != T_OBS && inb[id] >= 0) {
                    if (t == T_LIQ) s->ledger -= cell_rho(s, s->f, id);
                    else if (t == T_IF) s->ledger -= s->m[id];
                    s->type[id] = T_OBS;
                    s->bid[id] = inb[id];
                    s->m[id] = 0.0;
                    s->phi[id] = 0.0;
                } else if (t == T_OBS && inb[id] >= 0) {
                    s->bid[id] = inb[id];
                } else if (t == T_OBS) {
                    int r = rule[id];
                    const ob_body *b = &s->b[(int)s->bid[id]];
                    s->bid[id] = -1;
                    if (r == 1) {
                        s->type[id] = T_GAS;
                        s->m[id] = 0.0;
                        s->phi[id] = 0.0;
                        for (int i = 0; i < Q; ++i) s->f[(long)i * N + id] = 0.0;
                        continue;
                    }
                    double uw[3];
                    closest_surface_vel(s, b, x, y, z, uw);
                    for (int i = 0; i < Q; ++i) s->f[(long)i * N + id] = feq(i, rbar[id], uw);
                    if (r == 2) {
                        s->type[id] = T_LIQ;
                        s->phi[id] = 1.0;
                        s->m[id] = rbar[id];
                    } else {
                        s->type[id] = T_IF;
                        s->phi[id] = pbar[id];
                        s->m[id] = pbar[id] * rbar[id];
                    }
                    s->ledger += s->m[id];
                }
            }
    for (int k = 0; k < s->nb; ++k) s->b[k].moved = 0;
    free(inb);
    free(rule);
    free(rbar);
    free(pbar);
}

/* ---------------------------------------------------------------------------
 * S3: momentum exchange on the state at time t (Eqs. momentumexchange,
 * momentuminterface, netforce, torque).  For every non-obstacle cell x and
 * link i >= 1 whose source x - c_i is an obstacle cell of body b:
 *   phi^ = 1 (LIQ), phi_x (IF), 0 (GAS)
 *   dj   = 2 c_i [ phi^ f_ibar(x) + (1 - phi^) f_eq,i(rho_G, 0)
 *                  + phi^ (1/cs2) w_i rho_x (c_i . u_w) ]
 * (the rho factor missing from the printed equations is the one of
 * Eq. noslip, from which the exchange is derived).  dj is the momentum the
 * fluid gains, so the body receives F -= dj, T -= (x_c - o) x dj.  u_w is the
 * body velocity at the link midpoint x_c - c_i/2.
 * ------------------------------------------------------------------------- */
static void momentum_exchange(ob_state *s) {
    for (int k = 0; k < s->nb; ++k)
        for (int j = 0; j < 3; ++j) s->b[k].force[j] = s->b[k].torque[j] = 0.0;
    long N = s->N;
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = IDX(s, x, y, z);
                int t = s->type[id];
                if (t == T_OBS) continue;
                double ph = t == T_LIQ ? 1.0 : (t == T_IF ? s->phi[id] : 0.0);
                double rho = t == T_GAS ? 0.0 : cell_rho(s, s->f, id);
                double xc[3] = {x + 0.5, y + 0.5, z + 0.5};
                for (int i = 1; i < Q; ++i) {
                    long src;
                    if (!nbr(s, x, y, z, -CX[i], -CY[i], -CZ[i], &src)) continue;
                    if (s->type[src] != T_OBS) continue;
                    ob_body *b = &s->b[(int)s->bid[src]];
                    double pm[3] = {xc[0] - 0.5 * CX[i], xc[1] - 0.5 * CY[i], xc[2] - 0.5 * CZ[i]};
                    double d[3], uw[3];
                    rel(s, b, pm, d);
                    body_vel(b, d, uw);
                    double cu = CX[i] * uw[0] + CY[i] * uw[1] + CZ[i] * uw[2];
                    double fib = t == T_GAS ? 0.0 : s->f[(long)OPP[i] * N + id];
                    double zero[3] = {0, 0, 0};
                    double amp = 2.0 * (ph * fib + (1.0 - ph) * feq(i, s->rho_g, zero) + ph * W[i] * rho * cu / CS2);
                    double dj[3] = {amp * CX[i], amp * CY[i], amp * CZ[i]};
                    double r[3];
                    rel(s, b, xc, r);
                    b->force[0] -= dj[0];
                    b->force[1] -= dj[1];
                    b->force[2] -= dj[2];
                    b->torque[0] -= r[1] * dj[2] - r[2] * dj[1];
                    b->torque[1] -= r[2] * dj[0] - r[0] * dj[2];
                    b->torque[2] -= r[0] * dj[1] - r[1] * dj[0];
                }
            }
}

/* Free-surface normal n = -grad(phi) by central differences over the six
 * axis neighbours (Sec. 2.2 only says it is approximated from the fill-level
 * gradient).  Neighbour fill: LIQ 1, GAS 0, IF phi, obstacle/wall: phi_x.
 * It points from the liquid towards the gas. */
static double nb_fill(const ob_state *s, int x, int y, int z, int dx, int dy, int dz, double own) {
    long n;
    if (!nbr(s, x, y, z, dx, dy, dz, &n)) return own;
    switch (s->type[n]) {
    case T_LIQ: return 1.0;
    case T_GAS: return 0.0;
    case T_IF: return s->phi[n];
    default: return own;
    }
}

/* Fill of a cell as the normal sees it: LIQ 1, GAS 0, IF phi. */
static double own_fill(const ob_state *s, long id) {
    switch (s->type[id]) {
    case T_LIQ: return 1.0;
    case T_IF: return s->phi[id];
    default: return 0.0;
    }
}

/* Unit normal at a fluid cell: the central-difference normal of the
 * reconstruction, divided by its length; zero where the fill is flat. */
static void unit_normal(const ob_state *s, int x, int y, int z, double n[3]) {
    double o = own_fill(s, IDX(s, x, y, z));
    n[0] = 0.5 * (nb_fill(s, x, y, z, -1, 0, 0, o) - nb_fill(s, x, y, z, 1, 0, 0, o));
    n[1] = 0.5 * (nb_fill(s, x, y, z, 0, -1, 0, o) - nb_fill(s, x, y, z, 0, 1, 0, o));
    n[2] = 0.5 * (nb_fill(s, x, y, z, 0, 0, -1, o) - nb_fill(s, x, y, z, 0, 0, 1, o));
    double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (len > 0.0)
        for (int k = 0; k < 3; ++k) n[k] /= len;
}

/* Mean curvature of the free surface at interface cell (x,y,z), the second
 * step after the normals (Sec. 2.2 leaves the stencil open; it names Pohl's
 * approach of deriving kappa from the normals of a neighbourhood):
 *   kappa = 1/2 div(n_hat),
 * the divergence by central differences of the unit normals of the six axis
 * neighbours.  A neighbour that is an obstacle or lies beyond a wall lends
 * the cell's own normal.  With n pointing from the liquid to the gas, a
 * liquid sphere of radius R has kappa = 1/R and a gas bubble -1/R. */
static double curvature(const ob_state *s, int x, int y, int z) {
    double nx[3];
    unit_normal(s, x, y, z, nx);
    double div = 0.0;
    for (int a = 0; a < 3; ++a) {
        double side[2];
        for (int k = 0; k < 2; ++k) {
            int d[3] = {0, 0, 0};
            d[a] = k == 0 ? 1 : -1;
            long n;
            side[k] = nx[a];
            if (nbr(s, x, y, z, d[0], d[1], d[2], &n) && s->type[n] != T_OBS) {
                double nn[3];
                int q[3] = {x + d[0], y + d[1], z + d[2]};
                int dim[3] = {s->nx, s->ny, s->nz};
                for (int c = 0; c < 3; ++c) q[c] = (q[c] + dim[c]) % dim[c];
                unit_normal(s, q[0], q[1], q[2], nn);
                side[k] = nn[a];
            }
        }
        div += 0.5 * (side[0] - side[1]);
    }
    return 0.5 * div;
}

/* kappa of every interface cell of the current state (0 elsewhere). */
void ob_curvature(const ob_state *s, double *out) {
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = IDX(s, x, y, z);
                out[id] = s->type[id] == T_IF ? curvature(s, x, y, z) : 0.0;
            }
}

/* ---------------------------------------------------------------------------
 * S2: stream + boundaries + collide for one LIQ/IF cell (Sec. 2.1-2.4).
 * Pull form of Eq. stream: f'_i(x) comes from s = x - c_i.
 *   s wall / obstacle : Eq. noslip  f'_i = f_ibar(x) + (2/cs2) w_i rho_x c_i.u_w
 *                       (u_w: the body's velocity at the link midpoint, or
 *                       the wall velocity for a source beyond a face)
 *   s gas             : Eq. reconstruct with the partner read as this cell's
 *                       own outgoing f_ibar(x,t):
 *                       f'_i = f_eq,i(rho_G,u_x) + f_eq,ibar(rho_G,u_x) - f_ibar(x)
 *   s liquid/interface: f'_i = f_i(s); in interface cells the populations
 *                       arriving from the gas side (c_i.n < -tol) are also
 *                       reconstructed (recon_mode 0); recon_mode 2 uses the
 *                       printed "c_i.n <= 0" (c_i.n <= tol) for i >= 1;
 *                       recon_mode 1 only reconstructs gas-sourced links.
 *                       tol = NORMAL_TOL * |n|_1.
 * rho_x, u_x are the moments of the cell's own f(x,t).
 * Interface mass (Sec. 2.2 Delta m, with f_i(x) outgoing, f_ibar(x+c_i)
 * incoming): dm = sum_i { LIQ: f_ibar(y)-f_i(x); IF: (phi_x+phi_y)/2 (...);
 * otherwise 0 }.
 * Collide: f_i = f'_i - (f'_i - f_eq,i(rho,u))/tau + F_i, rho and u the
 * moments of f'.  (Eq. lbgk is printed with "+ f_eq" and "- F_i"; the collide
 * equation below it has the correct "-(f' - f_eq)"; the force enters with "+"
 * for a = gravity pointing down, so that the liquid gains momentum rho*a.)
 * Interface cells: m += dm, phi = m / rho.
 * ------------------------------------------------------------------------- */
static void sweep_cell(ob_state *s, int x, int y, int z) {
    long N = s->N;
    long id = IDX(s, x, y, z);
    int t = s->type[id];
    if (t != T_LIQ && t != T_IF) {
        for (int i = 0; i < Q; ++i) s->fn[(long)i * N + id] = s->f[(long)i * N + id];
        s->mn[id] = s->m[id];
        s->phin[id] = s->phi[id];
        return;
    }
    double fx[Q], fp[Q];
    for (int i = 0; i < Q; ++i) fx[i] = s->f[(long)i * N + id];
    double rhox = 0.0;
    for (int i = 0; i < Q; ++i) rhox += fx[i];
    double ux[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        ux[0] += CX[i] * fx[i];
        ux[1] += CY[i] * fx[i];
        ux[2] += CZ[i] * fx[i];
    }
    for (int k = 0; k < 3; ++k) ux[k] /= rhox;
    double nrm[3] = {0, 0, 0};
    double phx = s->phi[id];
    if (t == T_IF) {
        nrm[0] = 0.5 * (nb_fill(s, x, y, z, -1, 0, 0, phx) - nb_fill(s, x, y, z, 1, 0, 0, phx));
        nrm[1] = 0.5 * (nb_fill(s, x, y, z, 0, -1, 0, phx) - nb_fill(s, x, y, z, 0, 1, 0, phx));
        nrm[2] = 0.5 * (nb_fill(s, x, y, z, 0, 0, -1, phx) - nb_fill(s, x, y, z, 0, 0, 1, phx));
    }
    /* Links within NORMAL_TOL * |n|_1 of tangential count as tangential, so
     * that round-off in the fill levels (exactly planar surfaces give exactly
     * zero tangential components only in exact arithmetic) does not decide
     * which links are rebuilt. */
    double nthr = NORMAL_TOL * ((fabs(nrm[0]) + fabs(nrm[1])) + fabs(nrm[2]));
    /* gas density of the reconstruction, raised by the Laplace pressure */
    double rg = s->rho_g;
    if (t == T_IF && s->sigma != 0.0) rg += 2.0 * s->sigma * curvature(s, x, y, z) / CS2;
    double xc[3] = {x + 0.5, y + 0.5, z + 0.5};
    fp[0] = fx[0];
    for (int i = 1; i < Q; ++i) {
        long src;
        int ib = OPP[i];
        int inb = nbr(s, x, y, z, -CX[i], -CY[i], -CZ[i], &src);
        int st = inb ? s->type[src] : T_OBS;
        if (st == T_OBS) {
            double uw[3] = {s->wall_u[0], s->wall_u[1], s->wall_u[2]};
            if (inb) {
                const ob_body *b = &s->b[(int)s->bid[src]];
                double pm[3] = {xc[0] - 0.5 * CX[i], xc[1] - 0.5 * CY[i], xc[2] - 0.5 * CZ[i]};
                double d[3];
                rel(s, b, pm, d);
                body_vel(b, d, uw);
            }
            double cu = CX[i] * uw[0] + CY[i] * uw[1] + CZ[i] * uw[2];
            fp[i] = fx[ib] + (2.0 / CS2) * W[i] * cu * rhox;
            continue;
        }
        int recon = 0;
        if (st == T_GAS) {
            recon = 1;
        } else if (t == T_IF && s->recon_mode != 1) {
            double cn = CX[i] * nrm[0] + CY[i] * nrm[1] + CZ[i] * nrm[2];
            if (s->recon_mode == 0 ? (cn < -nthr) : (cn <= nthr)) recon = 1;
        }
        if (recon) fp[i] = feq(i, rg, ux) + feq(ib, rg, ux) - fx[ib];
        else fp[i] = s->f[(long)i * N + src];
    }
    /* mass exchange (interface cells), on the state at t */
    double dm = 0.0;
    if (t == T_IF) {
        for (int i = 1; i < Q; ++i) {
            long n;
            if (!nbr(s, x, y, z, CX[i], CY[i], CZ[i], &n)) continue;
            int nt = s->type[n];
            double ex = s->f[(long)OPP[i] * N + n] - fx[i];
            if (nt == T_LIQ) dm += ex;
            else if (nt == T_IF) dm += 0.5 * (phx + s->phi[n]) * ex;
        }
    }
    double rho = 0.0, u[3] = {0, 0, 0};
    for (int i = 0; i < Q; ++i) {
        rho += fp[i];
        u[0] += CX[i] * fp[i];
        u[1] += CY[i] * fp[i];
        u[2] += CZ[i] * fp[i];
    }
    for (int k = 0; k < 3; ++k) u[k] /= rho;
    for (int i = 0; i < Q; ++i)
        s->fn[(long)i * N + id] = fp[i] - (fp[i] - feq(i, rho, u)) / s->tau + fterm(i, rho, u, s->a);
    if (t == T_IF) {
        double m = s->m[id] + dm;
        s->mn[id] = m;
        s->phin[id] = m / rho;
    } else {
        s->mn[id] = s->m[id];
        s->phin[id] = s->phi[id];
    }
}

static void sweep(ob_state *s) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(s->nthreads)
#endif
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) sweep_cell(s, x, y, z);
    double *t;
    t = s->f; s->f = s->fn; s->fn = t;
    t = s->m; s->m = s->mn; s->mn = t;
    t = s->phi; s->phi = s->phin; s->phin = t;
}

/* ---------------------------------------------------------------------------
 * S4: free-surface conversions on the state at t+1 (Sec. 2.2; the paper gives
 * the thresholds -eps / 1+eps, forbids direct gas<->liquid transitions and
 * initialises new interface cells at phi 0 or 1; the rest is this reading):
 *  1. F = IF with phi >= 1+eps (filled), E = IF with phi <= -eps (emptied),
 *     and also E = IF not in F that is stranded: no liquid cell among its 18
 *     neighbours, and no interface neighbour that has one (a droplet or film
 *     of interface cells cut off from the liquid; the outer cells of a
 *     two-cell-thick curved surface reach liquid through an interface
 *     neighbour and are not stranded).  The paper gives no rule for such
 *     cells; without one an isolated interface cell keeps rebuilding its
 *     gas-side links from its own populations and can reach a negative
 *     density.
 *  2. Filling wins: an E cell touching an F cell stays interface.
 *  3. GAS neighbours of F become IF: f = f_eq(mean rho, mean u) over the
 *     neighbours that were LIQ/IF and are not emptying; m = 0.
 *  4. LIQ neighbours of (remaining) E become IF with m = rho.
 *  5. F -> LIQ with excess m - rho; E -> GAS with excess m.
 *  6. each converted cell shares its excess equally among its neighbours that
 *     are IF after 3-5; receivers add their shares in link order i = 1..18;
 *     with no receiver the excess leaves the fluid (ledger).
 *  7. phi = m / rho for every interface cell whose mass changed.
 * ------------------------------------------------------------------------- */
enum { C_NONE = 0, C_FILL = 1, C_EMPTY = 2, C_NEWG = 3, C_NEWL = 4 };

static void convert(ob_state *s) {
    long N = s->N;
    unsigned char *c = (unsigned char *)calloc(N, 1);
    double *ex = (double *)calloc(N, sizeof(double));
    double *sh = (double *)calloc(N, sizeof(double));
    long cnt[4] = {0, 0, 0, 0};
    /* interface cells with a liquid neighbour */
    unsigned char *lnb = (unsigned char *)calloc(N, 1);
    for (long id = 0; id < N; ++id) {
        if (s->type[id] != T_IF) continue;
        int x, y, z;
        coords(s, id, &x, &y, &z);
        for (int i = 1; i < Q && !lnb[id]; ++i) {
            long n;
            if (nbr(s, x, y, z, CX[i], CY[i], CZ[i], &n) && s->type[n] == T_LIQ) lnb[id] = 1;
        }
    }
    for (long id = 0; id < N; ++id) {
        if (s->type[id] != T_IF) continue;
        if (s->phi[id] >= 1.0 + s->eps) c[id] = C_FILL;
        else if (s->phi[id] <= -s->eps) c[id] = C_EMPTY;
        else if (s->stranded_rule && !lnb[id]) {
            int x, y, z, near = 0;
            coords(s, id, &x, &y, &z);
            for (int i = 1; i < Q && !near; ++i) {
                long n;
                if (nbr(s, x, y, z, CX[i], CY[i], CZ[i], &n) && s->type[n] == T_IF && lnb[n]) near = 1;
            }
            if (!near) c[id] = C_EMPTY;
        }
    }
    free(lnb);
    /* filling wins */
    unsigned char *keep = (unsigned char *)calloc(N, 1);
    for (long id = 0; id < N; ++id) {
        if (c[id] != C_EMPTY) continue;
        int x, y, z;
        coords(s, id, &x, &y, &z);
        for (int i = 1; i < Q; ++i) {
            long n;
            if (nbr(s, x, y, z, CX[i], CY[i], CZ[i], &n) && c[n] == C_FILL) {
                keep[id] = 1;
                break;
            }
        }
    }
    for (long id = 0; id < N; ++id)
        if (keep[id]) c[id] = C_NONE;
    free(keep);
    /* neighbours of F (gas) and E (liquid) */
    for (long id = 0; id < N; ++id) {
        if (c[id] != C_FILL && c[id] != C_EMPTY) continue;
        int x, y, z;
        coords(s, id, &x, &y, &z);
        for (int i = 1; i < Q; ++i) {
            long n;
            if (!nbr(s, x, y, z, CX[i], CY[i], CZ[i], &n)) continue;
            if (c[id] == C_FILL && s->type[n] == T_GAS) c[n] = C_NEWG;
            if (c[id] == C_EMPTY && s->type[n] == T_LIQ) c[n] = C_NEWL;
        }
    }
    /* initialise new interface cells from gas */
    for (long id = 0; id < N; ++id) {
        if (c[id] != C_NEWG) continue;
        int x, y, z;
        coords(s, id, &x, &y, &z);
        int ns = 0;
        double rs = 0.0, us[3] = {0, 0, 0};
        for (int i = 1; i < Q; ++i) {
            long n;
            if (!nbr(s, x, y, z, CX[i], CY[i], CZ[i], &n)) continue;
            int nt = s->type[n];
            if ((nt != T_LIQ && nt != T_IF) || c[n] == C_EMPTY) continue;
            double r = cell_rho(s, s->f, n), u[3];
            cell_u(s, s->f, n, r, u);
            rs += r;
            us[0] += u[0];
            us[1] += u[1];
            us[2] += u[2];
            ns++;
        }
        double rb = rs / ns, ub[3] = {us[0] / ns, us[1] / ns, us[2] / ns};
        for (int i = 0; i < Q; ++i) s->fn[(long)i * N + id] = feq(i, rb, ub);
    }
    for (long id = 0; id < N; ++id) {
        if (c[id] != C_NEWG) continue;
        for (int i = 0; i < Q; ++i) s->f[(long)i * N + id] = s->fn[(long)i * N + id];
    }
    /* type changes and excess */
    for (long id = 0; id < N; ++id) {
        switch (c[id]) {
        case C_NEWG:
            s->type[id] = T_IF;
            s->m[id] = 0.0;
            s->phi[id] = 0.0;
            cnt[2]++;
            break;
        case C_NEWL: {
            double r = cell_rho(s, s->f, id);
            s->type[id] = T_IF;
            s->m[id] = r;
            s->phi[id] = 1.0;
            cnt[3]++;
            break;
        }
        case C_FILL: {
            double r = cell_rho(s, s->f, id);
            ex[id] = s->m[id] - r;
            s->type[id] = T_LIQ;
            s->m[id] = r;
            s->phi[id] = 1.0;
            cnt[0]++;
            break;
        }
        case C_EMPTY:
            ex[id] = s->m[id];
            s->type[id] = T_GAS;
            s->m[id] = 0.0;
            s->phi[id] = 0.0;
            for (int i = 0; i < Q; ++i) s->f[(long)i * N + id] = 0.0;
            cnt[1]++;
            break;
        default: break;
        }
    }
    /* shares */
    for (long id = 0; id < N; ++id) {
        if (c[id] != C_FILL && c[id] != C_EMPTY) continue;
        int x, y, z;
        coords(s, id, &x, &y, &z);
        int nr = 0;
        for (int i = 1; i < Q; ++i) {
            long n;
            if (nbr(s, x, y, z, CX[i], CY[i], CZ[i], &n) && s->type[n] == T_IF) nr++;
        }
        if (nr > 0) sh[id] = ex[id] / nr;
        else s->ledger -= ex[id];
    }
    /* receivers, pull form in link order (an IF neighbour of a converted cell
     * is one of its receivers, so that cell's share is defined) */
    for (long id = 0; id < N; ++id) {
        if (s->type[id] != T_IF) continue;
        int x, y, z;
        coords(s, id, &x, &y, &z);
        int got = 0;
        double m = s->m[id];
        for (int i = 1; i < Q; ++i) {
            long n;
            if (!nbr(s, x, y, z, CX[i], CY[i], CZ[i], &n)) continue;
            if (c[n] == C_FILL || c[n] == C_EMPTY) {
                m += sh[n];
                got = 1;
            }
        }
        if (got) {
            s->m[id] = m;
            s->phi[id] = m / cell_rho(s, s->f, id);
        }
    }
    for (int k = 0; k < 4; ++k) s->last_conv[k] = cnt[k];
    free(c);
    free(ex);
    free(sh);
}

/* One time step: remap (if a body moved) -> momentum exchange and sweep on the
 * state at t -> conversions on t+1.  phase_mask selects parts (1 remap,
 * 2 sweep + momentum exchange, 4 conversions) for phase-isolated tests. */
int ob_step(ob_state *s, int nsteps, int phase_mask) {
    for (int n = 0; n < nsteps; ++n) {
        if (phase_mask & 1) remap(s);
        if (phase_mask & 2) {
            momentum_exchange(s);
            sweep(s);
        }
        if (phase_mask & 4) convert(s);
    }
    return 0;
}

/* Steps with free bodies: after every full step each body with a non-zero
 * DOF mask is advanced by the host update below, fed with the mean of this
 * and the previous step's fluid force and torque (the first step uses its own
 * force), and set again for the next step's remap. */
int ob_integrate_body(const double *half, const double *pos, const double *quat, const double *vel,
                      const double *omega, double density, const double *F, const double *T,
                      const double *a, int dof_mask, double *pos_out, double *quat_out, double *vel_out,
                      double *omega_out, int shape);

int ob_step_coupled(ob_state *s, int nsteps, const int *dof_masks) {
    for (int n = 0; n < nsteps; ++n) {
        ob_step(s, 1, 7);
        for (int k = 0; k < s->nb; ++k) {
            ob_body *b = &s->b[k];
            if (!b->active || !dof_masks[k]) continue;
            double F[3], T[3];
            for (int j = 0; j < 3; ++j) {
                F[j] = b->have_prev ? 0.5 * (b->force[j] + b->fprev[j]) : b->force[j];
                T[j] = b->have_prev ? 0.5 * (b->torque[j] + b->tprev[j]) : b->torque[j];
                b->fprev[j] = b->force[j];
                b->tprev[j] = b->torque[j];
            }
            b->have_prev = 1;
            double p[3], q[4], v[3], w[3];
            if (ob_integrate_body(b->half, b->pos, b->quat, b->vel, b->omega, b->density, F, T, s->a, dof_masks[k], p,
                                  q, v, w, b->shape))
                return -1;
            double fp[3] = {b->fprev[0], b->fprev[1], b->fprev[2]}, tp[3] = {b->tprev[0], b->tprev[1], b->tprev[2]};
            ob_set_body(s, k, b->half, p, q, v, w, b->density, b->fixed);
            for (int j = 0; j < 3; ++j) {
                b->fprev[j] = fp[j];
                b->tprev[j] = tp[j];
            }
            b->have_prev = 1;
        }
    }
    return 0;
}

void ob_last_conversions(const ob_state *s, long *out4) {
    for (int k = 0; k < 4; ++k) out4[k] = s->last_conv[k];
}

int ob_body_forces(const ob_state *s, int k, double *F, double *T) {
    if (k < 0 || k >= s->nb || !s->b[k].active) return -1;
    for (int j = 0; j < 3; ++j) {
        F[j] = s->b[k].force[j];
        T[j] = s->b[k].torque[j];
    }
    return 0;
}

/* Sum over LIQ cells of rho plus sum over IF cells of m; and the ledger. */
double ob_mass_total(const ob_state *s, double *ledger) {
    double M = 0.0;
    for (long id = 0; id < s->N; ++id) {
        if (s->type[id] == T_LIQ) M += cell_rho(s, s->f, id);
        else if (s->type[id] == T_IF) M += s->m[id];
    }
    if (ledger) *ledger = s->ledger;
    return M;
}

/* Number of LIQ cells with a GAS neighbour: the closed interface layer of
 * Sec. 2.2 requires zero. */
long ob_liq_gas_contacts(const ob_state *s) {
    long c = 0;
    for (int z = 0; z < s->nz; ++z)
        for (int y = 0; y < s->ny; ++y)
            for (int x = 0; x < s->nx; ++x) {
                long id = IDX(s, x, y, z);
                if (s->type[id] != T_LIQ) continue;
                for (int i = 1; i < Q; ++i) {
                    long n;
                    if (nbr(s, x, y, z, CX[i], CY[i], CZ[i], &n) && s->type[n] == T_GAS) {
                        c++;
                        break;
                    }
                }
            }
    return c;
}

/* Field access.  Flags use one byte per cell: bits 0-1 cell type (0 gas,
 * 1 liquid, 2 interface, 3 obstacle), bits 2-5 owning body for obstacles. */
void ob_get_f(const ob_state *s, double *out) { memcpy(out, s->f, sizeof(double) * Q * s->N); }
void ob_set_f(ob_state *s, const double *in) { memcpy(s->f, in, sizeof(double) * Q * s->N); }
void ob_get_mass(const ob_state *s, double *out) { memcpy(out, s->m, sizeof(double) * s->N); }
void ob_set_mass(ob_state *s, const double *in) { memcpy(s->m, in, sizeof(double) * s->N); }
void ob_get_phi(const ob_state *s, double *out) { memcpy(out, s->phi, sizeof(double) * s->N); }
void ob_set_phi(ob_state *s, const double *in) { memcpy(s->phi, in, sizeof(double) * s->N); }
void ob_get_flags(const ob_state *s, unsigned char *out) {
    for (long id = 0; id < s->N; ++id)
        out[id] = (unsigned char)(s->type[id] | (s->type[id] == T_OBS ? ((s->bid[id] & 15) << 2) : 0));
}
void ob_set_flags(ob_state *s, const unsigned char *in) {
    for (long id = 0; id < s->N; ++id) {
        s->type[id] = in[id] & 3;
        s->bid[id] = s->type[id] == T_OBS ? (signed char)((in[id] >> 2) & 15) : -1;
    }
}
void ob_set_ledger(ob_state *s, double v) { s->ledger = v; }
/* After injecting flags that already hold a body's mapping, mark it mapped. */
void ob_mark_mapped(ob_state *s) {
    for (int k = 0; k < s->nb; ++k) s->b[k].moved = 0;
}

/* ---------------------------------------------------------------------------
 * Rigid-body update (the paper couples to an external rigid-body engine; here
 * a plain semi-implicit Euler step with dt = 1, body mass from the continuous
 * volume, M_b = rho_s * 8 h_x h_y h_z, cuboid inertia about the centre):
 *   V     += (F + M_b a) / M_b          (translational DOFs in dof_mask bits 0-2)
 *   Omega += I_SS^-1 T_S                (rotational DOFs S in bits 3-5; I the
 *                                        world-frame inertia, no gyroscopic term)
 *   o     += V ;  q <- rot(|Omega|, Omega/|Omega|) * q, renormalised.
 * ------------------------------------------------------------------------- */
int ob_integrate_body(const double *half, const double *pos, const double *quat, const double *vel,
                      const double *omega, double density, const double *F, const double *T,
                      const double *a, int dof_mask, double *pos_out, double *quat_out, double *vel_out,
                      double *omega_out, int shape) {
    /* mass of the body's own volume: cuboid 8 h0 h1 h2, sphere 4/3 pi r^3 */
    const double r3 = half[0] * half[0] * half[0];
    double M = shape == OB_SPHERE ? density * (4.0 / 3.0) * OB_PI * r3 : density * 8.0 * half[0] * half[1] * half[2];
    if (!(M > 0.0)) return -1;
    double v[3], w[3];
    for (int k = 0; k < 3; ++k) {
        v[k] = vel[k];
        w[k] = omega[k];
        if (dof_mask & (1 << k)) v[k] = vel[k] + (F[k] + M * a[k]) / M;
    }
    double R[9];
    quat_to_R(quat, R);
    /* principal moments: cuboid M/3 (h_j^2 + h_k^2), sphere 2/5 M r^2 */
    double Ib[3] = {M / 3.0 * (half[1] * half[1] + half[2] * half[2]),
                    M / 3.0 * (half[0] * half[0] + half[2] * half[2]),
                    M / 3.0 * (half[0] * half[0] + half[1] * half[1])};
    if (shape == OB_SPHERE)
        for (int k = 0; k < 3; ++k) Ib[k] = 0.4 * M * half[0] * half[0];
    double I[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += R[r * 3 + k] * Ib[k] * R[c * 3 + k];
            I[r * 3 + c] = acc;
        }
    int S[3], ns = 0;
    for (int k = 0; k < 3; ++k)
        if (dof_mask & (8 << k)) S[ns++] = k;
    if (ns > 0) {
        /* solve I_SS dw = T_S by Gaussian elimination (ns <= 3) */
        double A[3][4];
        for (int r = 0; r < ns; ++r) {
            for (int c = 0; c < ns; ++c) A[r][c] = I[S[r] * 3 + S[c]];
            A[r][ns] = T[S[r]];
        }
        for (int p = 0; p < ns; ++p) {
            int piv = p;
            for (int r = p + 1; r < ns; ++r)
                if (fabs(A[r][p]) > fabs(A[piv][p])) piv = r;
            if (piv != p)
                for (int c = 0; c <= ns; ++c) {
                    double tmp = A[p][c];
                    A[p][c] = A[piv][c];
                    A[piv][c] = tmp;
                }
            for (int r = p + 1; r < ns; ++r) {
                double fct = A[r][p] / A[p][p];
                for (int c = p; c <= ns; ++c) A[r][c] -= fct * A[p][c];
            }
        }
        double dw[3];
        for (int r = ns - 1; r >= 0; --r) {
            double acc = A[r][ns];
            for (int c = r + 1; c < ns; ++c) acc -= A[r][c] * dw[c];
            dw[r] = acc / A[r][r];
        }
        for (int r = 0; r < ns; ++r) w[S[r]] = omega[S[r]] + dw[r];
    }
    for (int k = 0; k < 3; ++k) {
        vel_out[k] = v[k];
        omega_out[k] = w[k];
        pos_out[k] = pos[k] + v[k];
    }
    double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double q[4] = {quat[0], quat[1], quat[2], quat[3]};
    if (th > 0.0) {
        double sh = sin(0.5 * th) / th, dq[4] = {cos(0.5 * th), sh * w[0], sh * w[1], sh * w[2]};
        double r[4];
        r[0] = dq[0] * q[0] - dq[1] * q[1] - dq[2] * q[2] - dq[3] * q[3];
        r[1] = dq[0] * q[1] + dq[1] * q[0] + dq[2] * q[3] - dq[3] * q[2];
        r[2] = dq[0] * q[2] - dq[1] * q[3] + dq[2] * q[0] + dq[3] * q[1];
        r[3] = dq[0] * q[3] + dq[1] * q[2] - dq[2] * q[1] + dq[3] * q[0];
        double nn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
        for (int k = 0; k < 4; ++k) q[k] = r[k] / nn;
    }
    for (int k = 0; k < 4; ++k) quat_out[k] = q[k];
    return 0;
}
