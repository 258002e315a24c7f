/*
 * tete_oracle.c -- plain, slow, FP64 CPU oracle for the explicit TE/TM scheme
 * of Dohlus & Zagorodnov, "Explicit TE/TM scheme for particle beam simulations".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or constant generator with
 * the HIP implementation.
 *
 * What it computes (all in FP64, plain loops, in the order the paper gives):
 *   - the Cartesian FIT grid doublet of Sec. 2, eq. (4): edge voltages e^, facet
 *     fluxes via diagonal M_eps^-1 (kappa) and M_mu^-1 (mu); PEC edges have
 *     kappa = 0, so n x E = 0 of eq. (1) holds on them for all time;
 *   - one time step of the explicit TE/TM scheme (23) written as the ten
 *     Yee-form sub-updates of Sec. 4.2 (TM-like group u = (h_x, h_y, e_z) first,
 *     then the TE-like group v = (e_x, e_y, h_z)), alpha = dtau/2 as in (17);
 *   - the discrete energy W^{n,e} = 1/2 <Q^e y^n, y^n> of Sec. 4.4, expanded in
 *     FIT variables;
 *   - the conserved charges of Sec. 4.5 (charge conservation), eqs. (34), (35);
 *   - a rigid Gaussian bunch moving at v = c on a node line, with its current
 *     injected so that the charge moves one cell per step at dtau = dz (Fig. 1);
 *   - the longitudinal wake potential W_par(s) of Sec. 5 by the grid quadrature
 *     of the time-staggered e_z on the bunch line;
 *   - for comparison, one step of Yee's E/M scheme (7) of Sec. 3, its leapfrog
 *     invariant and its node charges (dual divergence).
 *
 * Readings of the paper used here (the text is ambiguous or garbled at these
 * places; each reading is pinned by a CPU test):
 *   - P^* is the matrix transpose, so the operators T_i of (15) are skew;
 *   - physical sign of the current: d/dtau d = C^T h - j (eq. (4)); the
 *     scaled forms print "+j" in places;
 *   - L_T U_T = I - alpha T_i - alpha^2 R_i, hence Q^e = B^e - alpha A =
 *     [[I - a^2 R_0, a L], [a L^T, I - a^2 R_1]] and the charges carry
 *     (I - alpha^2 r_i);
 *   - staircase PEC: a cell is PEC or not; an edge is PEC if any of its up to
 *     four adjacent cells is PEC, cells outside the box counting as PEC.
 *
 * Units: c = eps0 = mu0 = 1, lengths in metres, charge in coulombs.
 *
 * Layout: every component is an array of (nx+1)(ny+1)(nz+1) doubles,
 * z fastest: idx = k + (nz+1) * (j + (ny+1) * i).  Entries outside a
 * component's index range are unused and held at zero.
 *
 * Component positions (node (i,j,k) at (i dx, j dy, k dz)):
 *   e_x (i+1/2, j, k)   e_y (i, j+1/2, k)   e_z (i, j, k+1/2)
 *   h_x (i, j+1/2, k+1/2)  h_y (i+1/2, j, k+1/2)  h_z (i+1/2, j+1/2, k)
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

enum { EX = 0, EY = 1, EZ = 2, HX = 3, HY = 4, HZ = 5 };

typedef struct {
    int nx, ny, nz;
    int periodic_xy;           /* 1: x and y periodic (for tests); z walls stay PEC */
    double dx, dy, dz, cdt;    /* cdt = dtau = c dt */
} orc_geom;

static size_t idx(const orc_geom* g, int i, int j, int k)
{
    return (size_t)k + (size_t)(g->nz + 1) * ((size_t)j + (size_t)(g->ny + 1) * (size_t)i);
}

/* Index range of each component.  Non-periodic: the six ranges listed in the
 * header.  Periodic in x/y: i < nx and j < ny for every component. */
static int in_range(const orc_geom* g, int c, int i, int j, int k)
{
    int imax = g->nx, jmax = g->ny, kmax = g->nz;      /* inclusive node bounds */
    if (g->periodic_xy) { imax = g->nx - 1; jmax = g->ny - 1; }
    if (i < 0 || j < 0 || k < 0 || i > imax || j > jmax || k > kmax) return 0;
    switch (c) {
    case EX: return g->periodic_xy || i < g->nx;
    case EY: return g->periodic_xy || j < g->ny;
    case EZ: return k < g->nz;
    case HX: return (g->periodic_xy || j < g->ny) && k < g->nz;
    case HY: return (g->periodic_xy || i < g->nx) && k < g->nz;
    case HZ: return g->periodic_xy || (i < g->nx && j < g->ny);
    }
    return 0;
}

/* Value of component c at (i,j,k); zero outside its range (there is no grid
 * object there).  In periodic mode x and y indices wrap. */
static double at(const orc_geom* g, double* const f[6], int c, int i, int j, int k)
{
    if (g->periodic_xy) {
        i = ((i % g->nx) + g->nx) % g->nx;
        j = ((j % g->ny) + g->ny) % g->ny;
    }
    if (!in_range(g, c, i, j, k)) return 0.0;
    return f[c][idx(g, i, j, k)];
}

#define LOOP(g, c)                                     \
    for (int i = 0; i <= (g)->nx; ++i)                 \
        for (int j = 0; j <= (g)->ny; ++j)             \
            for (int k = 0; k <= (g)->nz; ++k)         \
                if (in_range((g), (c), i, j, k))

/* LOOP with its planes shared among OpenMP threads.  Used only by the
 * sub-updates, each of which writes one component from values of the other
 * components alone: every entry gets the same operands and the same operations
 * whatever the thread count, so results are bitwise those of one thread.  Sums
 * (energy, charges, wake) stay serial. */
#define PLOOP(g, c)                                    \
    _Pragma("omp parallel for schedule(static)")       \
    for (int i = 0; i <= (g)->nx; ++i)                 \
        for (int j = 0; j <= (g)->ny; ++j)             \
            for (int k = 0; k <= (g)->nz; ++k)         \
                if (in_range((g), (c), i, j, k))

/* Threads used by the sub-updates (OpenMP; 1 without it). */
#ifdef _OPENMP
#include <omp.h>
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }
#else
void orc_set_threads(int n) { (void)n; }
int orc_get_threads(void) { return 1; }
#endif

/* ---------------------------------------------------------------------------
 * Materials (Sec. 2): diagonal M_eps^-1 = kappa on edges, M_mu^-1 = mu on
 * facets, vacuum values for uniform cells in units c = eps0 = mu0 = 1:
 *   kappa_x = dx / (dy dz)  (edge length over dual-facet area), cyclic;
 *   mu_x    = dx / (dy dz)  (dual-edge length over facet area), cyclic.
 * A PEC edge has kappa = 0 (staircase rule in the header).  cell_pec may be
 * NULL (empty box); it has nx*ny*nz bytes, index k + nz*(j + ny*i).
 * ------------------------------------------------------------------------- */
static int cell_is_pec(const orc_geom* g, const unsigned char* cell, int i, int j, int k)
{
    if (g->periodic_xy) {
        i = ((i % g->nx) + g->nx) % g->nx;
        j = ((j % g->ny) + g->ny) % g->ny;
    }
    if (i < 0 || j < 0 || k < 0 || i >= g->nx || j >= g->ny || k >= g->nz) return 1;
    if (!cell) return 0;
    return cell[(size_t)k + (size_t)g->nz * ((size_t)j + (size_t)g->ny * (size_t)i)] != 0;
}

void orc_vacuum_materials(const orc_geom* g, const unsigned char* cell_pec, double* m[6])
{
    const double kx = g->dx / (g->dy * g->dz), ky = g->dy / (g->dz * g->dx),
                 kz = g->dz / (g->dx * g->dy);
    for (int c = 0; c < 6; ++c)
        memset(m[c], 0, sizeof(double) * (size_t)(g->nx + 1) * (g->ny + 1) * (g->nz + 1));
    /* e_x edge (i+1/2, j, k) touches cells (i, j-1..j, k-1..k) */
    LOOP(g, EX) {
        int pec = cell_is_pec(g, cell_pec, i, j - 1, k - 1) || cell_is_pec(g, cell_pec, i, j, k - 1) ||
                  cell_is_pec(g, cell_pec, i, j - 1, k) || cell_is_pec(g, cell_pec, i, j, k);
        m[EX][idx(g, i, j, k)] = pec ? 0.0 : kx;
    }
    /* e_y edge (i, j+1/2, k) touches cells (i-1..i, j, k-1..k) */
    LOOP(g, EY) {
        int pec = cell_is_pec(g, cell_pec, i - 1, j, k - 1) || cell_is_pec(g, cell_pec, i, j, k - 1) ||
                  cell_is_pec(g, cell_pec, i - 1, j, k) || cell_is_pec(g, cell_pec, i, j, k);
        m[EY][idx(g, i, j, k)] = pec ? 0.0 : ky;
    }
    /* e_z edge (i, j, k+1/2) touches cells (i-1..i, j-1..j, k) */
    LOOP(g, EZ) {
        int pec = cell_is_pec(g, cell_pec, i - 1, j - 1, k) || cell_is_pec(g, cell_pec, i, j - 1, k) ||
                  cell_is_pec(g, cell_pec, i - 1, j, k) || cell_is_pec(g, cell_pec, i, j, k);
        m[EZ][idx(g, i, j, k)] = pec ? 0.0 : kz;
    }
    LOOP(g, HX) m[HX][idx(g, i, j, k)] = g->dx / (g->dy * g->dz);
    LOOP(g, HY) m[HY][idx(g, i, j, k)] = g->dy / (g->dz * g->dx);
    LOOP(g, HZ) m[HZ][idx(g, i, j, k)] = g->dz / (g->dx * g->dy);
}

/* n x E = 0: zero every e entry whose kappa is zero (PEC edge). */
void orc_apply_pec(const orc_geom* g, double* const m[6], double* f[6])
{
    for (int c = EX; c <= EZ; ++c)
        LOOP(g, c) if (m[c][idx(g, i, j, k)] == 0.0) f[c][idx(g, i, j, k)] = 0.0;
}

/* ---------------------------------------------------------------------------
 * Differences.  P_x is the forward difference along x (node -> x-edge), so
 * (P_x f)(i) = f(i+1) - f(i); its transpose is (P_x^T g)(i) = g(i-1) - g(i).
 * The curl C of Sec. 2 is [[0,-P_z,P_y],[P_z,0,-P_x],[-P_y,P_x,0]].
 * ------------------------------------------------------------------------- */

/* S1 / S4: h_x += alpha mu_x [P_z e_y - P_y e_z] */
static void upd_hx(const orc_geom* g, double* const m[6], double* f[6], double a)
{
    PLOOP(g, HX) {
        double pz_ey = at(g, f, EY, i, j, k + 1) - at(g, f, EY, i, j, k);
        double py_ez = at(g, f, EZ, i, j + 1, k) - at(g, f, EZ, i, j, k);
        f[HX][idx(g, i, j, k)] += a * m[HX][idx(g, i, j, k)] * (pz_ey - py_ez);
    }
}

/* S2 / S5: h_y += alpha mu_y [-P_z e_x + P_x e_z] */
static void upd_hy(const orc_geom* g, double* const m[6], double* f[6], double a)
{
    PLOOP(g, HY) {
        double pz_ex = at(g, f, EX, i, j, k + 1) - at(g, f, EX, i, j, k);
        double px_ez = at(g, f, EZ, i + 1, j, k) - at(g, f, EZ, i, j, k);
        f[HY][idx(g, i, j, k)] += a * m[HY][idx(g, i, j, k)] * (-pz_ex + px_ez);
    }
}

/* S3: e_z += 2 alpha kappa_z [P_y^T h_x - P_x^T h_y - j_z] */
static void upd_ez(const orc_geom* g, double* const m[6], double* f[6], double a2, const double* jz)
{
    PLOOP(g, EZ) {
        double pyt_hx = at(g, f, HX, i, j - 1, k) - at(g, f, HX, i, j, k);
        double pxt_hy = at(g, f, HY, i - 1, j, k) - at(g, f, HY, i, j, k);
        double src = jz ? jz[idx(g, i, j, k)] : 0.0;
        f[EZ][idx(g, i, j, k)] += a2 * m[EZ][idx(g, i, j, k)] * (pyt_hx - pxt_hy - src);
    }
}

/* S6 / S9: e_x += alpha kappa_x [P_z^T h_y - P_y^T h_z - j_x] */
static void upd_ex(const orc_geom* g, double* const m[6], double* f[6], double a, const double* jx)
{
    PLOOP(g, EX) {
        double pzt_hy = at(g, f, HY, i, j, k - 1) - at(g, f, HY, i, j, k);
        double pyt_hz = at(g, f, HZ, i, j - 1, k) - at(g, f, HZ, i, j, k);
        double src = jx ? jx[idx(g, i, j, k)] : 0.0;
        f[EX][idx(g, i, j, k)] += a * m[EX][idx(g, i, j, k)] * (pzt_hy - pyt_hz - src);
    }
}

/* S7 / S10: e_y += alpha kappa_y [-P_z^T h_x + P_x^T h_z - j_y] */
static void upd_ey(const orc_geom* g, double* const m[6], double* f[6], double a, const double* jy)
{
    PLOOP(g, EY) {
        double pzt_hx = at(g, f, HX, i, j, k - 1) - at(g, f, HX, i, j, k);
        double pxt_hz = at(g, f, HZ, i - 1, j, k) - at(g, f, HZ, i, j, k);
        double src = jy ? jy[idx(g, i, j, k)] : 0.0;
        f[EY][idx(g, i, j, k)] += a * m[EY][idx(g, i, j, k)] * (-pzt_hx + pxt_hz - src);
    }
}

/* S8: h_z += 2 alpha mu_z [P_y e_x - P_x e_y] */
static void upd_hz(const orc_geom* g, double* const m[6], double* f[6], double a2)
{
    PLOOP(g, HZ) {
        double py_ex = at(g, f, EX, i, j + 1, k) - at(g, f, EX, i, j, k);
        double px_ey = at(g, f, EY, i + 1, j, k) - at(g, f, EY, i, j, k);
        f[HZ][idx(g, i, j, k)] += a2 * m[HZ][idx(g, i, j, k)] * (py_ex - px_ey);
    }
}

/*
 * One step of scheme (23): y^n = (u^{n-1/2}, v^n) -> y^{n+1}, in place, as the
 * ten sub-updates of Sec. 4.2 in the paper's order.  Currents are per-edge
 * arrays (or NULL): jz = j_z^n, jx = j_x^{n+1/2}, jy = j_y^{n+1/2}, as current
 * through the dual facet (charge per unit of tau).
 */
void orc_step(const orc_geom* g, double* const m[6], double* f[6],
              const double* jx, const double* jy, const double* jz)
{
    const double a = 0.5 * g->cdt;     /* alpha = dtau / 2, eq. (17) */
    upd_hx(g, m, f, a);                /* S1: h_x^n        */
    upd_hy(g, m, f, a);                /* S2: h_y^n        */
    upd_ez(g, m, f, 2.0 * a, jz);      /* S3: e_z^{n+1/2}  */
    upd_hx(g, m, f, a);                /* S4: h_x^{n+1/2}  */
    upd_hy(g, m, f, a);                /* S5: h_y^{n+1/2}  */
    upd_ex(g, m, f, a, jx);            /* S6: e_x^{n+1/2}  */
    upd_ey(g, m, f, a, jy);            /* S7: e_y^{n+1/2}  */
    upd_hz(g, m, f, 2.0 * a);          /* S8: h_z^{n+1}    */
    upd_ex(g, m, f, a, jx);            /* S9: e_x^{n+1}    */
    upd_ey(g, m, f, a, jy);            /* S10: e_y^{n+1}   */
}

/*
 * Discrete energy W^{n,e} = 1/2 <Q^e y^n, y^n> (Sec. 4.4) with
 * Q^e = [[I - a^2 R_0, a L], [a L^T, I - a^2 R_1]], written in FIT variables
 * (e = kappa^-1/2 e^, h = mu^-1/2 h^).  Edges with kappa = 0 (PEC) carry no
 * degree of freedom and are left out of every e-sum.
 *   |u|^2 + |v|^2      = sum h^2/mu + sum_{kappa>0} e^2/kappa
 *   <R_0 u, u>         = sum_hx mu_x (P_y e_z)^2 + sum_hy mu_y (P_x e_z)^2
 *   <R_1 v, v>         = sum_{ex, kappa>0} kappa_x (P_y^T h_z)^2 + sum_{ey, kappa>0} kappa_y (P_x^T h_z)^2
 *   <L v, u>           = sum_hx h_x P_z e_y - sum_hy h_y P_z e_x
 */
/* Compensated running sum (Neumaier's variant of Kahan summation): a grid's
 * energy adds up ~1e8 terms, and a plain running sum of that many loses about
 * 1e-12 of the total, the size of the parity tolerance; the compensation
 * keeps the rounding error of the sum near one unit of the result. */
typedef struct { double s, c; } orc_sum;

static void add(orc_sum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

static double total(const orc_sum* a) { return a->s + a->c; }

double orc_energy(const orc_geom* g, double* const m[6], double* f[6])
{
    const double a = 0.5 * g->cdt;
    orc_sum sq = {0, 0}, r0 = {0, 0}, r1 = {0, 0}, lc = {0, 0};
    for (int c = EX; c <= EZ; ++c)
        LOOP(g, c) {
            double kap = m[c][idx(g, i, j, k)];
            if (kap > 0.0) { double e = f[c][idx(g, i, j, k)]; add(&sq, e * e / kap); }
        }
    for (int c = HX; c <= HZ; ++c)
        LOOP(g, c) {
            double mu = m[c][idx(g, i, j, k)];
            double h = f[c][idx(g, i, j, k)];
            if (mu > 0.0) add(&sq, h * h / mu);
        }
    LOOP(g, HX) {
        double d = at(g, f, EZ, i, j + 1, k) - at(g, f, EZ, i, j, k);
        add(&r0, m[HX][idx(g, i, j, k)] * d * d);
        add(&lc, f[HX][idx(g, i, j, k)] * (at(g, f, EY, i, j, k + 1) - at(g, f, EY, i, j, k)));
    }
    LOOP(g, HY) {
        double d = at(g, f, EZ, i + 1, j, k) - at(g, f, EZ, i, j, k);
        add(&r0, m[HY][idx(g, i, j, k)] * d * d);
        add(&lc, -f[HY][idx(g, i, j, k)] * (at(g, f, EX, i, j, k + 1) - at(g, f, EX, i, j, k)));
    }
    LOOP(g, EX) {
        double kap = m[EX][idx(g, i, j, k)];
        if (kap > 0.0) {
            double d = at(g, f, HZ, i, j - 1, k) - at(g, f, HZ, i, j, k);
            add(&r1, kap * d * d);
        }
    }
    LOOP(g, EY) {
        double kap = m[EY][idx(g, i, j, k)];
        if (kap > 0.0) {
            double d = at(g, f, HZ, i - 1, j, k) - at(g, f, HZ, i, j, k);
            add(&r1, kap * d * d);
        }
    }
    return 0.5 * total(&sq) - 0.5 * a * a * (total(&r0) + total(&r1)) + a * total(&lc);
}

/*
 * Conserved charges of Sec. 4.5 (charge conservation), eqs. (34) and (35),
 * with the (I - alpha^2 r_i) reading.  Inputs: the state before a step,
 * fo = y^n = (u^{n-1/2}, v^n), and after it, fn = y^{n+1} = (u^{n+1/2}, v^{n+1}).
 *
 * qe[node] = q_e^{n+1/2} = -[P_x^T dbar_x + P_y^T dbar_y + P_z^T dtil_z], with
 *   dbar = (e^n + e^{n+1}) / (2 kappa) on x/y edges,
 *   dtil_z = e_z^{n+1/2}/kappa_z - alpha^2 (P_y^T mu_x P_y + P_x^T mu_y P_x) e_z^{n+1/2};
 *   PEC edges (kappa = 0) contribute nothing.  The law (35) holds at every node
 *   whose six edges are all non-PEC.
 * qh[cell] = q_h^n = P_x bbar_x + P_y bbar_y + P_z btil_z  (cell (i,j,k) at its
 *   centre, array index k + nz*(j + ny*i)), with
 *   bbar = (h^{n-1/2} + h^{n+1/2}) / (2 mu),
 *   btil_z = h_z^n/mu_z - alpha^2 (P_y kappa_x P_y^T + P_x kappa_y P_x^T) h_z^n.
 */
static double dbar(const orc_geom* g, double* const m[6], double* fo[6], double* fn[6],
                   int c, int i, int j, int k)
{
    if (!in_range(g, c, i, j, k)) return 0.0;
    double kap = m[c][idx(g, i, j, k)];
    if (kap == 0.0) return 0.0;
    return 0.5 * (fo[c][idx(g, i, j, k)] + fn[c][idx(g, i, j, k)]) / kap;
}

static double dtilz(const orc_geom* g, double* const m[6], double* fn[6], int i, int j, int k)
{
    const double a = 0.5 * g->cdt;
    if (!in_range(g, EZ, i, j, k)) return 0.0;
    double kap = m[EZ][idx(g, i, j, k)];
    if (kap == 0.0) return 0.0;
    /* (P_y^T mu_x P_y e_z)(i,j) = mu_x(j-1) (e_z(j) - e_z(j-1)) - mu_x(j) (e_z(j+1) - e_z(j)) */
    double muxm = in_range(g, HX, i, j - 1, k) ? m[HX][idx(g, i, j - 1, k)] : 0.0;
    double muxp = in_range(g, HX, i, j, k) ? m[HX][idx(g, i, j, k)] : 0.0;
    double muym = in_range(g, HY, i - 1, j, k) ? m[HY][idx(g, i - 1, j, k)] : 0.0;
    double muyp = in_range(g, HY, i, j, k) ? m[HY][idx(g, i, j, k)] : 0.0;
    double e0 = fn[EZ][idx(g, i, j, k)];
    double r = muxm * (e0 - at(g, fn, EZ, i, j - 1, k)) - muxp * (at(g, fn, EZ, i, j + 1, k) - e0)
             + muym * (e0 - at(g, fn, EZ, i - 1, j, k)) - muyp * (at(g, fn, EZ, i + 1, j, k) - e0);
    return e0 / kap - a * a * r;
}

static double bbar(const orc_geom* g, double* const m[6], double* fo[6], double* fn[6],
                   int c, int i, int j, int k)
{
    if (!in_range(g, c, i, j, k)) return 0.0;
    double mu = m[c][idx(g, i, j, k)];
    if (mu == 0.0) return 0.0;
    return 0.5 * (fo[c][idx(g, i, j, k)] + fn[c][idx(g, i, j, k)]) / mu;
}

static double btilz(const orc_geom* g, double* const m[6], double* fo[6], int i, int j, int k)
{
    const double a = 0.5 * g->cdt;
    if (!in_range(g, HZ, i, j, k)) return 0.0;
    double mu = m[HZ][idx(g, i, j, k)];
    if (mu == 0.0) return 0.0;
    /* gx(i,j) = (kappa_x P_y^T h_z)(i,j) at e_x = kappa_x(i,j) (h_z(j-1) - h_z(j));
       (P_y gx)(i,j) at h_z = gx(i,j+1) - gx(i,j).  Same along x with e_y. */
#define KAP(c, ii, jj) (in_range(g, (c), (ii), (jj), k) ? m[(c)][idx(g, (ii), (jj), k)] : 0.0)
    double gx_p = KAP(EX, i, j + 1) * (at(g, fo, HZ, i, j, k) - at(g, fo, HZ, i, j + 1, k));
    double gx_0 = KAP(EX, i, j) * (at(g, fo, HZ, i, j - 1, k) - at(g, fo, HZ, i, j, k));
    double gy_p = KAP(EY, i + 1, j) * (at(g, fo, HZ, i, j, k) - at(g, fo, HZ, i + 1, j, k));
    double gy_0 = KAP(EY, i, j) * (at(g, fo, HZ, i - 1, j, k) - at(g, fo, HZ, i, j, k));
#undef KAP
    double r = (gx_p - gx_0) + (gy_p - gy_0);
    return fo[HZ][idx(g, i, j, k)] / mu - a * a * r;
}

void orc_charges(const orc_geom* g, double* const m[6], double* fo[6], double* fn[6],
                 double* qe, double* qh)
{
    for (int i = 0; i <= g->nx; ++i)
        for (int j = 0; j <= g->ny; ++j)
            for (int k = 0; k <= g->nz; ++k) {
                double q = dbar(g, m, fo, fn, EX, i, j, k) - dbar(g, m, fo, fn, EX, i - 1, j, k)
                         + dbar(g, m, fo, fn, EY, i, j, k) - dbar(g, m, fo, fn, EY, i, j - 1, k)
                         + dtilz(g, m, fn, i, j, k) - dtilz(g, m, fn, i, j, k - 1);
                qe[idx(g, i, j, k)] = q;
            }
    for (int i = 0; i < g->nx; ++i)
        for (int j = 0; j < g->ny; ++j)
            for (int k = 0; k < g->nz; ++k) {
                double q = bbar(g, m, fo, fn, HX, i + 1, j, k) - bbar(g, m, fo, fn, HX, i, j, k)
                         + bbar(g, m, fo, fn, HY, i, j + 1, k) - bbar(g, m, fo, fn, HY, i, j, k)
                         + btilz(g, m, fo, i, j, k + 1) - btilz(g, m, fo, i, j, k);
                qh[(size_t)k + (size_t)g->nz * ((size_t)j + (size_t)g->ny * (size_t)i)] = q;
            }
}

/*
 * Rigid Gaussian bunch, RMS length sigma, total charge Q, truncated at |m| <= M
 * cells (no renormalisation).  lam[m + M] = charge of the bunch in a cell of
 * length dz whose centre is m*dz ahead of the bunch centre:
 *   lam_m = Q [Phi((m+1/2) dz/sigma) - Phi((m-1/2) dz/sigma)],
 * with Phi the standard normal distribution, evaluated via erfc so that the
 * tails keep their relative accuracy.
 */
void orc_bunch_cells(double Q, double sigma, double dz, int M, double* lam)
{
    for (int mm = -M; mm <= M; ++mm) {
        double a = (mm - 0.5) * dz / sigma, b = (mm + 0.5) * dz / sigma;
        double v;
        if (a >= 0.0)      v = 0.5 * (erfc(a / sqrt(2.0)) - erfc(b / sqrt(2.0)));
        else if (b <= 0.0) v = 0.5 * (erfc(-b / sqrt(2.0)) - erfc(-a / sqrt(2.0)));
        else               v = 1.0 - 0.5 * erfc(-a / sqrt(2.0)) - 0.5 * erfc(b / sqrt(2.0));
        lam[mm + M] = Q * v;
    }
}

/*
 * Wake run.  The bunch moves along +z on the node line (i0, j0) at v = c with
 * dtau = dz, so it advances exactly one cell per step (Fig. 1).  Its centre is
 * at z_c(tau) = tau - (M - 1/2) dz.  The charge crossing the dual facet of
 * e_z edge k during [tau_{n-1/2}, tau_{n+1/2}] is then the charge of cell
 * m = k - n + M, i.e. j_z^n(k) dtau = lam_{k-n+M}: the head crosses edge 0 in
 * step 0 and the centre crosses edge k in step n = k + M.
 *
 * Wake potential (Sec. 5): W(s) = -(1/Q) int E_z(z, t = (z+s)/c) dz, s > 0
 * behind the centre.  With e_z the edge voltage (E_z dz) and the time of
 * edge k for s_j = j dz being tau = (k + M + j) dz, the time-staggered e_z is
 * averaged:  acc[j - jmin] += -1/2 (e_z^{n-1/2} + e_z^{n+1/2})(i0,j0,k) with
 * n = k + M + j.  The caller divides by Q (and by eps0 for V/C).
 *
 * Only edges k < kend enter the quadrature (kend <= 0: every edge): the wake
 * integral of a run with open pipes ends there, so that no field reflected
 * by the exit wall reaches it (reading of the infinite pipes of Sec. 5).
 *
 * Per step n in [n0, n0+nsteps): energy[n-n0] = W^{n,e} of y^n (if energy),
 * probe_out[(n-n0)*nprobe + p] = f[EZ][probe_idx[p]] after the step (e_z^{n+1/2}).
 */
typedef struct {
    int active;
    int i0, j0, M;
    const double* lam;   /* 2M+1 cell charges */
    int jmin, nw;        /* wake samples s_j, j = jmin .. jmin+nw-1 */
    int kend;            /* quadrature over edges k < kend; <= 0: all nz edges */
} orc_bunch;

int orc_run(const orc_geom* g, double* const m[6], double* f[6], int n0, int nsteps,
            const orc_bunch* b, double* acc, double* energy,
            const long long* probe_idx, int nprobe, double* probe_out)
{
    size_t np = (size_t)(g->nx + 1) * (g->ny + 1) * (g->nz + 1);
    double* jz = NULL;
    double* ezo = NULL;
    if (b && b->active) {
        jz = (double*)calloc(np, sizeof(double));
        ezo = (double*)calloc((size_t)g->nz, sizeof(double));
        if (!jz || !ezo) { free(jz); free(ezo); return -1; }
    }
    for (int s = 0; s < nsteps; ++s) {
        int n = n0 + s;
        if (energy) energy[s] = orc_energy(g, m, f);
        if (jz) {
            for (int k = 0; k < g->nz; ++k) {
                int mm = k - n + b->M;
                double q = (mm >= -b->M && mm <= b->M) ? b->lam[mm + b->M] : 0.0;
                jz[idx(g, b->i0, b->j0, k)] = q / g->cdt;     /* current = charge / dtau */
                ezo[k] = f[EZ][idx(g, b->i0, b->j0, k)];
            }
        }
        orc_step(g, m, f, NULL, NULL, jz);
        if (jz && acc) {
            const int kend = b->kend > 0 && b->kend < g->nz ? b->kend : g->nz;
            for (int k = 0; k < kend; ++k) {
                int jj = n - k - b->M;
                if (jj >= b->jmin && jj < b->jmin + b->nw)
                    acc[jj - b->jmin] += -0.5 * (ezo[k] + f[EZ][idx(g, b->i0, b->j0, k)]);
            }
        }
        if (probe_out)
            for (int p = 0; p < nprobe; ++p)
                probe_out[(size_t)s * nprobe + p] = f[EZ][probe_idx[p]];
    }
    free(jz);
    free(ezo);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Yee's E/M scheme (7), the baseline the paper compares against (Sec. 3):
 *   e^{n+1/2} = e^{n-1/2} + dtau C_0^* h^n - dtau j^n,
 *   h^{n+1}   = h^n - dtau C_0 e^{n+1/2},
 * in FIT variables: every e component is updated from h^n first, then every h
 * component from e^{n+1/2}; stable in vacuum for dtau up to (8).  The state
 * holds (e^{n-1/2}, h^n).  jz (or NULL) is j_z^n per e_z edge as current
 * through the dual facet, as for orc_step.
 * ------------------------------------------------------------------------- */
void orc_step_yee(const orc_geom* g, double* const m[6], double* f[6], const double* jz)
{
    const double dt = g->cdt;
    upd_ex(g, m, f, dt, NULL);          /* e_x^{n+1/2} */
    upd_ey(g, m, f, dt, NULL);          /* e_y^{n+1/2} */
    upd_ez(g, m, f, dt, jz);            /* e_z^{n+1/2} */
    /* h^{n+1} = h^n - dtau mu C e^{n+1/2}: the h sub-updates with factor dtau */
    upd_hx(g, m, f, dt);
    upd_hy(g, m, f, dt);
    upd_hz(g, m, f, dt);
}

/*
 * Leapfrog invariant of Yee's scheme with j = 0 (exactly conserved: the change
 * from n to n+1 is dtau (<e, C_0^* H> - <C_0 e, H>) = 0 with H = h^n + h^{n+1}):
 *   I^n = <e^{n+1/2}, e^{n-1/2}> + |h^n|^2  (scaled variables), i.e. in FIT
 *   variables sum_{kappa>0} e^{n+1/2} e^{n-1/2} / kappa + sum h^2 / mu.
 * Inputs: fo = (e^{n-1/2}, h^n) and fn = the state after the step (its e part
 * is e^{n+1/2}).  Returns I^n / 2 (an energy).
 */
double orc_yee_invariant(const orc_geom* g, double* const m[6], double* fo[6], double* fn[6])
{
    double s = 0.0;
    for (int c = EX; c <= EZ; ++c)
        LOOP(g, c) {
            double kap = m[c][idx(g, i, j, k)];
            if (kap > 0.0) s += fo[c][idx(g, i, j, k)] * fn[c][idx(g, i, j, k)] / kap;
        }
    for (int c = HX; c <= HZ; ++c)
        LOOP(g, c) {
            double mu = m[c][idx(g, i, j, k)];
            if (mu > 0.0) s += fo[c][idx(g, i, j, k)] * fo[c][idx(g, i, j, k)] / mu;
        }
    return 0.5 * s;
}

/*
 * Discrete Gauss law of Yee's scheme: with j = 0 the dual divergence of the
 * flux d = e / kappa is constant in time, because the dual divergence of
 * C^T h vanishes identically.  Writes, for every node (i,j,k), the value
 *   -[P_x^T d_x + P_y^T d_y + P_z^T d_z](i,j,k)
 *   = d_x(i,j,k) - d_x(i-1,j,k) + d_y(i,j,k) - d_y(i,j-1,k) + d_z(i,j,k) - d_z(i,j,k-1)
 * into q (index as the field arrays); PEC edges carry no flux.
 */
void orc_yee_charge(const orc_geom* g, double* const m[6], double* f[6], double* q)
{
    memset(q, 0, sizeof(double) * (size_t)(g->nx + 1) * (g->ny + 1) * (g->nz + 1));
    for (int i = 0; i <= g->nx; ++i)
        for (int j = 0; j <= g->ny; ++j)
            for (int k = 0; k <= g->nz; ++k) {
                double s = 0.0;
                const int di[3] = {1, 0, 0}, dj[3] = {0, 1, 0}, dk[3] = {0, 0, 1};
                for (int c = EX; c <= EZ; ++c) {
                    /* outgoing edge from this node, incoming edge from the previous node */
                    int io = i, jo = j, ko = k, ii = i - di[c], ji = j - dj[c], ki = k - dk[c];
                    if (g->periodic_xy) {
                        ii = ((ii % g->nx) + g->nx) % g->nx;
                        ji = ((ji % g->ny) + g->ny) % g->ny;
                    }
                    if (in_range(g, c, io, jo, ko)) {
                        double kap = m[c][idx(g, io, jo, ko)];
                        if (kap > 0.0) s += f[c][idx(g, io, jo, ko)] / kap;
                    }
                    if (in_range(g, c, ii, ji, ki)) {
                        double kap = m[c][idx(g, ii, ji, ki)];
                        if (kap > 0.0) s -= f[c][idx(g, ii, ji, ki)] / kap;
                    }
                }
                q[idx(g, i, j, k)] = s;
            }
}
