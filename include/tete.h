/*
 * tete.h -- C-ABI of the explicit TE/TM wakefield time stepper for MI355X
 * (gfx950), after Dohlus & Zagorodnov, "Explicit TE/TM scheme for particle
 * beam simulations".
 *
 * The library advances the discrete Cauchy problem of Sec. 2, eq. (1) with
 * PEC walls (n x E = 0 on the boundary), in the finite-integration form (4):
 * the curl C and its transpose on a Cartesian grid doublet, diagonal material
 * matrices M_eps^-1 and M_mu^-1, and a current j.  Time stepping is the
 * explicit TE/TM scheme (23), executed as the ten sub-updates of Sec. 4.2 on
 * the GPU.  The source is a rigid Gaussian bunch moving at v = c along a node
 * line; the library accumulates the longitudinal wake potential of Sec. 5 and
 * evaluates the discrete energy of Sec. 4.4 and the conserved charges (34),
 * (35).
 *
 * Units: c = eps0 = mu0 = 1 internally; lengths in metres; charge in
 * coulombs.  Field values are FIT voltages: e^ = E * edge length,
 * h^ = H * dual-edge length, in these units.  tete_wake converts to V/C.
 *
 * Grid and layout: nx, ny, nz cells; node (i,j,k) at (i dx, j dy, k dz).
 * Every component is one array of np = (nx+1)(ny+1)(nz+1) entries, z fastest:
 * index = k + (nz+1) * (j + (ny+1) * i).  Component positions:
 *   e_x (i+1/2, j, k)   e_y (i, j+1/2, k)   e_z (i, j, k+1/2)
 *   h_x (i, j+1/2, k+1/2)  h_y (i+1/2, j, k+1/2)  h_z (i+1/2, j+1/2, k)
 * Entries outside a component's index range (e.g. e_x at i = nx) hold no grid
 * object; the library keeps them at zero.  Array order in the [6] arguments
 * below: e_x, e_y, e_z, h_x, h_y, h_z.
 *
 * Memory: the caller owns one device workspace (tete_workspace_bytes) and
 * the HIP stream; the library never allocates or frees device memory.  All
 * bulk array arguments are DEVICE pointers, read or written on the grid's
 * stream; small result arguments are HOST pointers.  A call that returns an
 * error leaves the grid state unchanged unless stated otherwise.
 *
 * Error state: a read-out (tete_wake, tete_witness_wake, tete_energy,
 * tete_energy_series, tete_probes, tete_charges) that finds NaN or Inf puts
 * the grid into the sticky TETE_ERR_NONFINITE state.  The read-out still
 * fills its outputs; meanwhile tete_step does nothing and returns
 * TETE_ERR_NONFINITE, every read-out returns it, and the grid cannot join or
 * step in a batch.  tete_set_fields (a new initial state) clears it;
 * tete_grid_status reports it.
 *
 * Ordering: calls are ordered on the grid's stream.  tete_step only enqueues
 * work; tete_wake, tete_energy, tete_energy_series, tete_probes and
 * tete_charges synchronise the stream before they return.  One grid may be
 * used by one host thread at a time.
 */
#ifndef TETE_H
#define TETE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tete_grid tete_grid; /* opaque handle */

typedef enum {
    TETE_OK = 0,
    TETE_ERR_ARG = -1,       /* invalid argument (size, index, pointer, alignment) */
    TETE_ERR_UNSTABLE = -2,  /* cdt violates the stability bound (25), or materials
                              * fail the sufficient Q^e >= 0 test (Sec. 4.4) */
    TETE_ERR_NOMEM = -3,     /* workspace smaller than tete_workspace_bytes */
    TETE_ERR_DEVICE = -4,    /* a HIP call or kernel launch failed */
    TETE_ERR_STATE = -5,     /* call not valid in the grid's current state */
    TETE_ERR_NONFINITE = -6  /* a read-out found NaN or Inf (fields diverged); the grid
                              * stays in this state until tete_set_fields */
} tete_status;

/* Arithmetic type of the field arrays.  FP32 keeps the wake accumulation,
 * energy and charge diagnostics and the bunch table in FP64. */
enum { TETE_FP64 = 0, TETE_FP32 = 1 };

/* desc.flags */
enum {
    TETE_F_MATERIALS = 1u << 0, /* reserve per-entry material arrays (tete_set_materials) */
    TETE_F_YEE = 1u << 1,       /* step with Yee's E/M scheme (7) instead of (23): a
                                 * baseline for comparison.  State (e^{n-1/2}, h^n);
                                 * stability bound (8); vacuum with staircase PEC only
                                 * (not with TETE_F_MATERIALS); no bunch (its current
                                 * needs cdt = dz, which (8) excludes), no energy,
                                 * energy series or charges (TETE_ERR_STATE); probes
                                 * record e_z^{n+1/2}. */
    TETE_F_SKIP_STATIC = 1u << 3, /* the fused kernels leave out tiles that lie wholly in
                                 * PEC: every entry such a tile reads has its three e
                                 * edges PEC, so e stays zero and h constant there and a
                                 * step changes none of its entries.  Fields and wakes
                                 * equal those of a grid without the flag.  Tiles are left out
                                 * only once both ping-pong sets agree (from the second
                                 * launch after tete_set_fields or tete_set_pec_cells).
                                 * Two-step and fused single-step launches take only
                                 * the other tiles (the two-kernel step of
                                 * TETE_KERNEL_SPLIT and batches take all); with tuning
                                 * x-chunk 0 the two-step launches use chunks of 32
                                 * planes.
                                 * The tile list is built, and the stream synchronised,
                                 * at the first such launch after the codes or the
                                 * tiling (rows, x-chunk, order; witness set or not)
                                 * change.  With TETE_F_MATERIALS, once materials are
                                 * set, the fused single step leaves out the tiles
                                 * whose kappa is zero on every e edge they load, by
                                 * the same rules (the list is rebuilt after
                                 * tete_set_materials).  tete_static_tiles reports
                                 * the tiling of the next step.  Not with TETE_F_YEE
                                 * or TETE_F_IMPLICIT. */
    TETE_F_IMPLICIT = 1u << 2   /* step with the implicit TE/TM scheme (16) of Sec. 4.1
                                 * instead of (23): a comparator.  Each half step solves
                                 * (I - alpha T_i) x = rhs; per z-plane this is one
                                 * positive definite system for e_z (h_z), solved by a
                                 * fixed number of Chebyshev iterations on the spectral
                                 * bounds [1, 1 + alpha^2 (4/dx^2 + 4/dy^2)] (to 1e-17 in
                                 * FP64, 1e-8 in FP32 relative to the first iterate's
                                 * error), over lists of the systems' rows that the
                                 * first tete_step after tete_set_pec_cells builds
                                 * (that call synchronises the stream; the workspace
                                 * holds two int32 lists of np entries).  Stable for
                                 * cdt <= dz with any transverse
                                 * mesh; vacuum with staircase PEC only (not with
                                 * TETE_F_MATERIALS or TETE_F_YEE); bunch, wake, probes,
                                 * energy (Q = B - alpha A of (16): no alpha^2 terms)
                                 * and charges (the time-averaged charge, no alpha^2
                                 * term) as for (23); not in batches. */
};

/* Capacities of the small per-grid tables held in the workspace. */
enum {
    TETE_MAX_BUNCH_CELLS = 8191, /* 2M+1 cells of the truncated bunch */
    TETE_MAX_WAKE = 65536,       /* wake samples */
    TETE_MAX_PROBES = 16,        /* e_z probe points */
    TETE_WITNESS_LINES = 5,      /* e_z lines of a witness: its node and four neighbours */
    TETE_MAX_BATCH = 256,        /* instances of one batch */
    TETE_MAX_CLASSES = 256       /* material classes (tete_set_material_classes) */
};

typedef struct {
    int32_t nx, ny, nz;   /* cells, each >= 2; (nx+1)(ny+1)(nz+1) <= 2^31 - 2^24 */
    double dx, dy, dz;    /* cell sizes [m] */
    double cdt;           /* dtau = c dt [m]; must satisfy (25):
                             cdt <= dz and cdt <= (dx^-2 + dy^-2)^(-1/2) */
    int32_t precision;    /* TETE_FP64 or TETE_FP32 */
    uint32_t flags;       /* TETE_F_* */
    int32_t max_series;   /* capacity of energy / probe series (0: 4096) */
} tete_grid_desc;

/* Stability and size check of a descriptor (host only, no device access).
 * Returns TETE_OK, TETE_ERR_ARG or TETE_ERR_UNSTABLE (bound (25), Sec. 4.4;
 * with TETE_F_YEE bound (8), Sec. 3; with TETE_F_IMPLICIT cdt <= dz, (22)). */
tete_status tete_check_desc(const tete_grid_desc* desc);

/* Bytes of device workspace a grid with this descriptor needs (0 if the
 * descriptor is invalid).  This is the grid's whole HBM footprint. */
size_t tete_workspace_bytes(const tete_grid_desc* desc);

/* Create a grid on the current HIP device inside the caller's workspace
 * (dev_ws, 256-byte aligned, ws_bytes >= tete_workspace_bytes(desc)), using
 * the HIP stream hip_stream (a hipStream_t; NULL = null stream).  The fields
 * start at zero, the domain is an empty vacuum PEC box (kappa = 0 on the
 * edges tangential to the walls, Sec. 2), no bunch, step counter 0.
 * Errors: TETE_ERR_ARG, TETE_ERR_UNSTABLE, TETE_ERR_NOMEM, TETE_ERR_DEVICE. */
tete_status tete_grid_create(const tete_grid_desc* desc, void* dev_ws, size_t ws_bytes,
                             void* hip_stream, tete_grid** out);

/* Release the host handle (the workspace stays the caller's). */
tete_status tete_grid_destroy(tete_grid* g);

/* Staircase geometry (Sec. 4.4 bound and Sec. 2 PEC): cell_is_pec is a DEVICE
 * array of nx*ny*nz bytes, index k + nz*(j + ny*i), non-zero = perfectly
 * conducting cell.  An edge becomes PEC (kappa = 0) if any of its up to four
 * adjacent cells is PEC; cells outside the box count as PEC.  Vacuum values
 * elsewhere: kappa_x = mu_x = dx/(dy dz), cyclic.  NULL = empty box.  Zeroes
 * e on the new PEC edges (n x E = 0).  Copies; the caller keeps its array. */
tete_status tete_set_pec_cells(tete_grid* g, const uint8_t* cell_is_pec);

/* General diagonal materials (Sec. 2, eq. (4)): DEVICE arrays of np entries
 * of type dtype (TETE_FP64/TETE_FP32): inv_eps[0..2] = M_eps^-1 on e_x,e_y,e_z
 * edges (0 = PEC edge), inv_mu[0..2] = M_mu^-1 on h_x,h_y,h_z.  Requires a grid
 * created with TETE_F_MATERIALS, else TETE_ERR_STATE.  Values in each
 * component's index range must be finite and >= 0 (TETE_ERR_ARG otherwise;
 * entries outside it are ignored).  Zeroes e where inv_eps = 0.  Replaces the
 * staircase vacuum.
 * Stability (Sec. 4.4: the scheme is stable when Q^e is positive definite):
 * before importing, the library checks a sufficient condition on the GPU.  In
 * the scaled variables h / sqrt(mu), e / sqrt(kappa), Q^e falls into three
 * independent blocks -- e_z alone (I - alpha^2 R_0), h_z alone
 * (I - alpha^2 R_1) and (h_x, h_y, e_x, e_y) coupled by alpha L -- and each is
 * positive semi-definite when every Gershgorin row sum of its subtracted and
 * off-diagonal parts is at most 1, alpha = cdt/2:
 *   e_z row:  alpha^2 sum over its 4 h facets of mu (kappa_z + sqrt(kappa_z kappa_z'))
 *   h_z row:  alpha^2 sum over its 4 e edges of kappa (mu_z + sqrt(mu_z mu_z'))
 *   h_x row:  alpha sqrt(mu_x) (sqrt(kappa_y(k)) + sqrt(kappa_y(k+1))), h_y likewise
 *             with kappa_x; e_y row: alpha sqrt(kappa_y) (sqrt(mu_x(k-1)) +
 *             sqrt(mu_x(k))), e_x likewise with mu_y,
 * primes denoting the neighbour across the facet or edge.  With vacuum
 * coefficients this is the bound (25).  If the largest sum exceeds 1 (to
 * 1e-12) the call returns TETE_ERR_UNSTABLE and changes nothing.  The test
 * is sufficient, not necessary.
 * Classes found in the arrays: after importing, the library collects the
 * distinct tuples (kappa_x, kappa_y, kappa_z, mu_x, mu_y, mu_z) of the entries
 * (in the grid's precision; 0 outside a component's range) with a hash table
 * on the GPU.  If there are at most TETE_MAX_CLASSES and kappa is 0 on every
 * edge the PEC codes mark (the box walls and tete_set_pec_cells), the grid
 * runs as after tete_set_material_classes with those tuples: paired steps
 * take the two-step kernel's class instance, with the same results as the
 * materials step over the arrays.  Otherwise, with FP32 fields, paired steps
 * take the two-step kernel's arrays instance (16 rows of 32 lanes, the six
 * arrays read with the fields once per two steps; not with witness lines or
 * TETE_F_SKIP_STATIC), with the same results as single materials steps; every
 * other step (and every step with FP64 fields) is the materials step.
 * Synchronises the stream. */
tete_status tete_set_materials(tete_grid* g, const void* const inv_eps[3],
                               const void* const inv_mu[3], int32_t dtype);

/* Materials by class: an exact compact form of the general diagonal
 * M_eps^-1, M_mu^-1 of eq. (4) (Sec. 2) for media with at most
 * TETE_MAX_CLASSES distinct coefficient tuples.  cls: DEVICE array of np
 * bytes, the class of each entry; table: HOST array of ncls x 6 doubles,
 * (kappa_x, kappa_y, kappa_z, mu_x, mu_y, mu_z) of class c at table[6c ..
 * 6c+5], finite and >= 0, 1 <= ncls <= TETE_MAX_CLASSES.  Entry e then has
 * the coefficients of class cls[e], except that kappa is 0 on the PEC edges
 * of the current geometry (tete_set_pec_cells: staircase cells and the box
 * walls; call that first, it drops the materials) and entries outside a
 * component's range hold no object.  Requires TETE_F_MATERIALS
 * (TETE_ERR_STATE).  Class bytes >= ncls are TETE_ERR_ARG; the stability
 * test of tete_set_materials applies (TETE_ERR_UNSTABLE), and on any error
 * nothing changes.  The classes are expanded into the per-entry arrays
 * (single steps, diagnostics), and steps paired by tete_step run the
 * two-step kernel's class instance (FP32 24 rows of 32 lanes; FP64 16 rows
 * of 32 lanes; the tuning's rows and depth do not apply): it reads one class
 * byte per entry and the class table from LDS instead of the six arrays, with
 * the same results as single materials steps.  With witness lines every step
 * is a single step.  Zeroes e on PEC edges.  Synchronises the stream. */
tete_status tete_set_material_classes(tete_grid* g, const uint8_t* cls, const double* table, int32_t ncls);

/* Initial field y^0 = (u^{-1/2}, v^0) (time levels of eq. (17)): h_x, h_y, e_z
 * at tau = -cdt/2 and e_x, e_y, h_z at tau = 0.  f[6] are DEVICE arrays of np
 * entries of type dtype.  Out-of-range entries and e on PEC edges are
 * stored as zero.  Resets the step counter, the wake accumulator and the
 * series. */
tete_status tete_set_fields(tete_grid* g, const void* const f[6], int32_t dtype);

/* Copy the current state y^n into DEVICE arrays f[6] (np entries of dtype). */
tete_status tete_get_fields(tete_grid* g, void* const f[6], int32_t dtype);

/* Rigid Gaussian bunch (Fig. 1): total charge charge_C, RMS length sigma_z,
 * moving at v = c along +z on the node line (i0, j0), 0 < i0 < nx,
 * 0 < j0 < ny.  It is cut to 2*half_cells+1 cells of length dz; cell m
 * (|m| <= half_cells, m dz ahead of the centre) carries
 * charge_C [Phi((m+1/2) dz/sigma) - Phi((m-1/2) dz/sigma)].  Requires
 * cdt == dz (one cell per step).  The charge crossing e_z edge k in step n is
 * the charge of cell m = k - n + half_cells: the head crosses edge 0 in step
 * 0.  Wake samples s_j = j dz for j = jmin .. jmin+nw-1 (s > 0 behind the
 * centre).  Resets the wake accumulator; the step counter is not changed.
 * Errors: TETE_ERR_ARG (bounds, capacities), TETE_ERR_STATE (cdt != dz). */
typedef struct {
    double charge_C;
    double sigma_z;       /* [m] */
    int32_t i0, j0;
    int32_t half_cells;   /* M */
    int32_t jmin;
    int32_t nw;           /* <= TETE_MAX_WAKE */
} tete_bunch;
tete_status tete_set_bunch(tete_grid* g, const tete_bunch* b);

/* Remove the bunch (no current; wake accumulation stops). */
tete_status tete_clear_bunch(tete_grid* g);

/* Diagnostics recorded during tete_step: every > 0 records W^{n,e} of y^n
 * (Sec. 4.4) before each step n with n % every == 0; 0 disables.  On vacuum
 * grids (also with witness lines) and grids with materials by class, without
 * TETE_F_SKIP_STATIC, a launch of the two-step kernel takes the samples of its
 * input y^n and of y^{n+1} itself (FP64 sums
 * of the same terms in another order: equal to the energy kernel's to
 * rounding), so samples do not break the pairing of steps; otherwise a sample
 * is a separate pass over the state and a sample at n+1 leaves step n
 * single. */
tete_status tete_set_diagnostics(tete_grid* g, int32_t every);

/* e_z probes recorded after every step (e_z^{n+1/2}); idx are HOST array
 * indices into the e_z array (0 <= idx < np), np_ <= TETE_MAX_PROBES.  Probes
 * leave steps paired: for the state a two-step launch passes through, the
 * probes' e_z is evaluated from the launch's input (S1-S3 at each probe edge,
 * the arithmetic of the step). */
tete_status tete_set_probes(tete_grid* g, const int64_t* idx, int32_t np_);

/* Enqueue nsteps steps of scheme (23) on the grid's stream (asynchronous).
 * Errors: TETE_ERR_ARG (nsteps < 0), TETE_ERR_STATE (series full while
 * recording), TETE_ERR_DEVICE (launch failure). */
tete_status tete_step(tete_grid* g, int64_t nsteps);

/* Number of completed steps (host counter, no synchronisation). */
tete_status tete_steps_done(tete_grid* g, int64_t* n);

/* The grid's sticky error state (see "Error state" above): TETE_OK or
 * TETE_ERR_NONFINITE.  Host only, no synchronisation. */
tete_status tete_grid_status(tete_grid* g);

/* Longitudinal wake potential (Sec. 5) W(s_j) = -(1/Q) int E_z dz at
 * t = (z + s)/c on the bunch line, in V/C, for the nw samples of the bunch
 * (HOST array W of at least nw doubles).  Sample j is complete once step
 * kend - 1 + half_cells + j has run (kend = nz, or the end an open-pipe run
 * set).  Synchronises the stream. */
tete_status tete_wake(tete_grid* g, double* W, int32_t nw);

/* Open entrance and exit pipes.  The structure of Sec. 5 lies between
 * infinitely long ingoing and outgoing pipes; the paper gives no method for
 * them, and this call emulates both on the closed grid of scheme (23):
 *
 * Entrance.  The state y^n0, n0 = start_step, becomes the field that the
 * bunch of tete_set_bunch carries through a uniform pipe, and the step
 * counter becomes n0, so that the bunch centre sits on edge n0 - half_cells,
 * inside the grid, with its field in place; the entrance wall sees no
 * transition.  With p = k - n:
 *   e_x = -(P_x phi) F(p), e_y = -(P_y phi) F(p) (plane k, time n),
 *   h_x = (dx/dy)(P_y phi) F(p+1), h_y = -(dy/dx)(P_x phi) F(p+1)
 *   (plane k + 1/2, time n - 1/2), e_z = h_z = 0,
 * where phi solves the cross-section's 5-point problem
 *   (dy/dx)(2 phi - phi(i+1,j) - phi(i-1,j)) + (dx/dy)(2 phi - phi(i,j+1) - phi(i,j-1))
 *   = 1 at (i0, j0), 0 at the other nodes whose e_z edge is not PEC,
 * phi = 0 on the PEC nodes (conjugate gradients in FP64 to a residual of
 * 1e-16), and (F(p) + F(p+1))/2 = lam_{p+M}/dtau is the bunch current
 * (cell p + M crosses edge k in step n), F(p) = 0 for p > 0.  The scheme
 * carries this state one cell per step while the pipe stays uniform: e_z and
 * h_z stay 0 to rounding.  Below the bunch F continues as a checkerboard of
 * the truncated bunch's alternating charge sum (a free wave without charge);
 * the entrance wall cuts it, which samples j >= n0 - half_cells - 1 feel at
 * the level of the last bunch cell's charge.
 *
 * Exit.  The wake quadrature (tete_wake, tete_witness_wake) ends before edge
 * kend (0: nz).  A field reflected by the exit wall reaches edge k no earlier
 * than step 2 nz - k, and sample j meets edge k in step k + half_cells + j,
 * so samples j <= 2 (nz - kend) - half_cells - 2 never meet a reflection.
 *
 * Requires: a bunch; an explicit TE/TM grid without TETE_F_MATERIALS (the
 * pipe is vacuum with PEC walls); cell planes 0 .. n0 uniform in z (the codes
 * of every node line repeat plane 0's, e_x and e_y from plane 1), the bunch
 * node not on PEC; 0 <= n0 < nz, 0 <= kend <= nz.  The other field set and
 * the witness accumulators serve as scratch; the wake and witness
 * accumulators, series and sticky error are reset, as by tete_set_fields.
 * tete_set_fields, tete_set_bunch, tete_clear_bunch and tete_set_pec_cells
 * end the open-pipe run (the quadrature takes all edges again).
 * *iterations (may be NULL) receives the conjugate-gradient iterations.
 * Synchronises the stream.  Errors: TETE_ERR_ARG (ranges, a non-uniform
 * entrance pipe, the bunch node on PEC), TETE_ERR_STATE (no bunch, a Yee,
 * implicit or materials grid, or no convergence). */
tete_status tete_set_open_pipes(tete_grid* g, int64_t start_step, int32_t kend, int32_t* iterations);

/* Witness lines: off-axis and transverse wakes (Sec. 5 with the Panofsky-
 * Wenzel theorem).  The longitudinal wake of tete_wake is also sampled, with
 * the same quadrature, samples s_j and normalisation, on the e_z node lines
 * through (iw, jw), (iw-1, jw), (iw+1, jw), (iw, jw-1) and (iw, jw+1), for
 * 1 <= iw <= nx-1, 1 <= jw <= ny-1; the bunch line (i0, j0) may be another.
 * Requires a bunch (TETE_ERR_STATE otherwise); resets the witness
 * accumulators, as do tete_set_bunch and tete_set_fields.  A two-step launch
 * also keeps e_z^{n+1/2} of the five lines (in the workspace; the FP32 32-row
 * shape then runs as 16 rows), and a small kernel over the lines adds both
 * steps' terms after it; a single step is followed by the same kernel for
 * one step.  The results do not depend on the kernel.  A grid with a
 * witness cannot join a batch, and a batch with a member that has one does
 * not step (TETE_ERR_STATE from tete_batch_set / tete_batch_step).  Errors:
 * TETE_ERR_ARG (range). */
tete_status tete_set_witness(tete_grid* g, int32_t iw, int32_t jw);

/* Stop sampling the witness lines. */
tete_status tete_clear_witness(tete_grid* g);

/* Witness wakes for nw samples (1 <= nw <= the bunch's nw), HOST arrays:
 * W[l * nw + j] = W_par(s_j) on line l in the order of tete_set_witness
 * (witness node first), in V/C.  Wx, Wy (either may be NULL; nw doubles
 * each): the transverse wake at the witness node, W_perp(s_j) = integral
 * from s_jmin to s_j of grad_perp W_par ds, the gradient by centred
 * differences over 2 dx (2 dy) and the integral by the trapezoid rule, zero
 * at the first sample (choose jmin ahead of the bunch, jmin <= -half_cells,
 * so that the integral starts before any wake), in V/C; W_perp is the
 * integral of (E + v x B)_perp along the witness path over Q.  Sample j is
 * complete once step kend - 1 + half_cells + j has run (kend as for
 * tete_wake).  Synchronises the stream.  TETE_ERR_STATE without a bunch or
 * witness. */
tete_status tete_witness_wake(tete_grid* g, double* W, double* Wx, double* Wy, int32_t nw);

/* Static tiles of a TETE_F_SKIP_STATIC grid for its current geometry (or
 * materials): *skipped of *total tiles lie wholly in PEC, for the tiling of
 * the two-step kernel where tete_step pairs steps, else (no two-step kernel,
 * or an energy sample before every step) for the fused single step's.  The
 * two kinds keep separate tables.  Builds the table if needed; synchronises
 * the stream.  TETE_ERR_STATE without the flag. */
tete_status tete_static_tiles(tete_grid* g, int64_t* skipped, int64_t* total);

/* Discrete energy W^{n,e} = 1/2 <Q^e y^n, y^n> (Sec. 4.4) of the current
 * state, FP64, internal units (joules = W / eps0 with charge in coulombs);
 * *n = steps done.  Synchronises.  TETE_ERR_NONFINITE if the sum is not finite. */
tete_status tete_energy(tete_grid* g, double* W, int64_t* n);

/* tete_energy for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same value by the same kernels, with the reduction's partial sums and
 * result in a file-scope device array of the library instead of the grid's
 * workspace.  That array holds RED_BLOCKS = 2048 partial sums and the result
 * (16,448 bytes; each GPU the library runs on keeps its own copy until the
 * process ends); the reduction uses 2048 partial sums for every grid, so
 * every grid tete_check_desc accepts fits and no size is rejected.  The call
 * allocates nothing (no hipMalloc, hipFree or other allocating routine); its
 * address is looked up once per device, on the first call there.  Every
 * partial sum and the result are written before they are read, so nothing
 * needs clearing; calls that overlap on one GPU (other host threads, other
 * streams) share the array and race.  Synchronises the grid's stream.
 * Errors as tete_energy. */
tete_status tete_energy_noalloc(tete_grid* g, double* W, int64_t* n);

/* Copy the energies recorded during tete_step (see tete_set_diagnostics):
 * out[0..count-1] in step order, *count = entries recorded (<= max).  Synchronises. */
tete_status tete_energy_series(tete_grid* g, double* out, int64_t max, int64_t* count);

/* Copy the probe series: out[s * nprobes + p] for recorded steps s, HOST
 * array of max entries; *count = steps recorded.  Synchronises. */
tete_status tete_probes(tete_grid* g, double* out, int64_t max, int64_t* count);

/* Conserved charges of Sec. 4.5 after the last step n (needs >= 1 step since
 * the last tete_set_fields): max over nodes whose six edges are non-PEC of
 * |q_e^{n+1/2} - bunch charge of the node's dual cell| (eq. (35)), and max over
 * cells of |q_h^n| (eq. (34)), both FP64 in coulombs / internal flux units.
 * Synchronises.  TETE_ERR_STATE if no step has run. */
tete_status tete_charges(tete_grid* g, double* max_res_e, double* max_abs_h);

/* Kernel choice and launch shape (for tuning; results do not depend on it
 * beyond rounding order, and the fused kernels give identical results).
 * kernel:
 *   TETE_KERNEL_AUTO   the two-step kernel, or the fused single step with
 *                      per-entry materials it has no instance for (FP64
 *                      arrays, arrays with witness lines or the static-tile
 *                      skip);
 *   TETE_KERNEL_FUSED  the fused single-kernel step (with per-entry
 *                      materials: its materials instance, default rows and
 *                      one prefetched plane, the coefficients read with the
 *                      fields and carried to the sub-updates' planes);
 *   TETE_KERNEL_FUSED2 two steps per launch, temporally blocked
 *                      (TETE_ERR_STATE with FP64 per-entry arrays or arrays on a
 *                      TETE_F_SKIP_STATIC grid; materials by class and FP32
 *                      arrays use it).  tete_step
 *                      pairs consecutive steps except where an energy sample
 *                      needs the state in between; those steps, and
 *                      an odd last one, run as fused single steps;
 *   TETE_KERNEL_SPLIT  the two-kernel step (one kernel per half step).
 * rows: rows per workgroup of the fused single step, 12 or 16 (0: 16 for
 * FP32, 12 for FP64); of the two-step kernel, 16 (16 rows of 64 lanes for
 * FP32, of 32 lanes for FP64, the default) or 32 (FP32: 32 rows of 32
 * lanes); 32 leaves the single step at its default.  xchunk: x-planes
 * per workgroup of either fused kernel (0: chosen from the grid size).
 * depth: x-planes of old data the fused single step prefetches ahead, 1..3
 * (0: 2; the two-step kernel prefetches one).  order: order in which the
 * fused kernels' tiles are scheduled: 1 (j-tiles first), 2 (k-tiles first),
 * 3, 4, 5 or 6 (blocks of 8 k-tiles by 4 j-tiles, 16 by 2, 4 by 8 or 2 by
 * 16); 0: 4 where the grid has at least 16 k-tiles and 2 j-tiles and the
 * launch at least 2048 workgroups, else 2 (batches: 2).  tete_set_materials
 * turns a forced FUSED or FUSED2 back into AUTO.  tete_get_tuning reports the kernel
 * that tete_step will use (FUSED2, FUSED or SPLIT). */
enum { TETE_KERNEL_AUTO = 0, TETE_KERNEL_FUSED = 1, TETE_KERNEL_SPLIT = 2, TETE_KERNEL_FUSED2 = 3,
       TETE_KERNEL_YEE = 4 /* reported for TETE_F_YEE grids: two steps per launch
                            * (bitwise two single steps) unless kernel is
                            * TETE_KERNEL_FUSED (single steps); rows and depth
                            * are ignored */,
       TETE_KERNEL_IMPLICIT = 5 /* reported for TETE_F_IMPLICIT grids */ };
typedef struct {
    int32_t kernel;
    int32_t rows;
    int32_t xchunk;
    int32_t depth;
    int32_t order;
} tete_tuning;
tete_status tete_set_tuning(tete_grid* g, const tete_tuning* t);
tete_status tete_get_tuning(tete_grid* g, tete_tuning* t);

/* Live kernel timing for measurement.  max_steps > 0 arms up to max_steps
 * timed launches: each subsequent launch records HIP events on the grid's
 * stream around its kernels (fused step: one kernel; two-step kernel: one
 * kernel for two steps; two-kernel step: TM-like half S1-S5 with the source
 * and wake update, then TE-like half S6-S10).  0 disarms.  Synchronises.
 * Launches beyond the armed count fail with TETE_ERR_STATE. */
tete_status tete_set_timing(tete_grid* g, int64_t max_steps);

/* Sum of the kernel durations of the timed launches since the last call, in
 * ms: two-kernel step: ms[0] = TM-like kernel, ms[1] = TE-like kernel; fused
 * kernels: ms[0] = the kernel, ms[1] = 0 (nphase >= 2); *steps = number of
 * time steps the timed launches took (so ms[0] / *steps is the time per
 * step).  Resets the count.  Synchronises. */
tete_status tete_timing(tete_grid* g, double* ms, int32_t nphase, int64_t* steps);

/* ------------------------------------------------------------------------
 * Batches: many grids (of one precision, uneven sizes, own geometries and
 * bunches) stepped together, one persistent launch per time step (FP32: per
 * two time steps, with the two-step kernel) covering every member's tiles;
 * blocks of steps are replayed from a captured HIP graph.  A batch owns a small device table (tete_batch_bytes) in caller
 * memory; membership can change between calls (continuous batching) without
 * re-capturing the graph.  Members use the fused kernel (no per-entry
 * materials) with their own x-chunk and tile order (tete_set_tuning); energy
 * series and probes are not recorded for batched steps.  A member's results
 * are the same as stepping it alone (each entry is computed by the same
 * expressions).  The steps run on a private stream of the batch, ordered
 * after the work already enqueued on the batch's stream and before anything
 * enqueued there later (HIP events), so the batch's stream may be the null
 * stream.  All work is ordered on the batch's stream; the caller must
 * order work on the members' streams before and after (using one stream for
 * everything does that).  A member must not be stepped alone while a batch
 * step is in flight.
 * ---------------------------------------------------------------------- */
typedef struct tete_batch tete_batch;

/* Device table bytes of a batch of the given precision (0 if invalid). */
size_t tete_batch_bytes(int32_t precision);

/* Create a batch over a caller-owned device table (256-byte aligned, at least
 * tete_batch_bytes(precision)), using hip_stream.  Empty, launch shape:
 * automatic kernel, rows chosen by precision, prefetch depth 1, graph blocks
 * of 8 steps. */
tete_status tete_batch_create(int32_t precision, void* dev_table, size_t bytes, void* hip_stream,
                              tete_batch** out);
tete_status tete_batch_destroy(tete_batch* b);

/* Put grid g into slot (0 <= slot < TETE_MAX_BATCH), or empty the slot with
 * g = NULL.  TETE_ERR_ARG: wrong precision or device, or g already in
 * another slot; TETE_ERR_STATE: g has per-entry materials or planes too large
 * for the fused kernel.  Changing a member (its fields, bunch or tuning)
 * requires setting its slot again before the next batch step. */
tete_status tete_batch_set(tete_batch* b, int32_t slot, tete_grid* g);

/* Launch shape shared by the members.  kernel: TETE_KERNEL_AUTO (two steps
 * per launch where every member fits the two-step kernel, else single
 * steps), TETE_KERNEL_FUSED (single steps) or TETE_KERNEL_FUSED2 (as AUTO);
 * a block of an odd number of steps ends with a single step.  rows (0, 12 or 16) and prefetch depth (0..3, 0 = 1)
 * of the single-step kernel; steps per captured graph block (0 = no graph).
 * With the two-step kernel a member uses its own tile order and, if its
 * tuning asks for TETE_KERNEL_FUSED2, its own x-chunk. */
tete_status tete_batch_set_launch(tete_batch* b, int32_t kernel, int32_t rows, int32_t depth,
                                  int32_t graph_steps);

/* Enqueue nsteps steps of every member (asynchronous).  Each member's step
 * counter advances by nsteps, as if tete_step had been called on it. */
tete_status tete_batch_step(tete_batch* b, int64_t nsteps);

/* Number of occupied slots. */
tete_status tete_batch_count(tete_batch* b, int32_t* active);

/* ---------------------------------------------------------------------------
 * Rotationally symmetric structures: scheme (24) of Sec. 4.3 for one azimuthal
 * harmonic m on an r-z grid.
 *
 * Grid: nr x nz cells, node (j, k) at (r, z) = (j dr, k dz), j = 0 on the
 * axis, PEC walls at r = nr dr and at z = 0, nz dz.  The azimuthal derivative
 * of harmonic m is taken exactly (P_phi -> m), so every FIT quantity is per
 * radian: e^ = E * edge length per radian, h^ = H * dual-edge length per radian.
 * Six arrays of (nr+1)(nz+1) entries, z fastest: index = k + (nz+1) j.  Order
 * in the [6] arguments: e_phi, e_r, e_z, h_phi, h_r, h_z at
 *   e_phi (j, k)   e_r (j+1/2, k)   e_z (j, k+1/2)
 *   h_phi (j+1/2, k+1/2)   h_r (j, k+1/2)   h_z (j+1/2, k).
 * Material matrices (vacuum, per radian): kappa = edge / dual facet, mu =
 * dual edge / facet; the dual facet of the on-axis e_z edge is the disk of
 * radius dr/2 (area dr^2/8 per radian) and exists for m = 0 only; e_phi has
 * no length on the axis.  The implicit factors of (24) are taken on the
 * e_z / h_r and h_z / e_r positions: (1 + a^2 m^2 kappa_z mu_r)^-1 on e_z and
 * (1 + a^2 m^2 mu_z kappa_r)^-1 on h_z, a = cdt/2.
 *
 * Stability (Sec. 4.4): cdt <= dz and cdt <= dr for every m >= 1 (independent
 * of m); for m = 0 the on-axis cell limits cdt to 0.9089 dr (largest
 * eigenvalue 4.8419/dr^2 of the radial operator next to the axis).
 *
 * Memory, streams and errors as for tete_grid: caller-owned 256-byte aligned
 * device workspace, caller's HIP stream, bulk arrays are DEVICE pointers,
 * small results HOST pointers.
 * ------------------------------------------------------------------------- */
typedef struct tete_rz tete_rz; /* opaque handle */

typedef struct {
    int32_t nr, nz;       /* cells, each >= 2; (nr+1)(nz+1) < 2^31 */
    double dr, dz;        /* cell sizes [m] */
    double cdt;           /* dtau [m]: <= dz, <= dr (m >= 1) or <= 0.9089 dr (m = 0) */
    int32_t mode;         /* azimuthal harmonic m, 0 <= m <= 4096 */
    int32_t precision;    /* TETE_FP64 or TETE_FP32 */
} tete_rz_desc;

/* Size and stability check of a descriptor (host only).  TETE_OK,
 * TETE_ERR_ARG or TETE_ERR_UNSTABLE (the bounds above). */
tete_status tete_rz_check_desc(const tete_rz_desc* desc);

/* Device workspace bytes of an r-z grid (0 if the descriptor is invalid). */
size_t tete_rz_workspace_bytes(const tete_rz_desc* desc);

/* Create an r-z grid on the current device inside dev_ws (256-byte aligned,
 * ws_bytes >= tete_rz_workspace_bytes), stream hip_stream (NULL = null
 * stream).  Fields zero, empty vacuum PEC pillbox, no bunch, counter 0.
 * Errors: TETE_ERR_ARG, TETE_ERR_UNSTABLE, TETE_ERR_NOMEM, TETE_ERR_DEVICE. */
tete_status tete_rz_create(const tete_rz_desc* desc, void* dev_ws, size_t ws_bytes, void* hip_stream,
                           tete_rz** out);

/* Release the host handle (the workspace stays the caller's). */
tete_status tete_rz_destroy(tete_rz* g);

/* Staircase geometry: DEVICE array of nr*nz bytes, index k + nz*j, non-zero =
 * PEC cell (j+1/2, k+1/2).  An edge is PEC if any adjacent cell is; cells
 * outside r < nr dr and 0 < z < nz dz are PEC, the axis is not a wall (the
 * cell row j = -1 mirrors j = 0).  NULL = empty pillbox.  Zeroes e on the new
 * PEC edges.  Copies; the caller keeps its array. */
tete_status tete_rz_set_pec_cells(tete_rz* g, const uint8_t* cell_is_pec);

/* Initial state y^0 = (u^{-1/2}, v^0), u = (h_phi, h_r, e_z) at tau = -cdt/2
 * and v = (e_phi, e_r, h_z) at tau = 0 (DEVICE arrays, dtype TETE_FP64 or
 * TETE_FP32).  Out-of-range entries and e on PEC edges are stored as zero.
 * Resets the step counter and the wake accumulators. */
tete_status tete_rz_set_fields(tete_rz* g, const void* const f[6], int32_t dtype);

/* Copy the current state y^n into DEVICE arrays f[6] of dtype. */
tete_status tete_rz_get_fields(tete_rz* g, void* const f[6], int32_t dtype);

/* Ring bunch of the grid's harmonic m (Sec. 5 charge model; a point charge's
 * harmonic m carries the weight 1/(2 pi) per radian for m = 0 and 1/pi for
 * m >= 1): total charge charge_C, RMS length sigma_z, moving at v = c along
 * +z at radius j0 dr (0 <= j0 < nr; j0 = 0, the axis, for m = 0 only).  Cells,
 * timing and wake samples s_j = j dz (j = jmin .. jmin+nw-1) as for
 * tete_set_bunch.  The wake is sampled on the two e_z lines j = jw and jw+1
 * (0 <= jw < nr - 1; jw >= 1 for m >= 1).  Requires cdt == dz.  Resets the
 * wake accumulators.  Errors: TETE_ERR_ARG, TETE_ERR_STATE (cdt != dz). */
typedef struct {
    double charge_C;
    double sigma_z;       /* [m] */
    int32_t j0;           /* radius index of the ring */
    int32_t half_cells;   /* M, 2M+1 <= TETE_MAX_BUNCH_CELLS */
    int32_t jw;           /* first wake line */
    int32_t jmin;
    int32_t nw;           /* <= TETE_MAX_WAKE */
} tete_rz_bunch;
tete_status tete_rz_set_bunch(tete_rz* g, const tete_rz_bunch* b);

/* Enqueue nsteps steps of (24) (asynchronous; one or two steps per launch).
 * Errors: TETE_ERR_ARG (nsteps < 0), TETE_ERR_DEVICE. */
tete_status tete_rz_step(tete_rz* g, int64_t nsteps);

/* Open entrance and exit pipes for the r-z grid (the construction of
 * tete_set_open_pipes for scheme (24)).  The state of step start_step
 * becomes the ring bunch's own field in the uniform entrance pipe:
 *   e_phi = -m Phi_j F(p), e_r = -(Phi_{j+1} - Phi_j) F(p),
 *   h_phi = (r_{j+1/2}/dr)(Phi_{j+1} - Phi_j) F(p+1), h_r = (dr/r_j) e_phi-shape F(p+1),
 *   e_z = h_z = 0, p = k - n,
 * where Phi solves the radial problem
 *   [r_{j-1/2}(Phi_j - Phi_{j-1}) - r_{j+1/2}(Phi_{j+1} - Phi_j)]/dr + m^2 (dr/r_j) Phi_j = delta_{j, j0}
 * on the nodes whose e_z edge is free (r_{-1/2} = 0; Phi = 0 on the wall,
 * on PEC nodes and, for m >= 1, on the axis; a tridiagonal solve in FP64)
 * and F carries the ring current as in 3-D.  The wake quadrature (both
 * lines) ends before edge kend (0: nz).  Requires a bunch (TETE_ERR_STATE);
 * cell planes 0 .. start_step uniform in z and the ring's node free, 0 <=
 * start_step < nz, 0 <= kend <= nz (TETE_ERR_ARG otherwise).  The other field
 * set and the wake read-out area serve as scratch; the step counter becomes
 * start_step and the wake accumulators are reset.  tete_rz_set_fields,
 * tete_rz_set_bunch and tete_rz_set_pec_cells end the open-pipe run.
 * Synchronises the stream. */
tete_status tete_rz_set_open_pipes(tete_rz* g, int64_t start_step, int32_t kend);

/* Number of completed steps (host counter). */
tete_status tete_rz_steps_done(tete_rz* g, int64_t* n);

/* Wakes of harmonic m (Sec. 5) in V/C, HOST arrays: W_par[0..nw-1] on line
 * jw and W_par[nw..2nw-1] on line jw+1 (W = -(1/Q) int E_z dz at t = (z+s)/c,
 * the 3-D quadrature), and W_perp[0..nw-1] = the radial wake at
 * (r_{jw+1/2}, theta = 0) by the Panofsky-Wenzel relation d/ds W_perp =
 * grad_perp W_par: the trapezoidal integral over s of the lines' difference
 * divided by dr (W_perp may be NULL).  Synchronises. */
tete_status tete_rz_wake(tete_rz* g, double* W_par, double* W_perp, int32_t nw);

/* Discrete energy 1/2 <Q y^n, y^n> of (24) (Q = B^{e,r} - alpha A: the 3-D form
 * of Sec. 4.4 with only the radial part of the splitting operator), FP64,
 * internal units, per radian; *n = steps done.  Synchronises. */
tete_status tete_rz_energy(tete_rz* g, double* W, int64_t* n);

/* Launch tuning of the r-z kernel: kernel TETE_KERNEL_AUTO or
 * TETE_KERNEL_FUSED2 (two steps per launch: a second march stage follows the
 * first two rows behind it in the same wave, so each cell is read and written
 * once per two steps; an odd last step runs alone) or TETE_KERNEL_FUSED (one
 * step per launch); rows per r-chunk (0 = automatic, else 8 .. 4096), rows
 * loaded ahead (0 = automatic, else 1 .. 4) and the workgroup order (0 =
 * automatic, 1 = the r-chunks of a z-column consecutive, 2 = the z-strips of
 * a chunk consecutive).  Results do not depend on it. */
tete_status tete_rz_set_tuning(tete_rz* g, int32_t kernel, int32_t chunk_rows, int32_t prefetch, int32_t order);

/* Live kernel timing: max_launches > 0 records HIP events around each step
 * launch (0 disables); tete_rz_timing returns the summed kernel time [ms],
 * the launches recorded and the steps they took.  Synchronises. */
tete_status tete_rz_set_timing(tete_rz* g, int64_t max_launches);
tete_status tete_rz_timing(tete_rz* g, double* ms, int64_t* launches, int64_t* steps);

/* ------------------------------------------------------------------------
 * Measurement aid: the HBM ceiling of the step's access pattern.  One launch
 * reads six arrays of n entries of dtype and n code bytes and writes six
 * arrays: out[c][i] = in[c][i] (0 where bit 7 of code[i] is set, which the
 * library's PEC codes never have), every access a coalesced 16-byte load or
 * store.  The fused kernels move the same arrays (per launch: six fields
 * and the codes read, six fields written), so this kernel's rate bounds
 * theirs from above on the hardware.  DEVICE arrays, in/out 16-byte and code
 * 4-byte aligned; in and out must not overlap.  Asynchronous on hip_stream.
 * Errors: TETE_ERR_ARG, TETE_ERR_DEVICE.
 * ---------------------------------------------------------------------- */
tete_status tete_stream_probe(void* const in[6], void* const out[6], const uint8_t* code, int64_t n,
                              int32_t dtype, void* hip_stream);

/* Human-readable status name. */
const char* tete_status_str(tete_status s);

#ifdef __cplusplus
}
#endif
#endif /* TETE_H */
