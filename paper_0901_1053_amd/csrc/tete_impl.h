// Internal declarations shared by the host runtime and the kernel translation
// units of libtete.  Not part of the public ABI (include/tete.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tete.h"

namespace tete {

// Grid geometry as the kernels see it.  Arrays are (nx+1)(ny+1)(nz+1), z
// fastest; sz = nz+1 is the row length, sp = (ny+1)(nz+1) the plane length.
struct Geo {
    int nx, ny, nz;
    int sz;      // nz + 1
    int sp;      // (ny + 1) * (nz + 1)
    int np;      // (nx + 1) * sp
};

// Six field components of one time level.
template <typename R>
struct Fields {
    R* c[6];     // ex, ey, ez, hx, hy, hz
};

// Material description: vacuum scalars with PEC codes, or per-entry arrays;
// with materials by class also the class bytes and the class table that the
// two-step kernel reads instead of the arrays (the arrays hold the same
// values, expanded).
template <typename R>
struct Mat {
    const uint8_t* code;   // bit0: e_x PEC/absent, bit1: e_y, bit2: e_z
    const R* arr[6];       // kappa_x,y,z, mu_x,y,z per entry (nullptr: vacuum)
    R k[3], m[3];          // vacuum kappa_x,y,z and mu_x,y,z
    const uint8_t* cls;    // class per entry (nullptr: no classes)
    const R* ctab;         // class table, TETE_MAX_CLASSES x CLS_STRIDE
};

// Class table entries (per class, CLS_STRIDE values of the field type): the
// coefficients of the sub-updates multiplied by their factor, as the step
// kernels form them, and kappa_z alone for the bunch current.
enum { CLS_AMX = 0, CLS_AMY = 1, CLS_A2MZ = 2, CLS_A2KZ = 3, CLS_AKY = 4, CLS_AKX = 5, CLS_KZ = 6, CLS_STRIDE = 8 };
// Slots of the hash table that recognises classes in per-entry arrays
// (a power of two, twice the classes a grid may have)
enum { CLS_SLOTS = 2 * TETE_MAX_CLASSES };

// Rigid-bunch source and wake accumulator for one step.
struct Src {
    int on;
    int i0, j0, M;
    int64_t n;           // index of the step being taken
    const double* lam;   // 2M+1 cell charges
    double* wacc;        // wake accumulator (FP64)
    int jmin, nw;
    int kend;            // the wake quadrature takes edges k < kend (nz, or the end of an open-pipe run)
};

enum { RED_BLOCKS = 2048, RED_THREADS = 256 };

// Witness lines (tete_set_witness): array offset of (i, j, 0) of each e_z
// node line
struct Witness {
    int64_t base[TETE_WITNESS_LINES];
};
// e_z^{n+1/2} of the witness lines, kept by the two-step kernel for the line
// kernel that runs after it: mid[l * nz + k], lines l in the order (iw, jw),
// (iw-1, jw), (iw+1, jw), (iw, jw-1), (iw, jw+1)
template <typename R>
struct WitMid {
    R* mid;
    int iw, jw;
};

// Arguments of one grid's fused step: old and new fields, PEC codes, vacuum
// coefficients, source, and the tiling (tete_fused.hip).
template <typename R>
struct FArgs {
    const R* ex; const R* ey; const R* ez; const R* hx; const R* hy; const R* hz;
    R* ex1; R* ey1; R* ez1; R* hx1; R* hy1; R* hz1;
    const uint8_t* code;
    // materials by class (or null): one class byte per entry and the class
    // table, TETE_MAX_CLASSES x CLS_STRIDE values (CLS_* order, already
    // multiplied by their factor a or 2a)
    const uint8_t* cls;
    const R* ctab;
    Geo g;
    R a, kx, ky, kz, mx, my, mz;
    Src src;
    int nyt, nzt, nxc, xchunk;   // tiles along j, k; chunks along x; planes per chunk
    int order;                   // tile order
    int nblk;                    // work items (workgroups) of one step
};

// Device-resident table of a batch (tete_batch_*): the active instances, their
// work-item offsets, step indices, and kernel arguments for both ping-pong
// parities (a[q] is used when (phase + launches so far in the block) % 2 ==
// q): a for the single step, a2 for the two-step kernel (FP32 batches).
template <typename R>
struct BatchItem {
    FArgs<R> a[2];
    FArgs<R> a2[2];
};
template <typename R>
struct BatchTable {
    int ninst;                         // active instances (compacted)
    int total;                         // work items of one single step, all instances
    int total2;                        // work items of one two-step launch
    int phase;                         // parity of the launches taken so far
    int offset[TETE_MAX_BATCH + 1];    // first work item of each instance (single step)
    int offset2[TETE_MAX_BATCH + 1];   // first work item of each instance (two-step kernel)
    int64_t step[TETE_MAX_BATCH];      // step index n of each instance
    BatchItem<R> item[TETE_MAX_BATCH];
};

// ---- launchers (tete_kernels.hip) ---------------------------------------
hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_zero_bytes(void* p, size_t bytes, hipStream_t s);
hipError_t launch_build_codes(uint8_t* code, const uint8_t* cells, Geo g, hipStream_t s);
hipError_t launch_lambda(double* lam, double Q, double sigma, double dz, int M, hipStream_t s);

template <typename R>
hipError_t launch_import(Fields<R> dst, const void* const src[6], int src_fp32, Mat<R> mat, Geo g,
                         hipStream_t s);
template <typename R>
hipError_t launch_export(void* const dst[6], int dst_fp32, Fields<R> src, Geo g, hipStream_t s);
template <typename R>
hipError_t launch_import_materials(R* const dst[6], const void* const src[6], int src_fp32, Geo g,
                                   hipStream_t s);
template <typename R>
hipError_t launch_zero_pec(Fields<R> f, Mat<R> mat, Geo g, hipStream_t s);

// One step; ev (optional) receives three events: before the TM kernel,
// between the TM and TE kernels, after the TE kernel.
template <typename R>
hipError_t launch_step(Fields<R> oldf, Fields<R> newf, Mat<R> mat, Geo g, R alpha, Src src,
                       hipStream_t s, hipEvent_t* ev);

// Fused single-kernel step for vacuum + PEC codes (tete_fused.hip); rows = 12
// or 16 rows per workgroup, xchunk = planes per workgroup (0: automatic),
// depth = planes of old data prefetched ahead (1..3), order = tile order
// of the workgroups (0..2).
// Whether a grid's planes are small enough for the fused kernel's buffer
// addressing (five planes below 2^31 bytes).
bool fused_fits(Geo g, int real_bytes);
// act (or nullptr): the nact active tiles of fused_static_tiles for the same
// rows, xchunk and order
template <typename R>
hipError_t launch_step_fused(Fields<R> oldf, Fields<R> newf, Mat<R> mat, Geo g, R alpha, Src src, int rows,
                             int xchunk, int depth, int order, hipStream_t s, hipEvent_t* ev, const int* act,
                             int nact);
// Bytes a static-tile table of the materials step needs at most.
int64_t fused_tile_cap(Geo g);
// The static-tile table (tab) and the active tiles (act, *nact of them) of the
// single step for the tiling (rows, xchunk, order): with kap (kappa_x,
// kappa_y, kappa_z; the materials instance, default rows) static where kappa
// is zero on every e edge the tile loads, else where every loaded PEC code is
// 7.  Synchronises the stream.
template <typename R>
hipError_t fused_static_tiles(const R* const kap[3], const uint8_t* code, Geo g, int rows, int xchunk, int order,
                              uint8_t* tab, int* act, int64_t cap, int64_t* ntiles, int* nact, hipStream_t s);

template <typename R>
FArgs<R> fused_args(Fields<R> oldf, Fields<R> newf, Mat<R> mat, Geo g, R alpha, Src src);
// Fills the tiling of A for a launch shape; false if the shape is invalid or
// the grid's planes are too large for the fused kernel.
template <typename R>
bool fused_setup(FArgs<R>& A, int rows, int xchunk, int order);
int fused_default_rows(int real_bytes);
// Two steps in one launch (tete_fused2.hip): the fused step temporally
// blocked; xchunk and order as for the single step.
bool fused2_fits(Geo g, int real_bytes);
// rows: 0 (default), 16, or 24 or 32 (FP32 only: rows of 32 lanes).
template <typename R>
bool fused2_setup(FArgs<R>& A, int rows, int xchunk, int order, int lanes = 0);
// Energy samples taken by a two-step launch: want bit 0 the energy of its
// input y^n, bit 1 that of y^{n+1}; written to out[0], out[1] (only the ones
// wanted, in that order); part: cap pairs of FP64 partial sums.
struct EnergyPair {
    int want;
    double alpha;
    double* part;
    int64_t cap;
    double* out;
    const double* craw;   // materials by class: kappa_x .. mu_z per class (FP64), else nullptr
};
// wm (or nullptr): the witness lines whose e_z^{n+1/2} the launch keeps;
// act (or nullptr): the nact active tiles of fused2_static_tiles for the same
// rows (0 with wm), xchunk and order; the launch takes only these (none if
// nact is 0), and with wm stores witness values only in them; en (or
// nullptr, or want 0): energy samples, with vacuum coefficients only, in
// their own shape (16 rows of 32 lanes; the rows and depth asked for do not
// apply; hipErrorInvalidValue otherwise, or when the launch has more
// workgroups than en->cap)
template <typename R>
hipError_t launch_step_fused2(Fields<R> oldf, Fields<R> newf, Mat<R> mat, Geo g, R alpha, Src src,
                              const WitMid<R>* wm, int rows, int depth, int xchunk, int order, hipStream_t s,
                              hipEvent_t* ev, const int* act, int nact, const EnergyPair* en = nullptr);
// workgroups of a two-step launch that takes energy samples
template <typename R>
int64_t fused2_blocks(Geo g, int xchunk, int order);
// out[0] = sum of part[t * stride], t < n, in a fixed order (FP64)
hipError_t launch_sum(const double* part, int n, int stride, double* out, hipStream_t s);
// One byte per tile of the two-step kernel's tiling (rows, xchunk) in tab: 1
// where every entry the tile loads has its three e edges PEC, so that a step
// leaves the tile's entries unchanged; and in act the *nact other tiles in the
// launch order of the tile order `order`.  *ntiles = tiles (at most cap; act
// holds cap ints).  Synchronises the stream.
// Bytes a static-tile table needs at most, over every tiling.
int64_t fused2_tile_cap(Geo g);
template <typename R>
hipError_t fused2_static_tiles(const uint8_t* code, Geo g, int rows, int xchunk, int order, uint8_t* tab, int* act,
                               int64_t cap, int64_t* ntiles, int* nact, hipStream_t s);
// One step of Yee's scheme (7) (tete_yee.hip): state (e^{n-1/2}, h^n),
// dtau = 2 alpha; xchunk and order as for the fused step.
bool yee_fits(Geo g, int real_bytes);
template <typename R>
hipError_t launch_step_yee(Fields<R> oldf, Fields<R> newf, Mat<R> mat, Geo g, R alpha, int xchunk, int order,
                           hipStream_t s, hipEvent_t* ev);
// Two steps of Yee's scheme per launch, temporally blocked (bitwise two
// single steps)
bool yee2_fits(Geo g, int real_bytes);
template <typename R>
hipError_t launch_step_yee2(Fields<R> oldf, Fields<R> newf, Mat<R> mat, Geo g, R alpha, int xchunk, int order,
                            hipStream_t s, hipEvent_t* ev);
// One step of every instance of a batch (persistent grid of `grid`
// workgroups), the launch after `flips` earlier launches and `steps` earlier
// steps of the current block
template <typename R>
hipError_t launch_batch_step(BatchTable<R>* T, int rows, int depth, int grid, int flips, int steps, hipStream_t s);
// Two steps of every instance of a batch (tete_fused2.hip)
template <typename R>
hipError_t launch_batch_step2(BatchTable<R>* T, int grid, int flips, int steps, hipStream_t s);
// After a block: step indices += steps, phase += flips (launches)
template <typename R>
hipError_t launch_batch_advance(BatchTable<R>* T, int steps, int flips, hipStream_t s);

// energy of a state -> out[0] (FP64), using partial[RED_BLOCKS]; rw weighs
// the alpha^2 terms of Q (1: explicit scheme (23), 0: implicit scheme (16))
template <typename R>
hipError_t launch_energy(Fields<R> f, Mat<R> mat, Geo g, double alpha, double rw, double* partial, double* out,
                         hipStream_t s);
// Materials by class: table (TETE_MAX_CLASSES x 6 doubles, kappa_x,y,z,
// mu_x,y,z per class) and class bytes cls -> the six per-entry arrays dst (PEC
// codes zero kappa, entries outside a component's range 0) and the class
// table of the step kernels ctab (TETE_MAX_CLASSES x CLS_STRIDE, multiplied
// by alpha or 2 alpha in R).
template <typename R>
hipError_t launch_expand_classes(R* const dst[6], R* ctab, const uint8_t* code, const uint8_t* cls,
                                 const double* table, R alpha, Geo g, hipStream_t s);
// The Gershgorin bound below for materials by class (kappa from the table,
// zero on PEC codes); NaN also for a class byte >= ncls.
// classes in the per-entry arrays arr (tete_set_materials): pass 0 fills the
// hash table keys / vals (CLS_SLOTS each; keys and flags zero before), pass 1
// writes the class byte of every entry from slot_class (the class of each
// slot, -1 for none); flags[0..2]: overflow, kappa on a PEC-coded edge, a
// tuple unlike its slot's
template <typename R>
hipError_t launch_classify(R* const arr[6], const uint8_t* code, Geo g, unsigned long long* keys, double* vals,
                           const int* slot_class, uint8_t* cls, int* flags, int pass, hipStream_t s);
// the step kernels' class table from the table of doubles (TETE_MAX_CLASSES x 6)
template <typename R>
hipError_t launch_class_table(R* ctab, const double* table, R alpha, hipStream_t s);
hipError_t launch_mat_bound_cls(const uint8_t* code, const uint8_t* cls, const double* table, int ncls, Geo g,
                                double alpha, double* partial, double* out, hipStream_t s);
// Largest Gershgorin row sum of the three blocks of Q^e (Sec. 4.4) for
// general materials src[6] (kappa_x,y,z, mu_x,y,z; FP32 if src_fp32) ->
// out[0]: Q^e >= 0 if it is at most 1; NaN if a value in a component's range
// is negative or not finite.  Uses partial[RED_BLOCKS].
hipError_t launch_mat_bound(const void* const src[6], int src_fp32, Geo g, double alpha, double* partial,
                            double* out, hipStream_t s);
// Streaming ceiling of the step's access pattern: out_c = in_c for six arrays
// of n entries (FP32 or FP64, 16-byte aligned), the code byte of each entry
// read as well.
hipError_t launch_stream(void* const in[6], void* const out[6], const uint8_t* code, int64_t n, int fp32,
                         hipStream_t s);
// charges: out[0] = max |q_e - node charge| (interior nodes), out[1] = max |q_h|
template <typename R>
hipError_t launch_charges(Fields<R> oldf, Fields<R> newf, Mat<R> mat, Geo g, double alpha, Src src,
                          double* partial, double* out, hipStream_t s);
template <typename R>
hipError_t launch_probes(const R* ez, const int64_t* idx, int nprobe, double* out, hipStream_t s);
// e_z of the probes after one step from state o (the state a two-step launch
// passes through without storing it), nprobe <= 64
template <typename R>
hipError_t launch_probes_next(Fields<R> o, Mat<R> mat, Geo g, R alpha, Src src, const int64_t* idx, int nprobe,
                              double* out, hipStream_t s);
// wake quadrature of one step n on the witness lines: acc[l * TETE_MAX_WAKE +
// j - jmin] += -1/2 (e_z^{n-1/2} + e_z^{n+1/2}) of edge k < kend, j = n - k - M
template <typename R>
hipError_t launch_witness(const R* ez_old, const R* ez_new, Witness w, Geo g, int64_t n, int M, int jmin, int nw,
                          int kend, double* acc, hipStream_t s);
// the same for steps n and n+1 of one two-step launch, e_z^{n+1/2} from the
// lines' mid buffer (WitMid)
template <typename R>
hipError_t launch_witness2(const R* ez_old, const R* ez_mid, const R* ez_new, Witness w, Geo g, int64_t n, int M,
                           int jmin, int nw, int kend, double* acc, hipStream_t s);

// Work arrays of the implicit scheme's plane solves (np entries each)
template <typename R>
struct ImpWork {
    R* b;        // right-hand side
    R* r;        // residual
    R* d[2];     // Chebyshev directions (ping-pong), zero between solves
    const int* le;   // ascending array indices of the free e_z edges (ne of them)
    const int* lh;   // ascending array indices of the coupled h_z rows (nh)
    int ne, nh;
};
// Row lists of the implicit scheme's plane systems for the current geometry:
// cnt holds 2 ints per chunk (implicit_list_chunks), le and lh np ints each.
// Synchronises the stream.
int implicit_list_chunks(int64_t np);
template <typename R>
hipError_t implicit_build_lists(Mat<R> M, Geo g, int* cnt, int* le, int* lh, int* ne, int* nh, hipStream_t s);
// One step of the implicit scheme (16) (tete_implicit.hip); ev[0..2] around
// the two half steps if not NULL
template <typename R>
hipError_t launch_step_implicit(Fields<R> o, Fields<R> w, Mat<R> M, Geo g, double dx, double dy, R alpha, Src src,
                                ImpWork<R> wk, hipStream_t s, hipEvent_t* ev);
// Chebyshev iterations per plane solve and the spectral bound used
int implicit_iters(const Geo& g, double dx, double dy, double alpha, int fp32, double* lmax);

// ---- open pipes (tete_pipe.hip) ------------------------------------------
// Node plane of the entrance cross-section: (nx+1)(ny+1) nodes, node (i, j)
// at j + (ny+1) i; wx = dy/dx, wy = dx/dy weigh the x and y neighbours of the
// cross-section's Laplacian.
struct CgPlane {
    int nx, ny;
    int64_t n;
    double wx, wy;
};
// Conjugate-gradient work arrays (n doubles each), the free-node weights w,
// RED_BLOCKS partial sums and the iteration's scalars sc (8 doubles).
struct CgWork {
    double *x, *r, *p, *q, *w, *partial, *sc;
};
// free-node weights from the e_z codes of plane 0, and *bad = 1 unless cell
// planes 0 .. kst-1 are uniform (*bad must hold 0 before)
hipError_t launch_pipe_check(double* w, const uint8_t* code, Geo g, CgPlane P, int kst, int* bad, hipStream_t s);
// x = 0, r = p = delta at node src; tol bounds |r|^2 for convergence
hipError_t launch_cg_init(CgWork W, CgPlane P, int64_t src, double tol, hipStream_t s);
// iters iterations (a converged iteration leaves x unchanged); sc[0] = |r|^2,
// sc[3] = 1 once converged, sc[5] = the iterations taken
hipError_t launch_cg_iterations(CgWork W, CgPlane P, int iters, hipStream_t s);
// profile table F[p + 2M + 1], p = -2M-1 .. 1, of the bunch current lam
hipError_t launch_pipe_profile(double* F, const double* lam, int M, double dtau, hipStream_t s);
// the state y^{n0} of the bunch's field in the pipe into f
template <typename R>
hipError_t launch_pipe_field(Fields<R> f, const uint8_t* code, const double* phi, const double* F, int M, int64_t n0,
                             double rxy, double ryx, Geo g, hipStream_t s);

}  // namespace tete
