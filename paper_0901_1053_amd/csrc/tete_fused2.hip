// Two steps of scheme (23) in one kernel: temporal blocking of the fused step
// (FP32 fields, vacuum cells with staircase PEC codes).
//
// The x-march of a workgroup runs two copies of the single-step pipeline of
// tete_fused.hip.  Stage A takes the old fields (step n) loaded from HBM to
// step n+1; stage B takes stage A's results to step n+2, four planes behind
// stage A.  Stage A's results never leave the chip: per two steps the state is
// read once and written once.  Each stage keeps the single-step lag table (its
// ten sub-updates at plane lags 0-4 behind its input plane) and its own six
// j-exchange planes in LDS; both stages share the one barrier per plane.
//
// Halos.  One step invalidates one lane at each end of a wave and two rows
// at each edge of the workgroup; two steps invalidate two lanes and three
// rows (the sub-updates that reach two rows out in one step reach only one
// row out in the other, so the halo does not double along j).  A workgroup
// of 16 rows by 64 lanes thus owns 10 rows by 60 entries, and a chunk of
// planes xs .. xe-1 needs old data on planes xs-4 .. xe+3.
//
// Stage B's input plane at iteration p is plane p-4: e_x from stage A's S9 of
// this iteration, e_y (S10) and h_z (S8) from the previous one, h_x and h_y
// (S4, S5) from two iterations back and e_z (S3) from three; delay lines in
// LDS (one slot per thread) hold the older ones.
//
// Register budget.  Two stages of carried state fill the 128 VGPRs a
// 1024-thread workgroup allows, so the coefficients are pre-multiplied by
// their factor a or 2a, PEC selects are two bit operations, the delay lines
// live in LDS and one plane is prefetched (a second one spills 23 registers).
// The FP64 shape (512 threads, 256 VGPRs per wave) prefetches two.
//
// Wake.  The update of sample s at step n+1 from edge k and the update of the
// same sample at step n from edge k-1 coincide.  The lane of node k applies
// both in one read-modify-write, step n's term first, so every sample is
// written by one lane per launch and each sum is formed in the same order as
// by two single-step launches.  Step n's term needs e_z^{n-1/2} and
// e_z^{n+1/2} of edge k-1 on the source plane: the first is kept from stage
// A's pass over that plane, the second is stage B's old e_z there; both come
// over from the neighbouring lane when stage B reaches the plane.

#include <algorithm>
#include <type_traits>
#include <vector>

#include "tete_dev.h"

namespace tete {
namespace {


// Carried pipeline state of one stage, named by plane lag behind the stage's
// input plane q (m1 = q-1, ...), as in the single-step kernel.  The z
// differences of the old e_x and e_y are formed again when needed (a lane
// shift and a subtraction) rather than carried, which saves registers.
template <typename R>
struct Stage {
    R EXm1, EXm2;
    R EYm1, EYm2;
    R EZm1, HYm1;
    R HZm1, HZm2, HZm3;
    R hxn_m1, hxn_m2, hyn_m2, ezh_m2;
    R pztHX_m3, pztHY_m3, pztHY_m4;
    R exh_m3, exh_m4, eyh_m3, hzn_m4;
};

// Input plane of a stage (fields of the step it starts from).
template <typename R>
struct In {
    R ex, ey, ez, hx, hy, hz;
};
// j-neighbours read from LDS: e_z (j+1) at q, h_x^n (j-1) at q-1, e_z^{n+1/2}
// (j+1) at q-2, h_z^n (j-1) at q-2, e_x^{n+1/2} (j+1) at q-3, h_z^{n+1} (j-1)
// at q-4.
template <typename R>
struct Nb {
    R ez0_jp, hxn1_jm, ezh2_jp, hz2_jm, exh3_jp, hzn4_jm;
};
// Coefficients of the sub-updates of one iteration, each already multiplied
// by its factor a or 2a (the product the single-step kernel forms first, so
// the arithmetic is the same): mu masked by the index ranges of the h
// components, kappa zero on PEC edges.
template <typename R>
struct Co {
    R mx0, mx2, my1, my2, mz3, kz1, ky2, kx2, ky3, kx4;
};
// Results of one iteration: e_z^{n-1/2} and e_z^{n+1/2} at q-1, h_x^{n+1/2}
// and h_y^{n+1/2} at q-2, h_z^{n+1} and e_y^{n+1} at q-3, e_x^{n+1} at q-4.
template <typename R>
struct Out {
    R ezold1, ezh1, hxh2, hyh2, hzn3, ey13, ex14;
};

// One iteration of a stage: the ten sub-updates at their lags, then the
// rotation of the carried state by one plane.  inj is the bunch current term
// taken off e_z^{n+1/2} (zero off the source line; x - 0 is exact).
template <typename R>
__device__ __forceinline__ Out<R> stage_plane(Stage<R>& S, const In<R>& c, const Nb<R>& nb, const Co<R>& f,
                                              const R inj)
{
    // S1 at q: h_x^n = h_x^{n-1/2} + a mu_x [P_z e_y^n - P_y e_z^{n-1/2}]
    const R pzEY0 = lane_next(c.ey) - c.ey;
    const R hxn0 = c.hx + f.mx0 * (pzEY0 - (nb.ez0_jp - c.ez));
    // S2 at q-1: h_y^n = h_y^{n-1/2} + a mu_y [-P_z e_x^n + P_x e_z^{n-1/2}]
    const R pzEXm1 = lane_next(S.EXm1) - S.EXm1;
    const R hyn_m1 = S.HYm1 + f.my1 * (-pzEXm1 + (c.ez - S.EZm1));
    // S3 at q-1: e_z^{n+1/2} = e_z^{n-1/2} + 2a kappa_z [P_y^T h_x^n - P_x^T h_y^n - j_z^n]
    R ezh_m1 = S.EZm1 + f.kz1 * ((nb.hxn1_jm - S.hxn_m1) - (S.hyn_m2 - hyn_m1));
    {
#pragma clang fp contract(off)
        ezh_m1 -= inj;
    }
    // S4 at q-2: h_x^{n+1/2} = h_x^n + a mu_x [P_z e_y^n - P_y e_z^{n+1/2}]
    const R pzEYm2 = lane_next(S.EYm2) - S.EYm2;
    const R hxh_m2 = S.hxn_m2 + f.mx2 * (pzEYm2 - (nb.ezh2_jp - S.ezh_m2));
    // S5 at q-2: h_y^{n+1/2} = h_y^n + a mu_y [-P_z e_x^n + P_x e_z^{n+1/2}]
    const R pzEXm2 = lane_next(S.EXm2) - S.EXm2;
    const R hyh_m2 = S.hyn_m2 + f.my2 * (-pzEXm2 + (ezh_m1 - S.ezh_m2));
    // S7 at q-2: e_y^{n+1/2} = e_y^n + a kappa_y [-P_z^T h_x^{n+1/2} + P_x^T h_z^n]
    const R pztHX_m2 = lane_prev(hxh_m2) - hxh_m2;
    const R eyh_m2 = S.EYm2 + f.ky2 * (-pztHX_m2 + (S.HZm3 - S.HZm2));
    // S6 at q-2: e_x^{n+1/2} = e_x^n + a kappa_x [P_z^T h_y^{n+1/2} - P_y^T h_z^n]
    const R pztHY_m2 = lane_prev(hyh_m2) - hyh_m2;
    const R exh_m2 = S.EXm2 + f.kx2 * (pztHY_m2 - (nb.hz2_jm - S.HZm2));
    // S8 at q-3: h_z^{n+1} = h_z^n + 2a mu_z [P_y e_x^{n+1/2} - P_x e_y^{n+1/2}]
    const R hzn_m3 = S.HZm3 + f.mz3 * ((nb.exh3_jp - S.exh_m3) - (eyh_m2 - S.eyh_m3));
    // S9 at q-4: e_x^{n+1} = e_x^{n+1/2} + a kappa_x [P_z^T h_y^{n+1/2} - P_y^T h_z^{n+1}]
    const R ex1_m4 = S.exh_m4 + f.kx4 * (S.pztHY_m4 - (nb.hzn4_jm - S.hzn_m4));
    // S10 at q-3: e_y^{n+1} = e_y^{n+1/2} + a kappa_y [-P_z^T h_x^{n+1/2} + P_x^T h_z^{n+1}]
    const R ey1_m3 = S.eyh_m3 + f.ky3 * (-S.pztHX_m3 + (S.hzn_m4 - hzn_m3));

    const Out<R> o = {S.EZm1, ezh_m1, hxh_m2, hyh_m2, hzn_m3, ey1_m3, ex1_m4};

    S.EXm2 = S.EXm1; S.EXm1 = c.ex;
    S.EYm2 = S.EYm1; S.EYm1 = c.ey;
    S.EZm1 = c.ez; S.HYm1 = c.hy;
    S.HZm3 = S.HZm2; S.HZm2 = S.HZm1; S.HZm1 = c.hz;
    S.hxn_m2 = S.hxn_m1; S.hxn_m1 = hxn0;
    S.hyn_m2 = hyn_m1;
    S.ezh_m2 = ezh_m1;
    S.pztHX_m3 = pztHX_m2;
    S.pztHY_m4 = S.pztHY_m3; S.pztHY_m3 = pztHY_m2;
    S.exh_m4 = S.exh_m3; S.exh_m3 = exh_m2;
    S.eyh_m3 = eyh_m2;
    S.hzn_m4 = hzn_m3;
    return o;
}

// LDS of one workgroup: per stage, six j-exchange planes of TYH + 2 rows
// ([quantity][buffer][row][lane]), double-buffered by plane parity (NB = 2)
// or single (NB = 1, a second barrier per plane); and stage B's delay lines
// for e_z, h_x and h_y, two planes deep, one slot per thread
// ([quantity][plane parity][thread]), kept here to free registers.
// With materials by class (TAB) the class table is staged here too.
template <typename R, int TYH, int NB, int LW, bool TAB = false>
struct Lds2 {
    R a[6][NB][TYH + 2][LW];
    R b[6][NB][TYH + 2][LW];
    R d[3][2][LW * TYH];
    R tab[TAB ? TETE_MAX_CLASSES * CLS_STRIDE : 1];
};

// Launch shape of the two-step kernel per field type: rows of LW lanes
// (entries along k; a wave holds 64 / LW rows), 16 rows owning 10, LW - 4
// entries owned per row.  FP32: LW = 64, 1024 threads (16 waves, 128 VGPRs
// each).  FP64: LW = 32, 512 threads (8 waves, 256 VGPRs each), since two
// stages of doubles do not fit 128 registers; a row segment is then 256 bytes
// as in FP32.  Both double-buffer the exchange planes (135 KB of LDS).
template <typename R, int TYH, int LW>
struct Shape2 {
    static constexpr int rows = TYH, nb = 2, lw = LW, threads = TYH * LW;
};
// default rows, lanes per row and planes prefetched of the two-step kernel,
// and the other FP32 shapes: 24 rows of 32 lanes (768 threads, owning
// 18 x 28; 168 VGPRs per wave hold two prefetched planes) and 32 rows of 32
// lanes (owning 26 x 28), selected by rows = 24 or 32
template <typename R> struct Default2;
template <> struct Default2<float> { static constexpr int rows = 16, lw = 64, pd = 1; };
template <> struct Default2<double> { static constexpr int rows = 16, lw = 32, pd = 2; };
inline int lanes2(int real_bytes, int rows) { return real_bytes == 8 || rows == 24 || rows == 32 ? 32 : 64; }

// Two steps of one tile (ty, tz) and x-chunk cx.  Every thread of the
// workgroup must call it (it contains barriers).
// WIT: also keep stage A's e_z^{n+1/2} on the witness lines of wm (a
// separate instance; the kernel without witness lines is unchanged).
// PD: planes of old data loaded ahead (their loads in flight while a plane
// is processed): two fit the 256 VGPRs of the FP64 shape and the 168 of the
// FP32 24-row shape; the 128 of the 1024-thread FP32 shapes hold one.
// CLS: materials by class.  Each plane's class bytes are loaded with its
// fields and kept, a byte per plane, for the nine planes the two stages'
// sub-updates reach back; each coefficient is then read from the class table
// in LDS (already multiplied by a or 2a, the product the materials step forms
// from its arrays, so the results are those of single materials steps), the
// kappa of PEC edges zeroed by the codes as in vacuum.
// ARR: per-entry materials, the six arrays kappa_x,y,z, mu_x,y,z of MA (zero
// on PEC edges and outside each component's range, as the materials step
// takes them).  Each plane's six values are loaded with its fields and
// carried in registers for the planes the two stages reach back (kappa_x
// eight planes, kappa_y and mu_z seven, mu_x and mu_y six, kappa_z five);
// each coefficient is multiplied by a or 2a where it is used, the product the
// materials step forms, so the results are those of single materials steps.
// The PEC codes are not read.
template <typename R>
struct Arr6 {
    const R* m[6];
};
// EN: the energy W^{n,e} of Sec. 4.4 of the launch's input state y^n (from
// stage A's input, eo.want bit 0) and of y^{n+1} (from stage B's input, bit
// 1), summed in FP64 over the entries the tile owns and written as the
// workgroup's two partial sums eo.part[2 b], eo.part[2 b + 1].  Each term of
// an entry is taken where the stage holds its operands: e_z and h_x (with
// e_z at j+1 and e_y at k+1) at the input plane, h_y (e_z at i+1, e_x at k+1)
// one plane behind, e_x, e_y and h_z (h_z at j-1 and at i-1) two behind; the
// terms are those of the energy kernel, in another summation order.  With
// materials by class (CLS) each term's coefficients come from et, a table in
// LDS of ET_N FP64 values per class built from the class materials craw
// (kappa_x, kappa_y, kappa_z, mu_x, mu_y, mu_z per class, rounded to the
// field type as the per-entry arrays hold them): 1/(2 kappa) and 1/(2 mu), 0
// where kappa or mu is 0, and a^2 kappa / 2, a^2 mu / 2.
struct EnOut {
    double* part;
    int want;
    double a;
    const double* craw;
    const double* et;
};
enum { ET_SKX, ET_SKY, ET_SKZ, ET_SMX, ET_SMY, ET_SMZ, ET_DKX, ET_DKY, ET_DMX, ET_DMY, ET_N };
template <typename R, int TYH, int NB, int LW, int PD, bool WIT = false, bool CLS = false, bool ARR = false,
          class LDS, bool EN = false>
__device__ __forceinline__ void fused2_tile(const FArgs<R>& A, const int ty, const int tz, const int cx, LDS& L,
                                            const WitMid<R>& wm = WitMid<R>{}, const Arr6<R>& MA = Arr6<R>{},
                                            const EnOut& eo = EnOut{})
{
    static_assert(!(ARR && (CLS || WIT)), "one material source per instance");
    static_assert(!(EN && ARR), "energy with vacuum coefficients or materials by class only");
    constexpr int TY = TYH - 6;   // rows owned
    constexpr int KT2 = LW - 4;   // entries owned per row
    // Lane shifts act on the whole wave; with two rows per wave (LW = 32) the
    // shift across the row boundary only feeds halo lanes.
    const Geo g = A.g;

    const int kl = threadIdx.x % LW;
    const int jl = threadIdx.x / LW;
    const int j = ty * TY - 3 + jl;
    const int k = tz * KT2 - 2 + kl;
    const bool jin = (unsigned)j <= (unsigned)g.ny;
    const bool kin = (unsigned)k <= (unsigned)g.nz;
    const bool node = jin && kin;
    const bool owned = node && jl >= 3 && jl < 3 + TY && kl >= 2 && kl < 2 + KT2;
    const int roff = k + j * g.sz;

    // index-range masks of the h components in j and k (the x part needs
    // none, see coef below)
    const bool hx_jk = node && j < g.ny && k < g.nz;
    const bool hy_k = node && k < g.nz;
    const bool hz_j = node && j < g.ny;

    const int xs = cx * A.xchunk;
    const int xe = min(xs + A.xchunk, g.nx + 1);
    const int xload_end = min(xe + 3, g.nx);    // last plane whose old data is needed

    const R a2 = A.a + A.a;
    // with 64 lanes a wave is one row: the row test is then scalar, and so are
    // the source-plane tests built on it
    const int jrow = LW == 64 ? __builtin_amdgcn_readfirstlane(j) : j;
    const bool src_row = A.src.on && jrow == A.src.j0;
    // the source row lies in this wave (uniform over the wave: lane shifts
    // below run with every lane active)
    const int wj0 = ty * TY - 3 + (int)(threadIdx.x / 64) * (64 / LW);
    const bool src_wave = A.src.on && A.src.j0 >= wj0 && A.src.j0 < wj0 + 64 / LW;
    const bool src_k = kin && k < g.nz;                 // lane holds an e_z edge

    // Buffer resources over the chunk's planes, as in the single-step kernel:
    // loads cover planes pb = max(0, xs - 4) .. xload_end and out-of-range
    // loads return 0.  The
    // host keeps (xchunk + 8) planes below 2^31 bytes.
    constexpr uint32_t RB = sizeof(R);
    constexpr uint32_t OOB = 0x80000000u;
    const uint32_t plane_bytes = (uint32_t)g.sp * RB;
    const int pb = max(0, xs - 4);
    const int nload = xload_end >= pb ? xload_end - pb + 1 : 0;
    auto mk = [](const void* base, uint32_t bytes) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
    };
    const int64_t ld0 = (int64_t)pb * g.sp;
    const auto rEX = mk(A.ex + ld0, nload * plane_bytes), rEY = mk(A.ey + ld0, nload * plane_bytes),
               rEZ = mk(A.ez + ld0, nload * plane_bytes), rHX = mk(A.hx + ld0, nload * plane_bytes),
               rHY = mk(A.hy + ld0, nload * plane_bytes), rHZ = mk(A.hz + ld0, nload * plane_bytes);
    const auto rC = mk(A.code, (uint32_t)std::min<int64_t>((int64_t)g.np + 4, 0x7fffffff));
    __amdgpu_buffer_rsrc_t rK = rC;
    __amdgpu_buffer_rsrc_t rM[ARR ? 6 : 1];
    if constexpr (ARR) {
#pragma unroll
        for (int c = 0; c < 6; ++c) rM[c] = mk(MA.m[c] + ld0, nload * plane_bytes);
    }
    if constexpr (CLS) {
        rK = mk(A.cls, (uint32_t)std::min<int64_t>((int64_t)g.np + 4, 0x7fffffff));
        // the class table into LDS; the barrier of the first j-exchange
        // orders these writes before any read
        for (int t = threadIdx.x; t < TETE_MAX_CLASSES * CLS_STRIDE; t += TYH * LW) L.tab[t] = A.ctab[t];
    }
    // Stores are plain global stores: the chunk's first plane as a scalar base
    // plus a 32-bit byte offset, predicated on the plane lying in the chunk
    // (uniform) and the entry being owned; this keeps six buffer resources
    // (24 scalar registers) free.
    const int64_t st0 = (int64_t)xs * g.sp;
    char* const gEX = (char*)(A.ex1 + st0);
    char* const gEY = (char*)(A.ey1 + st0);
    char* const gEZ = (char*)(A.ez1 + st0);
    char* const gHX = (char*)(A.hx1 + st0);
    char* const gHY = (char*)(A.hy1 + st0);
    char* const gHZ = (char*)(A.hz1 + st0);
    const uint32_t in_ld = (uint32_t)roff * RB;
    auto gstore = [](char* base, uint32_t off, R v) { *(R*)(base + off) = v; };
    auto xown = [&](int q) { return q >= xs && q < xe; };
    const uint32_t cfix = node ? 0u : 7u;              // outside the grid: PEC

    struct PR {
        R ex, ey, ez, hx, hy, hz;
        uint32_t c;
        uint32_t k[CLS ? 1 : 0];
        R m[ARR ? 6 : 0];
    };
    auto load_plane = [&](int i, PR& d) {
        const uint32_t po = (uint32_t)(i - pb);
        const uint32_t off = node ? in_ld + po * plane_bytes : OOB;
        d.ex = bload<R>(rEX, off);
        d.ey = bload<R>(rEY, off);
        d.ez = bload<R>(rEZ, off);
        d.hx = bload<R>(rHX, off);
        d.hy = bload<R>(rHY, off);
        d.hz = bload<R>(rHZ, off);
        if constexpr (ARR) {
#pragma unroll
            for (int c = 0; c < 6; ++c) d.m[c] = bload<R>(rM[c], off);
            d.c = 0u;
        } else {
            const uint32_t offc = node ? ((uint32_t)(roff + i * g.sp) & ~3u) : OOB;
            d.c = __builtin_amdgcn_raw_buffer_load_b32(rC, offc, 0, 0);   // byte extracted when used
        }
        if constexpr (CLS) {
            const uint32_t offc = node ? ((uint32_t)(roff + i * g.sp) & ~3u) : OOB;
            d.k[0] = __builtin_amdgcn_raw_buffer_load_b32(rK, offc, 0, 0);
        }
    };

    Stage<R> SA = {}, SB = {};
    // class bytes of planes p .. p-3 (kh0, byte i = plane p-i), p-4 .. p-7 (kh1)
    // and p-8 (kh2) (CLS only)
    uint32_t kh0 = 0, kh1 = 0, kh2 = 0;
    // coefficient histories of ARR, index = planes behind p (index 0 is the
    // current plane's, set from its loads)
    R hKX[ARR ? 9 : 1] = {}, hKY[ARR ? 8 : 1] = {}, hKZ[ARR ? 6 : 1] = {}, hMX[ARR ? 7 : 1] = {},
      hMY[ARR ? 7 : 1] = {}, hMZ[ARR ? 8 : 1] = {};
    const int tid = threadIdx.x;
    for (int q = 0; q < 3; ++q) L.d[q][0][tid] = L.d[q][1][tid] = R(0);   // stage B's delay lines
    R d_ey4 = 0;                 // e_y^{n+1} of plane p-4
    uint32_t ch = 0x77777777u;   // PEC codes of planes p-1 .. p-8, four bits each
    R ezA = 0;                   // e_z^{n-1/2} of edge k on the source plane

    // coefficient factors: a mu and 2a mu zero outside the index range of the
    // h component in j and k, a kappa and 2a kappa
    const R amx = hx_jk ? A.a * A.mx : R(0), amy = hy_k ? A.a * A.my : R(0), a2mz = hz_j ? a2 * A.mz : R(0);
    const R akx = A.a * A.kx, aky = A.a * A.ky, a2kz = a2 * A.kz;
    // v, or 0 where bit b of the code history is set (a PEC edge)
    auto sel = [](uint32_t hist, int b, R v) {
        const uint32_t m = (uint32_t)(((int32_t)(hist << (31 - b))) >> 31);
        if constexpr (sizeof(R) == 4) {
            return __builtin_bit_cast(R, __builtin_bit_cast(uint32_t, v) & ~m);
        } else {
            const uint64_t m2 = ((uint64_t)m << 32) | m;
            return __builtin_bit_cast(R, __builtin_bit_cast(uint64_t, v) & ~m2);
        }
    };
    // coefficients of a stage whose input plane is q; hist holds the codes of
    // planes q-1 .. q-4 in bits 0-15.  The h components need no mask along x:
    // on the planes outside their range (i = nx for h_y and h_z, and planes
    // before the grid or past it, which have no old data) every e their
    // update reads lies on a wall or outside the grid, where e is 0, so the
    // update adds exactly 0 and they keep the 0 they hold; the e they feed
    // are wall or outside edges too (kappa 0).
    auto coef = [&](int q, uint32_t hist) {
        (void)q;
        Co<R> f;
        f.mx0 = amx;
        f.mx2 = amx;
        f.my1 = amy;
        f.my2 = amy;
        f.mz3 = a2mz;
        f.kz1 = sel(hist, 2, a2kz);
        f.ky2 = sel(hist, 5, aky);
        f.kx2 = sel(hist, 4, akx);
        f.ky3 = sel(hist, 9, aky);
        f.kx4 = sel(hist, 12, akx);
        return f;
    };
    // coefficients from the class table, for a stage whose input plane holds
    // class l0 and planes q-1 .. q-4 classes l1 .. l4 (CLS)
    auto tab = [&](uint32_t cls, int e) { return L.tab[cls * CLS_STRIDE + e]; };
    auto coefc = [&](uint32_t l0, uint32_t l1, uint32_t l2, uint32_t l3, uint32_t l4, uint32_t hist) {
        Co<R> f;
        f.mx0 = hx_jk ? tab(l0, CLS_AMX) : R(0);
        f.mx2 = hx_jk ? tab(l2, CLS_AMX) : R(0);
        f.my1 = hy_k ? tab(l1, CLS_AMY) : R(0);
        f.my2 = hy_k ? tab(l2, CLS_AMY) : R(0);
        f.mz3 = hz_j ? tab(l3, CLS_A2MZ) : R(0);
        f.kz1 = sel(hist, 2, tab(l1, CLS_A2KZ));
        f.ky2 = sel(hist, 5, tab(l2, CLS_AKY));
        f.kx2 = sel(hist, 4, tab(l2, CLS_AKX));
        f.ky3 = sel(hist, 9, tab(l3, CLS_AKY));
        f.kx4 = sel(hist, 12, tab(l4, CLS_AKX));
        return f;
    };
    auto cbyte = [](uint32_t h, int b) { return (h >> (8 * b)) & 0xffu; };
    // coefficients from the histories for a stage whose input plane is lb
    // planes behind p (ARR)
    auto coefa = [&](const int lb) {
        Co<R> f;
        f.mx0 = A.a * hMX[lb];
        f.mx2 = A.a * hMX[lb + 2];
        f.my1 = A.a * hMY[lb + 1];
        f.my2 = A.a * hMY[lb + 2];
        f.mz3 = a2 * hMZ[lb + 3];
        f.kz1 = a2 * hKZ[lb + 1];
        f.ky2 = A.a * hKY[lb + 2];
        f.kx2 = A.a * hKX[lb + 2];
        f.ky3 = A.a * hKY[lb + 3];
        f.kx4 = A.a * hKX[lb + 4];
        return f;
    };
    // bunch current of step n on edge k (zero where no cell crosses it),
    // rounded on its own before it is subtracted
    auto inject = [&](int64_t n, R kz) {
#pragma clang fp contract(off)
        const int64_t m = (int64_t)k - n + A.src.M;
        return (m >= -A.src.M && m <= A.src.M) ? (R)((double)kz * A.src.lam[m + A.src.M]) : R(0);
    };

    PR buf[PD + 1];
#pragma unroll
    for (int d = 0; d < PD; ++d) load_plane(xs - 4 + d, buf[d]);

    // energy partial sums of y^n and y^{n+1} (EN)
    double accA = 0.0, accB = 0.0;
    // the vacuum coefficients folded into the terms' factors: 1/(2 kappa) and
    // 1/(2 mu) for the squares, a^2 kappa / 2 and a^2 mu / 2 for the
    // differences (a product per term instead of a division; the terms then
    // differ from the energy kernel's by rounding)
    const double ea = eo.a, ha2 = 0.5 * ea * ea;
    const double skx0 = 0.5 / (double)A.kx, sky0 = 0.5 / (double)A.ky, skz0 = 0.5 / (double)A.kz;
    const double smx0 = 0.5 / (double)A.mx, smy0 = 0.5 / (double)A.my, smz0 = 0.5 / (double)A.mz;
    const double dkx0 = ha2 * (double)A.kx, dky0 = ha2 * (double)A.ky, dmx0 = ha2 * (double)A.mx,
                 dmy0 = ha2 * (double)A.my;
    // one stage's energy terms: input c at plane q with PEC code cq, carried
    // state S (before the stage rotates it), j-neighbours nb, codes of planes
    // q-1 .. q-4 in hist; with CLS the classes of planes q, q-1, q-2 in the
    // low bytes of kc
    auto en_terms = [&](const In<R>& c, const Stage<R>& S, const Nb<R>& nb, const uint32_t cq, const uint32_t hist,
                        const int q, const uint32_t kc) {
        const R eyk = lane_next(c.ey), exk = lane_next(S.EXm1);   // e_y(k+1) at q, e_x(k+1) at q-1
        double e = 0.0;
        if (!owned) return e;
        double skx = skx0, sky = sky0, skz = skz0, smx = smx0, smy = smy0, smz = smz0;
        double dkx = dkx0, dky = dky0, dmx = dmx0, dmy = dmy0;
        if constexpr (CLS) {
            const double* t0 = eo.et + ET_N * cbyte(kc, 0);
            const double* t1 = eo.et + ET_N * cbyte(kc, 1);
            const double* t2 = eo.et + ET_N * cbyte(kc, 2);
            skz = t0[ET_SKZ]; smx = t0[ET_SMX]; dmx = t0[ET_DMX];
            smy = t1[ET_SMY]; dmy = t1[ET_DMY];
            skx = t2[ET_SKX]; sky = t2[ET_SKY]; smz = t2[ET_SMZ]; dkx = t2[ET_DKX]; dky = t2[ET_DKY];
        } else {
            (void)kc;
        }
        if (xown(q)) {
            if (!(cq & 4u)) {                                   // e_z
                const double v = (double)c.ez;
                e += v * v * skz;
            }
            if (hx_jk) {                                        // h_x
                const double h = (double)c.hx, d = (double)nb.ez0_jp - (double)c.ez;
                e += h * h * smx - dmx * (d * d) + ea * (h * ((double)eyk - (double)c.ey));
            }
        }
        if (xown(q - 1) && hy_k && q - 1 < g.nx) {                 // h_y
            const double h = (double)S.HYm1, d = (double)c.ez - (double)S.EZm1;
            e += h * h * smy - dmy * (d * d) - ea * (h * ((double)exk - (double)S.EXm1));
        }
        if (xown(q - 2)) {
            if (!((hist >> 4) & 1u)) {                            // e_x
                const double v = (double)S.EXm2, d = (double)nb.hz2_jm - (double)S.HZm2;
                e += v * v * skx - dkx * (d * d);
            }
            if (!((hist >> 5) & 1u)) {                            // e_y
                const double v = (double)S.EYm2, d = (double)S.HZm3 - (double)S.HZm2;
                e += v * v * sky - dky * (d * d);
            }
            if (hz_j && q - 2 < g.nx) {                           // h_z
                const double h = (double)S.HZm2;
                e += h * h * smz;
            }
        }
        return e;
    };

    const int pend = xe + 7;
    auto body = [&](const int p, const PR& cur, PR& nxt) {
        load_plane(p + PD, nxt);
        // outside the grid, or a plane without old data: PEC on all edges
        const uint32_t bsh = ((uint32_t)(roff + p * g.sp) & 3u) * 8u;
        const uint32_t c0 = ((cur.c >> bsh) & 7u) | cfix | ((p >= pb && p <= xload_end) ? 0u : 7u);
        if constexpr (CLS) {
            kh2 = kh1 >> 24;
            kh1 = (kh1 << 8) | (kh0 >> 24);
            kh0 = (kh0 << 8) | ((cur.k[0] >> bsh) & 0xffu);
        }
        if constexpr (ARR) {
            hKX[0] = cur.m[0]; hKY[0] = cur.m[1]; hKZ[0] = cur.m[2];
            hMX[0] = cur.m[3]; hMY[0] = cur.m[4]; hMZ[0] = cur.m[5];
        }

        // stage B's input plane p-4, except e_x (stage A's S9 of this
        // iteration); the delay-line slot of this parity holds plane p-4 and
        // is refilled with plane p-2
        const int s = p & 1;
        const R bEY = d_ey4, bEZ = L.d[0][s][tid], bHX = L.d[1][s][tid], bHY = L.d[2][s][tid], bHZ = SA.hzn_m4;
        L.d[0][s][tid] = SA.ezh_m2;

        // j-exchange through LDS (row r of the tile is LDS row r+1; rows 0 and
        // TYH+1 are never written and reach only halo results)
        const int x = NB == 2 ? s : 0;   // exchange buffer
        L.a[0][x][jl + 1][kl] = cur.ez;
        L.a[1][x][jl + 1][kl] = SA.hxn_m1;
        L.a[2][x][jl + 1][kl] = SA.ezh_m2;
        L.a[3][x][jl + 1][kl] = SA.HZm2;
        L.a[4][x][jl + 1][kl] = SA.exh_m3;
        L.a[5][x][jl + 1][kl] = SA.hzn_m4;
        L.b[0][x][jl + 1][kl] = bEZ;
        L.b[1][x][jl + 1][kl] = SB.hxn_m1;
        L.b[2][x][jl + 1][kl] = SB.ezh_m2;
        L.b[3][x][jl + 1][kl] = SB.HZm2;
        L.b[4][x][jl + 1][kl] = SB.exh_m3;
        L.b[5][x][jl + 1][kl] = SB.hzn_m4;
        __syncthreads();
        const Nb<R> nA = {L.a[0][x][jl + 2][kl], L.a[1][x][jl][kl], L.a[2][x][jl + 2][kl],
                          L.a[3][x][jl][kl],     L.a[4][x][jl + 2][kl], L.a[5][x][jl][kl]};
        const Nb<R> nB = {L.b[0][x][jl + 2][kl], L.b[1][x][jl][kl], L.b[2][x][jl + 2][kl],
                          L.b[3][x][jl][kl],     L.b[4][x][jl + 2][kl], L.b[5][x][jl][kl]};
        if (NB == 1) __syncthreads();    // all reads done before the next plane's writes

        Co<R> fA, fB;
        if constexpr (CLS) {
            fA = coefc(cbyte(kh0, 0), cbyte(kh0, 1), cbyte(kh0, 2), cbyte(kh0, 3), cbyte(kh1, 0), ch);
            fB = coefc(cbyte(kh1, 0), cbyte(kh1, 1), cbyte(kh1, 2), cbyte(kh1, 3), cbyte(kh2, 0), ch >> 16);
        } else if constexpr (ARR) {
            fA = coefa(0);
            fB = coefa(4);
        } else {
            fA = coef(p, ch);
            fB = coef(p - 4, ch >> 16);
        }
        // S3 of stage A is at plane p-1 (step n), of stage B at plane p-5 (step n+1)
        const bool srcA = src_row && p - 1 == A.src.i0;
        const bool srcB = src_row && p - 5 == A.src.i0;
        const bool srcBw = LW == 64 ? srcB : src_wave && p - 5 == A.src.i0;   // wave-uniform
        R kzA = A.kz, kzB = A.kz;
        if constexpr (CLS) {
            kzA = tab(cbyte(kh0, 1), CLS_KZ);
            kzB = tab(cbyte(kh1, 1), CLS_KZ);
        }
        R injA, injB;
        if constexpr (ARR) {      // the arrays hold kappa_z = 0 on PEC edges
            injA = (srcA && src_k) ? inject(A.src.n, hKZ[1]) : R(0);
            injB = (srcB && src_k) ? inject(A.src.n + 1, hKZ[5]) : R(0);
        } else {
            injA = (srcA && src_k) ? inject(A.src.n, sel(ch, 2, kzA)) : R(0);
            injB = (srcB && src_k) ? inject(A.src.n + 1, sel(ch, 18, kzB)) : R(0);
        }

        if constexpr (EN) {      // y^n: stage A's input, before the stage rotates its state
            if (eo.want & 1)
                accA += en_terms(In<R>{cur.ex, cur.ey, cur.ez, cur.hx, cur.hy, cur.hz}, SA, nA, c0, ch, p, kh0);
        }
        const Out<R> oA = stage_plane(SA, In<R>{cur.ex, cur.ey, cur.ez, cur.hx, cur.hy, cur.hz}, nA, fA, injA);
        if constexpr (EN) {      // y^{n+1}: stage B's input at plane p-4 (its e_x is stage A's S9 above)
            if (eo.want & 2)
                accB += en_terms(In<R>{oA.ex14, bEY, bEZ, bHX, bHY, bHZ}, SB, nB, (ch >> 12) & 7u, ch >> 16, p - 4,
                                 kh1);
        }
        const Out<R> oB = stage_plane(SB, In<R>{oA.ex14, bEY, bEZ, bHX, bHY, bHZ}, nB, fB, injB);

        if (srcA) ezA = oA.ezold1;
        if constexpr (WIT) {
            // e_z^{n+1/2} of edge k at plane p-1, final on owned entries.  With
            // 64 lanes a wave is one row, so the line test is scalar and adds
            // no vector registers to the loop.
            const int jr = LW == 64 ? __builtin_amdgcn_readfirstlane(j) : j;
            const int di = p - 1 - wm.iw, dj = jr - wm.jw;
            const bool on = (dj == 0 && di >= -1 && di <= 1) || ((dj == 1 || dj == -1) && di == 0);
            if (on && xown(p - 1)) {
                const int l = dj == 0 ? (di == 0 ? 0 : di < 0 ? 1 : 2) : (dj < 0 ? 3 : 4);
                if (owned && k < g.nz) wm.mid[l * g.nz + k] = oA.ezh1;
            }
        }
        // wave-uniform (one row per wave: srcB itself)
        if (srcBw) {
            const R ezA_km = lane_prev(ezA), ezB_km = lane_prev(oB.ezold1);
            if ((LW == 64 || src_row) && owned && A.src.i0 >= xs && A.src.i0 < xe) {
                const int64_t js = A.src.n + 1 - k - A.src.M;   // edge k at step n+1, edge k-1 at step n
                if (js >= A.src.jmin && js < (int64_t)A.src.jmin + A.src.nw) {
                    double w = A.src.wacc[js - A.src.jmin];
                    if (k >= 1 && k - 1 < A.src.kend) w += -0.5 * ((double)ezA_km + (double)ezB_km);
                    if (src_k && k < A.src.kend) w += -0.5 * ((double)oB.ezold1 + (double)oB.ezh1);
                    A.src.wacc[js - A.src.jmin] = w;
                }
            }
        }

        if (owned) {
            const int q1 = p - 5;
            const uint32_t o1 = in_ld + (uint32_t)(q1 - xs) * plane_bytes;
            const uint32_t o2 = o1 - plane_bytes, o3 = o2 - plane_bytes, o4 = o3 - plane_bytes;
            if (xown(q1)) gstore(gEZ, o1, oB.ezh1);
            if (xown(q1 - 1)) {
                gstore(gHX, o2, oB.hxh2);
                gstore(gHY, o2, oB.hyh2);
            }
            if (xown(q1 - 2)) {
                gstore(gHZ, o3, oB.hzn3);
                gstore(gEY, o3, oB.ey13);
            }
            if (xown(q1 - 3)) gstore(gEX, o4, oB.ex14);
        }

        L.d[1][s][tid] = oA.hxh2;
        L.d[2][s][tid] = oA.hyh2;
        d_ey4 = oA.ey13;
        ch = (ch << 4) | c0;
        if constexpr (ARR) {      // histories one plane older
#pragma unroll
            for (int d = 8; d > 0; --d) hKX[d] = hKX[d - 1];
#pragma unroll
            for (int d = 7; d > 0; --d) { hKY[d] = hKY[d - 1]; hMZ[d] = hMZ[d - 1]; }
#pragma unroll
            for (int d = 6; d > 0; --d) { hMX[d] = hMX[d - 1]; hMY[d] = hMY[d - 1]; }
#pragma unroll
            for (int d = 5; d > 0; --d) hKZ[d] = hKZ[d - 1];
        }
    };

    // trip count rounded up to a multiple of PD+1, as in the single-step kernel
    for (int p = xs - 4; p <= pend; p += PD + 1) {
#pragma unroll
        for (int u = 0; u <= PD; ++u) body(p + u, buf[u], buf[(u + PD) % (PD + 1)]);
    }
    if constexpr (EN) {
        // the workgroup's two sums: waves by shuffles, then the waves in order
        constexpr int NW = TYH * LW / 64;
        __shared__ double ered[2][NW];
        for (int off = 32; off > 0; off >>= 1) {
            accA += __shfl_down(accA, off, 64);
            accB += __shfl_down(accB, off, 64);
        }
        if ((tid & 63) == 0) {
            ered[0][tid >> 6] = accA;
            ered[1][tid >> 6] = accB;
        }
        __syncthreads();
        if (tid == 0) {
            double sa = 0.0, sb = 0.0;
            for (int w = 0; w < NW; ++w) {
                sa += ered[0][w];
                sb += ered[1][w];
            }
            eo.part[2 * blockIdx.x] = sa;
            eo.part[2 * blockIdx.x + 1] = sb;
        }
    }
}

// Tile of workgroup blockIdx.x.  act (or null): the tiles that are not
// static, (cx nyt + ty) nzt + tz in the launch's tile order
// (fused2_static_tiles), one workgroup each; the XCD remap over the list
// spreads them evenly over the XCDs, while the static tiles, which lie
// together in the metal, are not launched at all.  False for the padding
// workgroups of a full launch.
template <typename R>
__device__ __forceinline__ bool fused2_tile_of(const FArgs<R>& A, const int* act, int& ty, int& tz, int& cx)
{
    if (act) {
        const int t = act[xcd_remap(blockIdx.x, gridDim.x)];
        tz = t % A.nzt;
        ty = (t / A.nzt) % A.nyt;
        cx = t / (A.nzt * A.nyt);
        return true;
    }
    return tile_of(xcd_remap(blockIdx.x, A.nblk), A.order, A.nyt, A.nzt, ty, tz, cx);
}

template <typename R, int TYH, int LW, int PD>
__global__ __launch_bounds__(TYH * LW) void k_fused2(FArgs<R> A, const int* act)
{
    typedef Shape2<R, TYH, LW> S;
    __shared__ Lds2<R, S::rows, S::nb, S::lw> L;
    int ty, tz, cx;
    if (!fused2_tile_of(A, act, ty, tz, cx)) return;   // whole group
    fused2_tile<R, S::rows, S::nb, S::lw, PD>(A, ty, tz, cx, L);
}

// The two-step kernel that also sums the energy of its input and of the
// state between its two steps (16 rows of 32 lanes, vacuum coefficients, the
// full tiling: one pair of partial sums per workgroup, zero for the padding
// workgroups of the blocked tile orders).
template <typename R, int TYH, int LW, int PD>
__global__ __launch_bounds__(TYH * LW) void k_fused2_en(FArgs<R> A, EnOut eo)
{
    typedef Shape2<R, TYH, LW> S;
    typedef Lds2<R, S::rows, S::nb, S::lw> LT;
    __shared__ LT L;
    int ty, tz, cx;
    if (!fused2_tile_of(A, nullptr, ty, tz, cx)) {      // whole group
        if (threadIdx.x == 0) eo.part[2 * blockIdx.x] = eo.part[2 * blockIdx.x + 1] = 0.0;
        return;
    }
    fused2_tile<R, S::rows, S::nb, S::lw, PD, false, false, false, LT, true>(A, ty, tz, cx, L, WitMid<R>{},
                                                                               Arr6<R>{}, eo);
}

// The same keeping stage A's e_z^{n+1/2} on the witness lines of wm (vacuum).
template <typename R, int TYH, int LW, int PD>
__global__ __launch_bounds__(TYH * LW) void k_fused2_en_wit(FArgs<R> A, EnOut eo, WitMid<R> wm)
{
    typedef Shape2<R, TYH, LW> S;
    typedef Lds2<R, S::rows, S::nb, S::lw> LT;
    __shared__ LT L;
    int ty, tz, cx;
    if (!fused2_tile_of(A, nullptr, ty, tz, cx)) {      // whole group
        if (threadIdx.x == 0) eo.part[2 * blockIdx.x] = eo.part[2 * blockIdx.x + 1] = 0.0;
        return;
    }
    fused2_tile<R, S::rows, S::nb, S::lw, PD, true, false, false, LT, true>(A, ty, tz, cx, L, wm, Arr6<R>{}, eo);
}

// The same with materials by class: the class table and the energy
// coefficients per class (EnOut) staged in LDS.  FP64 exchanges the
// j-neighbours through single buffers (a second barrier per plane) to leave
// room for the two tables.
template <typename R, int TYH, int LW, int PD>
__global__ __launch_bounds__(TYH * LW) void k_fused2_en_cls(FArgs<R> A, EnOut eo)
{
    typedef Shape2<R, TYH, LW> S;
    constexpr int NBC = sizeof(R) == 8 ? 1 : S::nb;
    typedef Lds2<R, S::rows, NBC, S::lw, true> LT;
    __shared__ LT L;
    __shared__ double et[TETE_MAX_CLASSES * ET_N];
    int ty, tz, cx;
    if (!fused2_tile_of(A, nullptr, ty, tz, cx)) {      // whole group
        if (threadIdx.x == 0) eo.part[2 * blockIdx.x] = eo.part[2 * blockIdx.x + 1] = 0.0;
        return;
    }
    const double ha2 = 0.5 * eo.a * eo.a;
    for (int t = threadIdx.x; t < TETE_MAX_CLASSES; t += TYH * LW) {
        double v[6];
        for (int c = 0; c < 6; ++c) v[c] = (double)(R)eo.craw[6 * t + c];
        double* o = et + ET_N * t;
        o[ET_SKX] = v[0] > 0.0 ? 0.5 / v[0] : 0.0;
        o[ET_SKY] = v[1] > 0.0 ? 0.5 / v[1] : 0.0;
        o[ET_SKZ] = v[2] > 0.0 ? 0.5 / v[2] : 0.0;
        o[ET_SMX] = v[3] > 0.0 ? 0.5 / v[3] : 0.0;
        o[ET_SMY] = v[4] > 0.0 ? 0.5 / v[4] : 0.0;
        o[ET_SMZ] = v[5] > 0.0 ? 0.5 / v[5] : 0.0;
        o[ET_DKX] = ha2 * v[0];
        o[ET_DKY] = ha2 * v[1];
        o[ET_DMX] = ha2 * v[3];
        o[ET_DMY] = ha2 * v[4];
    }
    __syncthreads();
    eo.et = et;
    fused2_tile<R, S::rows, NBC, S::lw, PD, false, true, false, LT, true>(A, ty, tz, cx, L, WitMid<R>{}, Arr6<R>{},
                                                                            eo);
}

// The two-step kernel with per-entry materials (FP32: 16 rows of 32 lanes,
// 512 threads, two planes loaded ahead).
template <typename R, int TYH, int LW, int PD>
__global__ __launch_bounds__(TYH * LW) void k_fused2_arr(FArgs<R> A, Arr6<R> MA, const int* act)
{
    typedef Shape2<R, TYH, LW> S;
    __shared__ Lds2<R, S::rows, S::nb, S::lw> L;
    int ty, tz, cx;
    if (!fused2_tile_of(A, act, ty, tz, cx)) return;   // whole group
    fused2_tile<R, S::rows, S::nb, S::lw, PD, false, false, true>(A, ty, tz, cx, L, WitMid<R>{}, MA);
}

// The two-step kernel with materials by class.
template <typename R, int TYH, int LW, int PD>
__global__ __launch_bounds__(TYH * LW) void k_fused2_cls(FArgs<R> A, const int* act)
{
    typedef Shape2<R, TYH, LW> S;
    __shared__ Lds2<R, S::rows, S::nb, S::lw, true> L;
    int ty, tz, cx;
    if (!fused2_tile_of(A, act, ty, tz, cx)) return;   // whole group
    fused2_tile<R, S::rows, S::nb, S::lw, PD, false, true>(A, ty, tz, cx, L);
}

// A tile of the two-step kernel is static when every entry it loads (its rows
// and lanes with their halos, over planes max(0, xs-4) .. min(xe+3, nx)) has
// all three e edges PEC or absent (code 7), entries outside the grid counting
// as PEC: then e stays zero and h constant there, and both steps leave every
// entry the tile owns bitwise unchanged.  One workgroup per tile.
__global__ __launch_bounds__(256) void k_static2(const uint8_t* code, Geo g, int TYH, int LW, int TY, int KT2,
                                                 int xchunk, int nyt, int nzt, uint8_t* out)
{
    __shared__ int active;
    const int t = blockIdx.x;
    const int tz = t % nzt, ty = (t / nzt) % nyt, cx = t / (nzt * nyt);
    if (threadIdx.x == 0) active = 0;
    __syncthreads();
    const int xs = cx * xchunk, xe = min(xs + xchunk, g.nx + 1);
    const int pb = max(0, xs - 4), pe = min(xe + 3, g.nx);
    const int rows = TYH, lanes = LW;
    const int64_t per_plane = (int64_t)rows * lanes;
    const int64_t n = (int64_t)(pe - pb + 1) * per_plane;
    bool found = false;
    for (int64_t e = threadIdx.x; e < n && !found; e += blockDim.x) {
        const int q = pb + (int)(e / per_plane);
        const int r = (int)(e % per_plane);
        const int j = ty * TY - 3 + r / lanes, k = tz * KT2 - 2 + r % lanes;
        if (j < 0 || j > g.ny || k < 0 || k > g.nz) continue;
        if ((code[(int64_t)q * g.sp + (int64_t)j * g.sz + k] & 7u) != 7u) found = true;
    }
    if (found) atomicOr(&active, 1);
    __syncthreads();
    if (threadIdx.x == 0) out[t] = active ? 0 : 1;
}

// The two-step kernel that also keeps e_z^{n+1/2} of the witness lines
// (static tiles, when left out, store nothing there: the caller clears the
// lines, whose e_z is zero in such tiles).
template <typename R, int TYH, int LW>
__global__ __launch_bounds__(TYH * LW) void k_fused2_wit(FArgs<R> A, WitMid<R> wm, const int* act)
{
    typedef Shape2<R, TYH, LW> S;
    __shared__ Lds2<R, S::rows, S::nb, S::lw> L;
    int ty, tz, cx;
    if (!fused2_tile_of(A, act, ty, tz, cx)) return;   // whole group
    fused2_tile<R, S::rows, S::nb, S::lw, Default2<R>::pd, true>(A, ty, tz, cx, L, wm);
}

// Two steps of every active instance of a batch, by a persistent grid, as the
// single-step batch kernel does it: work item w (instance, tile, x-chunk) is
// taken by workgroup w mod gridDim.x in round w / gridDim.x, remapped over
// the XCDs within a round; the launch follows `flips` launches and `steps`
// steps of the current block.
template <typename R>
__global__ __launch_bounds__(Default2<R>::rows * Default2<R>::lw) void k_fused2_batch(const BatchTable<R>* Tg,
                                                                                     int flips, int steps)
{
    typedef Shape2<R, Default2<R>::rows, Default2<R>::lw> S;
    __shared__ Lds2<R, S::rows, S::nb, S::lw> L;
    // The table is read-only during the launch: reading it through the
    // constant address space makes its (uniform) fields scalar loads into
    // scalar registers instead of vector loads that would occupy VGPRs.
    typedef const __attribute__((address_space(4))) BatchTable<R>* CTable;
    typedef const __attribute__((address_space(4))) uint32_t* CWords;
    const CTable T = (CTable)Tg;
    const int total = T->total2;
    const int ninst = T->ninst;
    const int parity = (T->phase + flips) & 1;
    for (int round = 0; round * (int)gridDim.x < total; ++round) {
        const int base = round * (int)gridDim.x;
        const int span = min((int)gridDim.x, total - base);
        if ((int)blockIdx.x >= span) break;
        const int w = __builtin_amdgcn_readfirstlane(base + xcd_remap(blockIdx.x, span));
        int lo = 0, hi = ninst - 1;               // last instance whose first item is <= w
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (T->offset2[mid] <= w) lo = mid;
            else hi = mid - 1;
        }
        const int inst = __builtin_amdgcn_readfirstlane(lo);
        FArgs<R> A;
        {
            const CWords src = (CWords)&T->item[inst].a2[parity];
            uint32_t* dst = (uint32_t*)&A;
#pragma unroll
            for (int i = 0; i < (int)(sizeof(FArgs<R>) / 4); ++i) dst[i] = src[i];
        }
        A.src.n = T->step[inst] + steps;
        int ty, tz, cx;
        if (tile_of(w - T->offset2[inst], A.order, A.nyt, A.nzt, ty, tz, cx))
            fused2_tile<R, S::rows, S::nb, S::lw, Default2<R>::pd>(A, ty, tz, cx, L);
        __syncthreads();   // the LDS is reused by the next item
    }
}

}  // namespace

template <typename R>
hipError_t launch_batch_step2(BatchTable<R>* T, int grid, int flips, int steps, hipStream_t s)
{
    k_fused2_batch<R><<<grid, Default2<R>::rows * Default2<R>::lw, 0, s>>>(T, flips, steps);
    return hipGetLastError();
}

template <typename R>
bool fused2_setup(FArgs<R>& A, int rows, int xchunk, int order, int lanes)
{
    if (rows == 0) rows = Default2<R>::rows;
    if (rows != 16 && !((rows == 24 || rows == 32) && sizeof(R) == 4)) return false;
    if (lanes != 0 && lanes != 32 && lanes != 64) return false;
    const int TY = rows - 6, KT2 = (lanes ? lanes : lanes2(sizeof(R), rows)) - 4;
    A.nyt = (A.g.ny + 1 + TY - 1) / TY;
    A.nzt = (A.g.nz + 1 + KT2 - 1) / KT2;
    const int nplanes = A.g.nx + 1;
    // every buffer range must stay below 2^31 bytes: (xchunk + 8) planes
    const int64_t plane_bytes = (int64_t)A.g.sp * sizeof(R);
    const int64_t xmax = ((int64_t(1) << 31) - 1) / plane_bytes - 8;
    if (xmax < 1) return false;
    int xc = xchunk;
    if (xc <= 0) {
        // as few chunks as possible (each re-reads seven halo planes and
        // refills the pipeline), but enough workgroups for half of the CUs,
        // chunks of at least 16 planes, and each within the buffer limit
        const int tiles = A.nyt * A.nzt;
        int chunks = (128 + tiles - 1) / tiles;
        chunks = std::min(chunks, std::max(1, nplanes / 16));
        chunks = (int)std::max<int64_t>(chunks, (nplanes + xmax - 1) / xmax);
        xc = (nplanes + chunks - 1) / chunks;
    }
    xc = (int)std::min<int64_t>(std::max(xc, 1), xmax);
    A.xchunk = xc;
    A.nxc = (nplanes + xc - 1) / xc;
    A.order = order != 0 ? order : default_order(A.nyt, A.nzt, A.nxc);
    A.nblk = launch_tiles(A.order, A.nyt, A.nzt, A.nxc);
    return true;
}

bool fused2_fits(Geo g, int real_bytes)
{
    return (int64_t)g.sp * real_bytes * 9 < (int64_t(1) << 31);
}

int64_t fused2_tile_cap(Geo g)
{
    // the smallest owned shape: 10 rows (16-row tiles) by 28 entries (32 lanes)
    // over tiles of single planes
    return (int64_t)(g.nx + 1) * ((g.ny + 1 + 9) / 10) * ((g.nz + 1 + 27) / 28);
}

template <typename R>
hipError_t fused2_static_tiles(const uint8_t* code, Geo g, int rows, int xchunk, int order, uint8_t* tab, int* act,
                               int64_t cap, int64_t* ntiles, int* nact, hipStream_t s)
{
    Fields<R> none = {};
    Mat<R> M = {};
    M.code = code;
    FArgs<R> A = fused_args<R>(none, none, M, g, R(0), Src{});
    if (!fused2_setup<R>(A, rows, xchunk, order)) return hipErrorInvalidValue;
    const int64_t nt = (int64_t)A.nyt * A.nzt * A.nxc;
    if (nt > cap || nt > 0x7fffffff) return hipErrorInvalidValue;
    const int r = rows == 0 ? Default2<R>::rows : rows;
    const int lw = lanes2(sizeof(R), r);
    k_static2<<<(int)nt, 256, 0, s>>>(code, g, r, lw, r - 6, lw - 4, A.xchunk, A.nyt, A.nzt, tab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    std::vector<uint8_t> h((size_t)nt);
    if ((e = hipMemcpyAsync(h.data(), tab, (size_t)nt, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    // the active tiles in the order the full launch takes them
    std::vector<int> list;
    list.reserve((size_t)nt);
    for (int lb = 0; lb < A.nblk; ++lb) {
        int ty, tz, cx;
        if (!tile_of(lb, A.order, A.nyt, A.nzt, ty, tz, cx)) continue;
        const int t = (cx * A.nyt + ty) * A.nzt + tz;
        if (!h[(size_t)t]) list.push_back(t);
    }
    if (!list.empty()) {
        if ((e = hipMemcpyAsync(act, list.data(), sizeof(int) * list.size(), hipMemcpyHostToDevice, s)) !=
            hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;   // list is a host temporary
    }
    *ntiles = nt;
    *nact = (int)list.size();
    return hipSuccess;
}

// One launch of k_fused2 with the given shape over the full tiling or the
// active list.
template <typename R, int TYH, int LW, int PD>
void run_fused2(const FArgs<R>& A, const int* act, int nact, hipStream_t s)
{
    if (!act) k_fused2<R, TYH, LW, PD><<<A.nblk, TYH * LW, 0, s>>>(A, nullptr);
    else if (nact > 0) k_fused2<R, TYH, LW, PD><<<nact, TYH * LW, 0, s>>>(A, act);
}

template <typename R>
int64_t fused2_blocks(Geo g, int xchunk, int order)
{
    Fields<R> none = {};
    Mat<R> M = {};
    FArgs<R> A = fused_args<R>(none, none, M, g, R(0), Src{});
    if (!fused2_setup<R>(A, 16, xchunk, order, 32)) return -1;
    return A.nblk;
}

template <typename R>
hipError_t launch_step_fused2(Fields<R> o, Fields<R> nf, Mat<R> M, Geo g, R alpha, Src src, const WitMid<R>* wm,
                              int rows, int depth, int xchunk, int order, hipStream_t s, hipEvent_t* ev,
                              const int* act, int nact, const EnergyPair* en)
{
    if (en && en->want) {
        // energy samples: the default shape over the full tiling, vacuum
        FArgs<R> A = fused_args<R>(o, nf, M, g, alpha, src);
        // 16 rows of 32 lanes: 512 threads, whose VGPRs hold the sums'
        // operands (FP32 two planes ahead, FP64 one)
        // (materials by class: their energy coefficients from en->craw; witness
        // lines on vacuum grids only)
        if (act || (M.arr[0] && !A.cls) || (A.cls && (!en->craw || wm)) || !fused2_setup<R>(A, 16, xchunk, order, 32))
            return hipErrorInvalidValue;
        if (wm && (wm->iw < 1 || wm->iw > g.nx - 1 || wm->jw < 1 || wm->jw > g.ny - 1)) return hipErrorInvalidValue;
        if (A.nblk > en->cap) return hipErrorInvalidValue;
        hipError_t e;
        if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
        constexpr int EPD = sizeof(R) == 4 ? 2 : 1;   // FP64: one plane ahead fits the VGPRs
        const EnOut eo = {en->part, en->want, en->alpha, en->craw, nullptr};
        if (A.cls) {
            k_fused2_en_cls<R, 16, 32, EPD><<<A.nblk, 16 * 32, 0, s>>>(A, eo);
        } else if (wm) {
            k_fused2_en_wit<R, 16, 32, EPD><<<A.nblk, 16 * 32, 0, s>>>(A, eo, *wm);
        } else {
            k_fused2_en<R, 16, 32, EPD><<<A.nblk, 16 * 32, 0, s>>>(A, eo);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
        int slot = 0;
        for (int b = 0; b < 2; ++b)
            if (en->want & (1 << b))
                if ((e = launch_sum(en->part + b, A.nblk, 2, en->out + slot++, s)) != hipSuccess) return e;
        if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
        return hipSuccess;
    }
    FArgs<R> A = fused_args<R>(o, nf, M, g, alpha, src);
    if (wm) rows = 0;   // the instance that keeps witness lines has the default shape only
    if (A.cls) {        // materials by class: the class instance's one shape, no witness lines
        if (wm) return hipErrorInvalidValue;
        rows = sizeof(R) == 4 ? 24 : 16;
    }
    // per-entry materials (FP32 only): one shape, 16 rows of 32 lanes; no
    // witness lines, no static-tile list
    const bool arr = !A.cls && M.arr[0] != nullptr;
    int lanes = 0;
    if (arr) {
        if (sizeof(R) != 4 || wm || act) return hipErrorInvalidValue;
        for (int c = 0; c < 6; ++c)
            if (!M.arr[c]) return hipErrorInvalidValue;
        rows = 16;
        lanes = 32;
    }
    // with a list of active tiles, one workgroup per entry (none: every tile is
    // static and the new set already holds the result)
    const int grid = act ? nact : 0;
    if (!fused2_setup<R>(A, rows, xchunk, order, lanes)) return hipErrorInvalidValue;
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    bool done = false;
    if constexpr (sizeof(R) == 4) {
        if (arr) {
            Arr6<R> MA;
            for (int c = 0; c < 6; ++c) MA.m[c] = M.arr[c];
            k_fused2_arr<R, 16, 32, 2><<<A.nblk, 16 * 32, 0, s>>>(A, MA, nullptr);
            done = true;
        }
    }
    if (wm) {
        if (wm->iw < 1 || wm->iw > g.nx - 1 || wm->jw < 1 || wm->jw > g.ny - 1) return hipErrorInvalidValue;
        constexpr int TW = Default2<R>::rows * Default2<R>::lw;
        if (!act) k_fused2_wit<R, Default2<R>::rows, Default2<R>::lw><<<A.nblk, TW, 0, s>>>(A, *wm, nullptr);
        else if (grid > 0) k_fused2_wit<R, Default2<R>::rows, Default2<R>::lw><<<grid, TW, 0, s>>>(A, *wm, act);
        done = true;
    }
    if (!done && A.cls) {
        // materials by class: one shape per field type (FP32: 24 rows of 32
        // lanes, two planes ahead, 167 VGPRs; FP64: 16 rows of 32 lanes, one
        // plane ahead), whatever the tuning asks
        constexpr int CR = sizeof(R) == 4 ? 24 : 16, CP = sizeof(R) == 4 ? 2 : 1;
        if (!act) k_fused2_cls<R, CR, 32, CP><<<A.nblk, CR * 32, 0, s>>>(A, nullptr);
        else if (grid > 0) k_fused2_cls<R, CR, 32, CP><<<grid, CR * 32, 0, s>>>(A, act);
        done = true;
    }
    if constexpr (sizeof(R) == 4) {
        // FP32 shapes: rows 16 (64 lanes, one plane ahead, or two with depth 2),
        // 24 (32 lanes, two planes ahead, or depth 1 or 3), 32 (32 lanes, one
        // plane ahead)
        if (!done && rows == 32) {
            run_fused2<R, 32, 32, 1>(A, act, grid, s);
            done = true;
        } else if (!done && rows == 24) {
            if (depth == 1) run_fused2<R, 24, 32, 1>(A, act, grid, s);
            else if (depth == 3) run_fused2<R, 24, 32, 3>(A, act, grid, s);
            else run_fused2<R, 24, 32, 2>(A, act, grid, s);
            done = true;
        } else if (!done && depth == 2) {
            run_fused2<R, 16, 64, 2>(A, act, grid, s);
            done = true;
        }
    }
    if (!done) run_fused2<R, Default2<R>::rows, Default2<R>::lw, Default2<R>::pd>(A, act, grid, s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    return hipSuccess;
}

#define TETE_FUSED2_INST(R)                                                                                    \
    template hipError_t launch_batch_step2<R>(BatchTable<R>*, int, int, int, hipStream_t);                     \
    template bool fused2_setup<R>(FArgs<R>&, int, int, int, int);                                              \
    template hipError_t launch_step_fused2<R>(Fields<R>, Fields<R>, Mat<R>, Geo, R, Src, const WitMid<R>*, int, \
                                              int, int, int, hipStream_t, hipEvent_t*, const int*, int,      \
                                              const EnergyPair*);                                            \
    template int64_t fused2_blocks<R>(Geo, int, int);                                                         \
    template hipError_t fused2_static_tiles<R>(const uint8_t*, Geo, int, int, int, uint8_t*, int*, int64_t,    \
                                               int64_t*, int*, hipStream_t);
TETE_FUSED2_INST(float)
TETE_FUSED2_INST(double)

}  // namespace tete
