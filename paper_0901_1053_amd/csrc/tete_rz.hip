// Rotationally symmetric structures: scheme (24) of Sec. 4.3 for one
// azimuthal harmonic m on an r-z grid -- the step kernel, its diagnostics and
// the tete_rz_* entry points of include/tete.h.
//
// Kernel design.  The step has no third direction to march along, so each
// wave owns a strip of 64 consecutive k (one per lane; neighbours along z are
// DPP lane shifts, lanes 0 and 63 are halo) and marches along r over a chunk
// of rows.  The r-dependencies of the ten sub-updates fix a two-row lag: when
// row p has been loaded, S1, S2, S3, S5 and S6 run at row p-1 and S4, S7, S8,
// S9 and S10 at row p-2, which is then final and stored.  Everything a row
// needs from its neighbours stays in registers, so there is no LDS and no
// barrier; a chunk re-reads two rows on each side.  Loads run PF rows ahead
// of the march.  Coefficients depend on r only: one table row per radius,
// read with scalar loads.  Fields are read from one time level and written to
// the other (chunks read each other's halo rows).

#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "tete_dev.h"

namespace tete {
namespace {

constexpr double kEps0 = 8.8541878128e-12;   // vacuum permittivity [F/m] (CODATA 2018)
constexpr double kPi = 3.14159265358979323846;
constexpr int kLanes = 64;                   // lanes per wave
constexpr int kWaves = 4;                    // waves (z-strips) per workgroup
constexpr int kPad = 4;                      // coefficient rows below 0 and above nr
constexpr int kRedBlocks = 1024, kRedThreads = 256;

// Node code bits: e edge PEC or absent; HK = no h_phi / h_r at this k (k = nz).
enum { C_EPHI = 1, C_ER = 2, C_EZ = 4, C_HK = 8, C_ALL = 15 };

// Update coefficients of one radius: a kappa_phi, a kappa_r, 2a kappa_z f_e,
// a mu_phi, a mu_r, 2a mu_z f_h with the implicit factors f_e = (1 + a^2 m^2
// kappa_z mu_r)^-1 and f_h = (1 + a^2 m^2 mu_z kappa_r)^-1.
template <typename R>
struct Coef {
    R cp, cr, cz, dp, dr, dz;
};

// kappa and mu of one radius (FP64, for the energy and set-up).
struct Raw {
    double kp, kr, kz, mp, mr, mz;
};

template <typename R>
struct RZArgs {
    const R* o[6];          // y^n: e_phi, e_r, e_z, h_phi, h_r, h_z
    R* w[6];                // y^{n+1}
    const uint8_t* code;
    const Coef<R>* coef;    // rows -kPad .. nr+kPad, entry 0 is row -kPad
    int nr, nz, sz;         // sz = nz + 1
    R m;                    // harmonic m
    int nzt, nzb, rows;     // z-strips, workgroups along z, rows per chunk
    int nrc, order;         // r-chunks, workgroup order (1: chunks fastest, 2: strips fastest)
    int src, j0, M, jw, jmin, nw;
    int kend;               // the wake quadrature takes edges k < kend
    int64_t n;              // step being taken
    const double* lamw;     // 2M+1: harmonic weight * cell charge / dtau
    double* acc;            // [step parity][line jw, jw+1][nw] wake accumulators
};

template <typename R>
struct Row {
    R ez, er, ep, hp, hr, hz;
    uint32_t c;             // the dword holding the node's code byte (loaded rows)
};

// Values of one row after a step.
template <typename R>
struct Fin {
    R hp, hr, ez, ep, er, hz;
};

// March state of one step along r.  With q the row it takes in: old values
// of row q-1, the partial results of row q-2 and the new h_z of row q-3.
// advance() runs S1, S2, S3, S5, S6 at row q-1 and S4, S7, S8, S9, S10 at row
// q-2, which it returns final.  The PEC / absence bits zero the coefficient of
// a masked entry (x + 0 * d == x) instead of selecting the result: a select
// around an update can be compiled into a branch, and a lane shift inside it
// would then read 0 from the lanes the branch disables.
template <typename R>
struct Stage {
    R EZ1 = 0, ER1 = 0, EP1 = 0, HP1 = 0, HR1 = 0, HZ1 = 0;
    uint32_t C1 = C_ALL;
    R HZ2 = 0, HPn2 = 0, EZh2 = 0, ER2 = 0, HRh2 = 0, EPh2 = 0;
    uint32_t C2 = C_ALL;
    R HZn3 = 0;

    // src(C1, cz1, ez_old, ez_new) adds the current to e_z of row q-1 and
    // accumulates the wake there.
    template <typename F>
    __device__ __forceinline__ Fin<R> advance(const Row<R>& cur, uint32_t cq, const Coef<R>& c1,
                                              const Coef<R>& c2, R m, F&& src)
    {
        const R hp1 = (C1 & C_HK) ? (R)0 : c1.dp, hr1c = (C1 & C_HK) ? (R)0 : c1.dr;
        const R ez1c = (C1 & C_EZ) ? (R)0 : c1.cz, ep1c = (C1 & C_EPHI) ? (R)0 : c1.cp;
        const R hp2 = (C2 & C_HK) ? (R)0 : c2.dp, er2c = (C2 & C_ER) ? (R)0 : c2.cr;
        const R ep2c = (C2 & C_EPHI) ? (R)0 : c2.cp;

        // S1 at q-1: h_phi^n = h_phi^{n-1/2} + a mu_phi [P_z e_r^n - P_r e_z^{n-1/2}]
        const R hpn1 = HP1 + hp1 * ((lane_next(ER1) - ER1) - (cur.ez - EZ1));
        // S2 at q-1: h_r^n = h_r^{n-1/2} + a mu_r [-P_z e_phi^n + m e_z^{n-1/2}]
        const R pzEP1 = lane_next(EP1) - EP1;
        const R hrn1 = HR1 + hr1c * (m * EZ1 - pzEP1);
        // S3 at q-1: e_z^{n+1/2} = e_z^{n-1/2} + f_e 2a kappa_z [P_r^* h_phi^n - m h_r^n - j_z^n]
        R ezh1 = EZ1 + ez1c * ((HPn2 - hpn1) - m * hrn1);
        src(C1, c1.cz, EZ1, ezh1);
        // S5 at q-1: h_r^{n+1/2} = h_r^n + a mu_r [-P_z e_phi^n + m e_z^{n+1/2}]
        const R hrh1 = hrn1 + hr1c * (m * ezh1 - pzEP1);
        // S6 at q-1: e_phi^{n+1/2} = e_phi^n + a kappa_phi [P_z^* h_r^{n+1/2} - P_r^* h_z^n]
        const R eph1 = EP1 + ep1c * ((lane_prev(hrh1) - hrh1) - (HZ2 - HZ1));
        // S4 at q-2: h_phi^{n+1/2} = h_phi^n + a mu_phi [P_z e_r^n - P_r e_z^{n+1/2}]
        const R hph2 = HPn2 + hp2 * ((lane_next(ER2) - ER2) - (ezh1 - EZh2));
        // S7 at q-2: e_r^{n+1/2} = e_r^n + a kappa_r [-P_z^* h_phi^{n+1/2} + m h_z^n]
        const R pzsHP2 = lane_prev(hph2) - hph2;
        const R erh2 = ER2 + er2c * (m * HZ2 - pzsHP2);
        // S8 at q-2: h_z^{n+1} = h_z^n + f_h 2a mu_z [P_r e_phi^{n+1/2} - m e_r^{n+1/2}]
        const R hzn2 = HZ2 + c2.dz * ((eph1 - EPh2) - m * erh2);
        // S9 at q-2: e_phi^{n+1} = e_phi^{n+1/2} + a kappa_phi [P_z^* h_r^{n+1/2} - P_r^* h_z^{n+1}]
        const R ep2 = EPh2 + ep2c * ((lane_prev(HRh2) - HRh2) - (HZn3 - hzn2));
        // S10 at q-2: e_r^{n+1} = e_r^{n+1/2} + a kappa_r [-P_z^* h_phi^{n+1/2} + m h_z^{n+1}]
        const R er2 = erh2 + er2c * (m * hzn2 - pzsHP2);
        const Fin<R> f{hph2, HRh2, EZh2, ep2, er2, hzn2};

        // advance by one row
        HZn3 = hzn2;
        EPh2 = eph1;
        HRh2 = hrh1;
        ER2 = ER1;
        EZh2 = ezh1;
        HPn2 = hpn1;
        HZ2 = HZ1;
        C2 = C1;
        EZ1 = cur.ez;
        ER1 = cur.er;
        EP1 = cur.ep;
        HP1 = cur.hp;
        HR1 = cur.hr;
        HZ1 = cur.hz;
        C1 = cq;
        return f;
    }
};

// NS steps per launch (1 or 2).  With two, a second stage marches two rows
// behind the first and takes its final rows (step n+1) as input, so that a
// cell is read and written once per two steps; each step costs two rows of
// halo on either side of a chunk and one lane on either side of the strip.
template <typename R, int PF, int NS>
__global__ __launch_bounds__(kLanes * kWaves) void k_rz(RZArgs<R> A)
{
    constexpr uint32_t RB = sizeof(R);
    constexpr uint32_t OOB = 0x80000000u;
    constexpr int OWN = kLanes - 2 * NS;             // owned lanes NS .. 63-NS
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    // the wave index is uniform: taking it through a scalar register keeps the
    // early return below a scalar branch
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kLanes), lane = threadIdx.x % kLanes;
    // order 1: the r-chunks of one z-column are consecutive (neighbouring
    // chunks, which share halo rows, run together on one XCD); order 2: the
    // z-strips of one chunk are consecutive
    const int zg = A.order == 1 ? lb / A.nrc : lb % A.nzb;
    const int rc = A.order == 1 ? lb % A.nrc : lb / A.nzb;
    const int zt = zg * kWaves + wave;
    if (zt >= A.nzt) return;                          // whole wave
    const int k = zt * OWN - NS + lane;
    const bool kin = k >= 0 && k <= A.nz;
    const bool own_k = kin && lane >= NS && lane < kLanes - NS;
    const int ra = rc * A.rows, rb = min(ra + A.rows, A.nr + 1);
    const int L0 = max(0, ra - 2 * NS), pend = rb + 2 * NS - 1;

    const uint32_t np = (uint32_t)(A.nr + 1) * (uint32_t)A.sz;
    auto mk = [](const void* base, uint32_t bytes) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
    };
    const auto rEP = mk(A.o[0], np * RB), rER = mk(A.o[1], np * RB), rEZ = mk(A.o[2], np * RB),
               rHP = mk(A.o[3], np * RB), rHR = mk(A.o[4], np * RB), rHZ = mk(A.o[5], np * RB);
    const auto sEP = mk(A.w[0], np * RB), sER = mk(A.w[1], np * RB), sEZ = mk(A.w[2], np * RB),
               sHP = mk(A.w[3], np * RB), sHR = mk(A.w[4], np * RB), sHZ = mk(A.w[5], np * RB);
    const auto rC = mk(A.code, np + 4);

    auto load = [&](int p) {
        Row<R> v;
        const bool ok = kin && p <= A.nr;
        const uint32_t idx = (uint32_t)p * (uint32_t)A.sz + (uint32_t)k;
        const uint32_t off = ok ? idx * RB : OOB;
        v.ez = bload<R>(rEZ, off);
        v.er = bload<R>(rER, off);
        v.ep = bload<R>(rEP, off);
        v.hp = bload<R>(rHP, off);
        v.hr = bload<R>(rHR, off);
        v.hz = bload<R>(rHZ, off);
        // the code byte is read as the aligned dword that holds it (out of range
        // the load returns 0); the byte is extracted when the row is used, so
        // that no wait for this load sits between the prefetch and the compute
        v.c = __builtin_amdgcn_raw_buffer_load_b32(rC, ok ? (idx & ~3u) : OOB, 0, 0);
        return v;
    };
    auto code_of = [&](int p, uint32_t cw) {
        const bool ok = kin && p <= A.nr;
        const uint32_t idx = (uint32_t)p * (uint32_t)A.sz + (uint32_t)k;
        return ((cw >> (8 * (idx & 3u))) & 0xffu) | (ok ? 0u : (uint32_t)C_ALL);
    };
    // The coefficient table is read through the constant address space with a
    // uniform row index: scalar loads, outside the vector-memory counter that
    // the row prefetch relies on (a vector load of it would wait for the
    // prefetched rows too).
    typedef const __attribute__((address_space(4))) R* CR;
    const CR ctab = (CR)(const void*)A.coef;
    auto coef = [&](int row) {
        const int o = __builtin_amdgcn_readfirstlane(row + kPad) * 6;
        Coef<R> c;
        c.cp = ctab[o + 0];
        c.cr = ctab[o + 1];
        c.cz = ctab[o + 2];
        c.dp = ctab[o + 3];
        c.dr = ctab[o + 4];
        c.dz = ctab[o + 5];
        return c;
    };
    // bunch current and wake lines of the step with index n at row j1
    auto source = [&](int j1, int64_t n) {
        return [&, j1, n](uint32_t C1, R cz1, R ezold, R& ezh1) {
            if (A.src && j1 == A.j0 && !(C1 & C_EZ) && k < A.nz) {
                const int64_t mm = (int64_t)k - n + A.M;         // cell mm crosses edge k in step n
                if (mm >= -A.M && mm <= A.M) {
                    // the current term is rounded on its own, as in the 3-D kernels
#pragma clang fp contract(off)
                    ezh1 -= (R)((double)cz1 * A.lamw[mm + A.M]);
                }
            }
            if (A.src && (j1 == A.jw || j1 == A.jw + 1) && j1 >= ra && j1 < rb && own_k && k < A.kend) {
                const int64_t js = n - k - A.M;                  // wake sample of edge k
                // even and odd steps accumulate into separate arrays: in a two-step
                // launch lane k's step n and lane k+1's step n+1 meet at one sample
                if (js >= A.jmin && js < (int64_t)A.jmin + A.nw)
                    A.acc[((int)(n & 1) * 2 + (j1 - A.jw)) * A.nw + (js - A.jmin)] +=
                        -0.5 * ((double)ezold + (double)ezh1);
            }
        };
    };
    auto store = [&](int q, const Fin<R>& f) {
        const bool st = own_k && q >= ra && q < rb;
        const uint32_t so = st ? ((uint32_t)q * (uint32_t)A.sz + (uint32_t)k) * RB : OOB;
        bstore<R>(sHP, so, f.hp);
        bstore<R>(sHR, so, f.hr);
        bstore<R>(sEZ, so, f.ez);
        bstore<R>(sEP, so, f.ep);
        bstore<R>(sER, so, f.er);
        bstore<R>(sHZ, so, f.hz);
    };

    const R m = A.m;
    Stage<R> SA, SB;
    Row<R> ring[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u) ring[u] = load(L0 + u);

    for (int p0 = L0; p0 <= pend; p0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int p = p0 + u;
            if (p > pend) break;
            const Row<R> cur = ring[u];
            ring[u] = load(p + PF);
            const uint32_t c_m2 = SA.C2;                 // code of row p-2
            const Fin<R> fa = SA.advance(cur, code_of(p, cur.c), coef(p - 1), coef(p - 2), m,
                                         source(p - 1, A.n));
            if constexpr (NS == 1) {
                store(p - 2, fa);
            } else {
                // row p-2 after step n is the second stage's input row
                const Row<R> rin{fa.ez, fa.er, fa.ep, fa.hp, fa.hr, fa.hz, 0u};
                const Fin<R> fb = SB.advance(rin, c_m2, coef(p - 3), coef(p - 4), m, source(p - 3, A.n + 1));
                store(p - 4, fb);
            }
        }
    }
}

// Node codes from a cell mask (NULL: empty pillbox).  Cells outside r < nr dr
// and 0 < z < nz dz are PEC; row j = -1 mirrors j = 0 (the axis is no wall).
__device__ __forceinline__ bool cell_pec(const uint8_t* cells, int nr, int nz, int j, int k)
{
    if (k < 0 || k >= nz || j >= nr) return true;
    if (j < 0) j = 0;
    return cells ? cells[(int64_t)k + (int64_t)nz * j] != 0 : false;
}

__global__ void k_rz_code(const uint8_t* cells, uint8_t* code, int nr, int nz)
{
    const int64_t np = (int64_t)(nr + 1) * (nz + 1);
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < np;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(idx / (nz + 1)), k = (int)(idx % (nz + 1));
        const bool a = cell_pec(cells, nr, nz, j - 1, k - 1), b = cell_pec(cells, nr, nz, j, k - 1),
                   c = cell_pec(cells, nr, nz, j - 1, k), d = cell_pec(cells, nr, nz, j, k);
        uint32_t v = 0;
        if (a || b || c || d) v |= C_EPHI;
        if (j >= nr || b || d) v |= C_ER;
        if (k >= nz || c || d) v |= C_EZ;
        if (k >= nz) v |= C_HK;
        code[idx] = (uint8_t)v;
    }
}

// Zero every entry outside its index range and e on PEC edges (also e_phi on
// the axis and, for m >= 1, e_z on the axis, whose kappa is zero).
template <typename R>
__global__ void k_rz_sanitize(R* const* f, const uint8_t* code, const Raw* raw, int nr, int nz)
{
    const int64_t np = (int64_t)(nr + 1) * (nz + 1);
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < np;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(idx / (nz + 1)), k = (int)(idx % (nz + 1));
        const uint32_t c = code[idx];
        if ((c & C_EPHI) || raw[j].kp == 0.0) f[0][idx] = 0;
        if ((c & C_ER) || raw[j].kr == 0.0) f[1][idx] = 0;
        if ((c & C_EZ) || raw[j].kz == 0.0) f[2][idx] = 0;
        if (j >= nr || k >= nz) f[3][idx] = 0;
        if (j == 0 || k >= nz) f[4][idx] = 0;
        if (j >= nr) f[5][idx] = 0;
    }
}

template <typename D, typename S>
__global__ void k_rz_convert(D* dst, const S* src, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (D)src[i];
}

__device__ double block_sum(double v)
{
    __shared__ double s[kRedThreads];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    return s[0];
}

// Energy 1/2 <Q y, y> of (24), summed per node:
//   1/2 [sum h^2/mu + sum_{kappa>0} e^2/kappa]
//   - a^2/2 [sum_{h_phi} mu_phi (P_r e_z)^2 + sum_{e_phi, kappa>0} kappa_phi (P_r^T h_z)^2]
//   + a [sum_{h_phi} h_phi P_z e_r - sum_{h_r} h_r P_z e_phi]
template <typename R>
__global__ __launch_bounds__(kRedThreads) void k_rz_energy(const R* const* f, const uint8_t* code, const Raw* raw,
                                                         int nr, int nz, double a, double* partial)
{
    const R *ep = f[0], *er = f[1], *ez = f[2], *hp = f[3], *hr = f[4], *hz = f[5];
    const int sz = nz + 1;
    const int64_t np = (int64_t)(nr + 1) * sz;
    double acc = 0.0;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < np;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(idx / sz), k = (int)(idx % sz);
        const uint32_t c = code[idx];
        const Raw w = raw[j];
        double sq = 0.0, r = 0.0, lc = 0.0;
        const double kp = (c & C_EPHI) ? 0.0 : w.kp, kr = (c & C_ER) ? 0.0 : w.kr, kz = (c & C_EZ) ? 0.0 : w.kz;
        if (kp > 0.0) {
            const double e = ep[idx], d = (j > 0 ? (double)hz[idx - sz] : 0.0) - (double)hz[idx];
            sq += e * e / kp;
            r += kp * d * d;
        }
        if (kr > 0.0) sq += (double)er[idx] * (double)er[idx] / kr;
        if (kz > 0.0) sq += (double)ez[idx] * (double)ez[idx] / kz;
        if (j < nr && k < nz && w.mp > 0.0) {
            const double h = hp[idx], d = (double)ez[idx + sz] - (double)ez[idx];
            sq += h * h / w.mp;
            r += w.mp * d * d;
            lc += h * ((double)er[idx + 1] - (double)er[idx]);
        }
        if (j > 0 && k < nz && w.mr > 0.0) {
            const double h = hr[idx];
            sq += h * h / w.mr;
            lc -= h * ((double)ep[idx + 1] - (double)ep[idx]);
        }
        if (j < nr && w.mz > 0.0) sq += (double)hz[idx] * (double)hz[idx] / w.mz;
        acc += 0.5 * sq - 0.5 * a * a * r + a * lc;
    }
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRedThreads) void k_rz_finish(const double* partial, int n, double* out)
{
    double v = 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) v += partial[t];
    const double s = block_sum(v);
    if (threadIdx.x == 0) *out = s;
}

// Wakes in V/C: W_par = (even + odd step sums) / (Q eps0) on both lines;
// W_perp by the trapezoidal s-integral of (line jw+1 - line jw) / dr from the
// first sample.
__global__ void k_rz_wakes(const double* acc, int nw, double scale, double dr, double ds, double* wpar,
                           double* wperp)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double prev = 0.0, run = 0.0;
    for (int j = 0; j < nw; ++j) {
        const double a0 = (acc[j] + acc[2 * nw + j]) * scale, a1 = (acc[nw + j] + acc[3 * nw + j]) * scale;
        wpar[j] = a0;
        wpar[nw + j] = a1;
        const double d = (a1 - a0) / dr;
        if (j > 0) run += 0.5 * (d + prev) * ds;
        wperp[j] = run;
        prev = d;
    }
}

size_t up(size_t v) { return (v + 255) / 256 * 256; }

// Open pipes (the infinite pipes of the structure of Sec. 5) on the r-z grid:
// the ring bunch's own field in a uniform entrance pipe as the starting state.
// With e_z = h_z = 0 the pairs (e_r, h_phi) and (e_phi, h_r) see the 1-D
// leapfrog at Courant number one along z; S8 keeps h_z = 0 for the radial
// gradient form e_r = -P_r Phi, e_phi = -m Phi; S3 keeps e_z = 0 when the
// radial problem
//   [r_{j-1/2}(Phi_j - Phi_{j-1}) - r_{j+1/2}(Phi_{j+1} - Phi_j)] / dr + m^2 (dr / r_j) Phi_j = delta_{j, j0}
// holds on the nodes whose e_z edge is free (r_{-1/2} = 0), Phi = 0 on the
// others, and the profile F carries the ring current (the weighted cell
// charges over dtau).  Then e_phi = -m Phi F(p), e_r = -(Phi_{j+1} - Phi_j) F(p),
// h_phi = (r_{j+1/2}/dr)(Phi_{j+1} - Phi_j) F(p+1), h_r = (dr/r_j) e_phi-shape F(p+1).

// bad = 1 unless every node line repeats, over planes 0 .. kst-1, the e_z bit
// of plane 0 and the e_phi, e_r bits of plane 1 (plane 0 of those is the wall)
__global__ void k_rz_pipe_check(const uint8_t* code, int nr, int nz, int kst, int* bad)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > nr) return;
    const uint8_t* c = code + (int64_t)j * (nz + 1);
    const int z0 = c[0] & C_EZ, t1 = c[1] & (C_EPHI | C_ER);
    int diff = 0;
    for (int k = 1; k < kst; ++k) diff |= ((c[k] & C_EZ) != z0) | ((c[k] & (C_EPHI | C_ER)) != t1);
    if (diff) *bad = 1;
}

// Phi by the Thomas algorithm (one thread; the system is tridiagonal and
// diagonally dominant).  A node is free when kappa_z > 0 and its plane-0 e_z
// edge is not PEC; other rows are Phi = 0.  cw, dw: nr + 1 doubles of work.
__global__ void k_rz_pipe_solve(const uint8_t* code, const Raw* raw, int nr, int nz, double dr, int m, int j0,
                                double* phi, double* cw, double* dw)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    auto free_node = [&](int j) { return raw[j].kz > 0.0 && !(code[(int64_t)j * (nz + 1)] & C_EZ); };
    double cp = 0.0, dp = 0.0;
    for (int j = 0; j <= nr; ++j) {
        double a = 0.0, b = 1.0, c = 0.0, d = 0.0;
        if (free_node(j)) {
            const double rm = j > 0 ? (j - 0.5) * dr : 0.0, rp = (j + 0.5) * dr;
            b = (rm + rp) / dr + (j > 0 ? (double)m * m * dr / (j * dr) : 0.0);
            if (j > 0 && rm != 0.0 && free_node(j - 1)) a = -(rm / dr);
            if (j < nr && free_node(j + 1)) c = -(rp / dr);
            d = j == j0 ? 1.0 : 0.0;
        }
        const double den = b - a * cp;
        cw[j] = c / den;
        dw[j] = (d - a * dp) / den;
        cp = cw[j];
        dp = dw[j];
    }
    phi[nr] = dw[nr];
    for (int j = nr - 1; j >= 0; --j) phi[j] = dw[j] - cw[j] * phi[j + 1];
}

__device__ __forceinline__ double rz_prof(const double* F, int lo, int64_t p)
{
    if (p > 0) return 0.0;
    if (p >= lo) return F[p - lo];
    return ((lo - p) & 1) ? -F[0] : F[0];
}

// The state y^{n0} of the field above into the six arrays f (sanitized after)
template <typename R>
__global__ void k_rz_pipe_field(R* const* f, const double* phi, const double* F, int lo, int64_t n0, int nr, int nz,
                                double dr, int m)
{
    const int64_t np = (int64_t)(nr + 1) * (nz + 1);
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < np;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(idx / (nz + 1)), k = (int)(idx % (nz + 1));
        const double fe = rz_prof(F, lo, (int64_t)k - n0), fh = rz_prof(F, lo, (int64_t)k + 1 - n0);
        const double Ep = -(double)m * phi[j];
        const double Er = j < nr ? -(phi[j + 1] - phi[j]) : 0.0;
        f[0][idx] = (R)(Ep * fe);
        f[1][idx] = (R)(Er * fe);
        f[2][idx] = R(0);
        f[3][idx] = (R)((((j + 0.5) * dr / dr) * (-Er)) * fh);
        f[4][idx] = j > 0 ? (R)(((dr / (j * dr)) * Ep) * fh) : R(0);
        f[5][idx] = R(0);
    }
}

struct RZLayout {
    size_t field[12], code, coef, raw, lamw, acc, partial, scal, wout, ptrs, total;
};

bool rz_valid(const tete_rz_desc* d)
{
    if (!d || d->nr < 2 || d->nz < 2 || d->mode < 0 || d->mode > 4096) return false;
    if (d->precision != TETE_FP64 && d->precision != TETE_FP32) return false;
    if (!(d->dr > 0.0) || !(d->dz > 0.0) || !(d->cdt > 0.0) || !isfinite(d->dr) || !isfinite(d->dz) ||
        !isfinite(d->cdt))
        return false;
    const int64_t np = (int64_t)(d->nr + 1) * (d->nz + 1);
    const int64_t rb = d->precision == TETE_FP32 ? 4 : 8;
    return np * rb < ((int64_t)1 << 31) - 256;
}

RZLayout rz_layout(const tete_rz_desc* d)
{
    RZLayout L;
    const size_t np = (size_t)(d->nr + 1) * (d->nz + 1);
    const size_t rb = d->precision == TETE_FP32 ? 4 : 8;
    size_t o = 0;
    for (int c = 0; c < 12; ++c) { L.field[c] = o; o = up(o + rb * np); }
    L.code = o;    o = up(o + np + 4);
    L.coef = o;    o = up(o + 6 * rb * (size_t)(d->nr + 1 + 2 * kPad));
    L.raw = o;     o = up(o + sizeof(Raw) * (size_t)(d->nr + 1));
    L.lamw = o;    o = up(o + sizeof(double) * TETE_MAX_BUNCH_CELLS);
    L.acc = o;     o = up(o + sizeof(double) * 4 * TETE_MAX_WAKE);
    L.partial = o; o = up(o + sizeof(double) * kRedBlocks);
    L.scal = o;    o = up(o + sizeof(double) * 8);
    L.wout = o;    o = up(o + sizeof(double) * 3 * TETE_MAX_WAKE);
    L.ptrs = o;    o = up(o + sizeof(void*) * 12);
    L.total = o;
    return L;
}

// Largest eigenvalue of the radial operator next to the axis for m = 0, in
// units of 1/dr^2 (dual facet dr^2/8 on the axis): limits cdt to 2/sqrt(.) dr.
constexpr double kAxisLambda = 4.8419422636;

}  // namespace
}  // namespace tete

using namespace tete;

struct tete_rz {
    tete_rz_desc d;
    hipStream_t stream;
    int device;
    char* ws;
    RZLayout L;
    int fp32;
    void* f[2][6];
    void** dptr;         // device copy of the 12 field pointers (set 0 then set 1)
    int cur;
    uint8_t* code;
    void* coef;
    Raw* raw;
    double *lamw, *acc, *partial, *scal, *wout;
    int64_t n;
    int has_bunch;
    tete_rz_bunch b;
    int32_t kend;        // open-pipe run: the wake quadrature ends before edge kend (0: all edges)
    int kernel, chunk_rows, prefetch;   // TETE_KERNEL_AUTO / FUSED (one step) / FUSED2 (two)
    int order;                          // workgroup order (0: default)
    int timing;
    hipEvent_t* ev;
    unsigned char* ev_nst;              // steps of each timed launch
    int64_t ev_cap, ev_used;
};

#define RZCHK(x)                                       \
    do {                                               \
        if ((x) != hipSuccess) return TETE_ERR_DEVICE; \
    } while (0)

namespace {

// kappa, mu per radian (vacuum) and the update coefficients of radius j.
void rz_raw(const tete_rz_desc* d, std::vector<Raw>& raw)
{
    const int nr = d->nr;
    const double dr = d->dr, dz = d->dz;
    raw.assign(nr + 1, Raw{0, 0, 0, 0, 0, 0});
    for (int j = 0; j <= nr; ++j) {
        const double r = j * dr, rh = (j + 0.5) * dr;
        Raw& w = raw[j];
        w.kp = j > 0 && j < nr ? r / (dr * dz) : 0.0;                          // wall e_phi is PEC
        w.kr = j < nr ? dr / (rh * dz) : 0.0;
        w.kz = j == 0 ? (d->mode == 0 ? dz / (dr * dr / 8.0) : 0.0) : (j < nr ? dz / (r * dr) : 0.0);
        w.mp = j < nr ? rh / (dr * dz) : 0.0;
        w.mr = j > 0 ? dr / (r * dz) : 0.0;
        w.mz = j < nr ? dz / (rh * dr) : 0.0;
    }
}

template <typename R>
void rz_coef(const tete_rz_desc* d, const std::vector<Raw>& raw, std::vector<Coef<R>>& co)
{
    const double a = 0.5 * d->cdt, mm = (double)d->mode * (double)d->mode;
    co.assign(d->nr + 1 + 2 * kPad, Coef<R>{0, 0, 0, 0, 0, 0});
    for (int j = 0; j <= d->nr; ++j) {
        const Raw& w = raw[j];
        const double fe = 1.0 / (1.0 + a * a * mm * w.kz * w.mr);
        const double fh = 1.0 / (1.0 + a * a * mm * w.mz * w.kr);
        Coef<R>& c = co[j + kPad];
        c.cp = (R)(a * w.kp);
        c.cr = (R)(a * w.kr);
        c.cz = (R)(fe * 2.0 * a * w.kz);
        c.dp = (R)(a * w.mp);
        c.dr = (R)(a * w.mr);
        c.dz = (R)(fh * 2.0 * a * w.mz);
    }
}

// z-strips of a launch taking ns steps: each owns 64 - 2 ns consecutive k
int rz_nzt(const tete_rz_desc* d, int ns)
{
    const int own = kLanes - 2 * ns;
    return (d->nz + 1 + own - 1) / own;
}

// Rows per r-chunk: 16 by default.  Short chunks give many workgroups (about
// 19 rounds of 256 on the 1000 x 18183 deflector-like grid), so the last
// round's tail is small; their halo rows are re-read mostly from L2.  On that
// grid 16 rows measured within 3 % of the best of 16 .. 256 for both kernels
// and precisions, while automatic chunks of 72 rows were 8 % slower.
int rz_rows(const tete_rz* g, int ns)
{
    (void)ns;
    return g->chunk_rows > 0 ? g->chunk_rows : 16;
}

template <typename R, int NS>
void rz_kernel(int pf, dim3 grid, dim3 block, hipStream_t s, const RZArgs<R>& A)
{
    switch (pf) {
        case 1: k_rz<R, 1, NS><<<grid, block, 0, s>>>(A); break;
        case 3: k_rz<R, 3, NS><<<grid, block, 0, s>>>(A); break;
        case 4: k_rz<R, 4, NS><<<grid, block, 0, s>>>(A); break;
        default: k_rz<R, 2, NS><<<grid, block, 0, s>>>(A); break;
    }
}

// One launch taking ns (1 or 2) steps from y^n in set cur to the other set.
template <typename R>
hipError_t rz_launch(tete_rz* g, int ns, hipStream_t s)
{
    RZArgs<R> A;
    const int in = g->cur, out = 1 - g->cur;
    for (int c = 0; c < 6; ++c) {
        A.o[c] = (const R*)g->f[in][c];
        A.w[c] = (R*)g->f[out][c];
    }
    A.code = g->code;
    A.coef = (const Coef<R>*)g->coef;
    A.nr = g->d.nr;
    A.nz = g->d.nz;
    A.sz = g->d.nz + 1;
    A.m = (R)g->d.mode;
    A.nzt = rz_nzt(&g->d, ns);
    A.nzb = (A.nzt + kWaves - 1) / kWaves;
    A.rows = rz_rows(g, ns);
    A.src = g->has_bunch;
    A.j0 = g->b.j0;
    A.M = g->b.half_cells;
    A.jw = g->b.jw;
    A.jmin = g->b.jmin;
    A.nw = g->b.nw;
    A.kend = g->kend > 0 ? g->kend : g->d.nz;
    A.n = g->n;
    A.lamw = g->lamw;
    A.acc = g->acc;
    const int nrc = (g->d.nr + 1 + A.rows - 1) / A.rows;
    A.nrc = nrc;
    A.order = g->order > 0 ? g->order : 2;
    const dim3 grid((unsigned)(A.nzb * nrc)), block(kLanes * kWaves);
    const int pf = g->prefetch > 0 ? g->prefetch : 2;
    if (ns == 2) rz_kernel<R, 2>(pf, grid, block, s, A);
    else rz_kernel<R, 1>(pf, grid, block, s, A);
    return hipGetLastError();
}

template <typename R>
hipError_t rz_sanitize(tete_rz* g, int set)
{
    R* const* p = (R* const*)(g->dptr + 6 * set);
    k_rz_sanitize<R><<<512, 256, 0, g->stream>>>(p, g->code, g->raw, g->d.nr, g->d.nz);
    return hipGetLastError();
}

hipError_t rz_sanitize_any(tete_rz* g, int set)
{
    return g->fp32 ? rz_sanitize<float>(g, set) : rz_sanitize<double>(g, set);
}

struct Guard {
    int prev = -1;
    bool ok = true;
    explicit Guard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~Guard()
    {
        int c;
        if (prev >= 0 && hipGetDevice(&c) == hipSuccess && c != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

tete_status tete_rz_check_desc(const tete_rz_desc* d)
{
    if (!rz_valid(d)) return TETE_ERR_ARG;
    const double tol = 1.0 + 1e-12;
    if (d->cdt > d->dz * tol) return TETE_ERR_UNSTABLE;
    const double rlim = d->mode == 0 ? 2.0 / sqrt(kAxisLambda) * d->dr : d->dr;
    if (d->cdt > rlim * tol) return TETE_ERR_UNSTABLE;
    return TETE_OK;
}

size_t tete_rz_workspace_bytes(const tete_rz_desc* d)
{
    if (!rz_valid(d)) return 0;
    return rz_layout(d).total;
}

tete_status tete_rz_create(const tete_rz_desc* d, void* dev_ws, size_t ws_bytes, void* hip_stream, tete_rz** out)
{
    if (!out || !dev_ws || ((uintptr_t)dev_ws & 255)) return TETE_ERR_ARG;
    *out = nullptr;
    const tete_status st = tete_rz_check_desc(d);
    if (st != TETE_OK) return st;
    const RZLayout L = rz_layout(d);
    if (ws_bytes < L.total) return TETE_ERR_NOMEM;
    tete_rz* g = (tete_rz*)calloc(1, sizeof(tete_rz));
    if (!g) return TETE_ERR_NOMEM;
    g->d = *d;
    g->stream = (hipStream_t)hip_stream;
    g->ws = (char*)dev_ws;
    g->L = L;
    g->fp32 = d->precision == TETE_FP32;
    if (hipGetDevice(&g->device) != hipSuccess) { free(g); return TETE_ERR_DEVICE; }
    for (int s = 0; s < 2; ++s)
        for (int c = 0; c < 6; ++c) g->f[s][c] = g->ws + L.field[6 * s + c];
    g->dptr = (void**)(g->ws + L.ptrs);
    g->code = (uint8_t*)(g->ws + L.code);
    g->coef = g->ws + L.coef;
    g->raw = (Raw*)(g->ws + L.raw);
    g->lamw = (double*)(g->ws + L.lamw);
    g->acc = (double*)(g->ws + L.acc);
    g->partial = (double*)(g->ws + L.partial);
    g->scal = (double*)(g->ws + L.scal);
    g->wout = (double*)(g->ws + L.wout);
    std::vector<Raw> raw;
    rz_raw(d, raw);
    hipError_t e = hipMemsetAsync(g->ws, 0, L.total, g->stream);
    void* ptrs[12];
    for (int s = 0; s < 2; ++s)
        for (int c = 0; c < 6; ++c) ptrs[6 * s + c] = g->f[s][c];
    if (e == hipSuccess) e = hipMemcpyAsync(g->dptr, ptrs, sizeof(ptrs), hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->raw, raw.data(), sizeof(Raw) * raw.size(), hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess) {
        if (g->fp32) {
            std::vector<Coef<float>> co;
            rz_coef<float>(d, raw, co);
            e = hipMemcpyAsync(g->coef, co.data(), sizeof(Coef<float>) * co.size(), hipMemcpyHostToDevice, g->stream);
        } else {
            std::vector<Coef<double>> co;
            rz_coef<double>(d, raw, co);
            e = hipMemcpyAsync(g->coef, co.data(), sizeof(Coef<double>) * co.size(), hipMemcpyHostToDevice,
                               g->stream);
        }
    }
    if (e == hipSuccess) {
        k_rz_code<<<512, 256, 0, g->stream>>>(nullptr, g->code, d->nr, d->nz);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) { free(g); return TETE_ERR_DEVICE; }
    *out = g;
    return TETE_OK;
}

tete_status tete_rz_destroy(tete_rz* g)
{
    if (!g) return TETE_ERR_ARG;
    if (g->ev) {
        for (int64_t i = 0; i < 2 * g->ev_cap; ++i) (void)hipEventDestroy(g->ev[i]);
        free(g->ev);
    }
    free(g->ev_nst);
    free(g);
    return TETE_OK;
}

tete_status tete_rz_set_pec_cells(tete_rz* g, const uint8_t* cells)
{
    if (!g) return TETE_ERR_ARG;
    Guard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    k_rz_code<<<512, 256, 0, g->stream>>>(cells, g->code, g->d.nr, g->d.nz);
    RZCHK(hipGetLastError());
    RZCHK(rz_sanitize_any(g, g->cur));
    g->kend = 0;
    return TETE_OK;
}

tete_status tete_rz_set_fields(tete_rz* g, const void* const f[6], int32_t dtype)
{
    if (!g || !f || (dtype != TETE_FP64 && dtype != TETE_FP32)) return TETE_ERR_ARG;
    for (int c = 0; c < 6; ++c)
        if (!f[c]) return TETE_ERR_ARG;
    Guard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    const int64_t np = (int64_t)(g->d.nr + 1) * (g->d.nz + 1);
    for (int c = 0; c < 6; ++c) {
        void* dst = g->f[g->cur][c];
        if (g->fp32 && dtype == TETE_FP32)
            k_rz_convert<float, float><<<512, 256, 0, g->stream>>>((float*)dst, (const float*)f[c], np);
        else if (g->fp32)
            k_rz_convert<float, double><<<512, 256, 0, g->stream>>>((float*)dst, (const double*)f[c], np);
        else if (dtype == TETE_FP32)
            k_rz_convert<double, float><<<512, 256, 0, g->stream>>>((double*)dst, (const float*)f[c], np);
        else
            k_rz_convert<double, double><<<512, 256, 0, g->stream>>>((double*)dst, (const double*)f[c], np);
        RZCHK(hipGetLastError());
    }
    RZCHK(rz_sanitize_any(g, g->cur));
    RZCHK(hipMemsetAsync(g->acc, 0, sizeof(double) * 4 * TETE_MAX_WAKE, g->stream));
    g->n = 0;
    g->kend = 0;
    return TETE_OK;
}

tete_status tete_rz_get_fields(tete_rz* g, void* const f[6], int32_t dtype)
{
    if (!g || !f || (dtype != TETE_FP64 && dtype != TETE_FP32)) return TETE_ERR_ARG;
    for (int c = 0; c < 6; ++c)
        if (!f[c]) return TETE_ERR_ARG;
    Guard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    const int64_t np = (int64_t)(g->d.nr + 1) * (g->d.nz + 1);
    for (int c = 0; c < 6; ++c) {
        const void* src = g->f[g->cur][c];
        if (g->fp32 && dtype == TETE_FP32)
            k_rz_convert<float, float><<<512, 256, 0, g->stream>>>((float*)f[c], (const float*)src, np);
        else if (g->fp32)
            k_rz_convert<double, float><<<512, 256, 0, g->stream>>>((double*)f[c], (const float*)src, np);
        else if (dtype == TETE_FP32)
            k_rz_convert<float, double><<<512, 256, 0, g->stream>>>((float*)f[c], (const double*)src, np);
        else
            k_rz_convert<double, double><<<512, 256, 0, g->stream>>>((double*)f[c], (const double*)src, np);
        RZCHK(hipGetLastError());
    }
    RZCHK(hipStreamSynchronize(g->stream));
    return TETE_OK;
}

tete_status tete_rz_set_bunch(tete_rz* g, const tete_rz_bunch* b)
{
    if (!g || !b) return TETE_ERR_ARG;
    const int M = b->half_cells;
    if (!(b->charge_C > 0.0) || !(b->sigma_z > 0.0) || !isfinite(b->charge_C) || !isfinite(b->sigma_z))
        return TETE_ERR_ARG;
    if (M < 0 || 2 * M + 1 > TETE_MAX_BUNCH_CELLS || b->nw < 1 || b->nw > TETE_MAX_WAKE) return TETE_ERR_ARG;
    if (b->j0 < 0 || b->j0 >= g->d.nr || (g->d.mode > 0 && b->j0 == 0)) return TETE_ERR_ARG;
    if (b->jw < 0 || b->jw + 1 >= g->d.nr || (g->d.mode > 0 && b->jw == 0)) return TETE_ERR_ARG;
    if (fabs(g->d.cdt - g->d.dz) > 1e-12 * g->d.dz) return TETE_ERR_STATE;
    Guard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    // cell charges of the truncated Gaussian (Fig. 1), times the harmonic
    // weight, as the current through a dual facet during one step
    const double w = g->d.mode == 0 ? 1.0 / (2.0 * kPi) : 1.0 / kPi;
    std::vector<double> lam(2 * M + 1);
    for (int mm = -M; mm <= M; ++mm) {
        const double lo = (mm - 0.5) * g->d.dz / b->sigma_z, hi = (mm + 0.5) * g->d.dz / b->sigma_z;
        double v;
        if (lo >= 0.0) v = 0.5 * (erfc(lo / sqrt(2.0)) - erfc(hi / sqrt(2.0)));
        else if (hi <= 0.0) v = 0.5 * (erfc(-hi / sqrt(2.0)) - erfc(-lo / sqrt(2.0)));
        else v = 1.0 - 0.5 * erfc(-lo / sqrt(2.0)) - 0.5 * erfc(hi / sqrt(2.0));
        lam[mm + M] = w * b->charge_C * v / g->d.cdt;
    }
    RZCHK(hipMemcpyAsync(g->lamw, lam.data(), sizeof(double) * lam.size(), hipMemcpyHostToDevice, g->stream));
    RZCHK(hipMemsetAsync(g->acc, 0, sizeof(double) * 4 * TETE_MAX_WAKE, g->stream));
    RZCHK(hipStreamSynchronize(g->stream));
    g->b = *b;
    g->has_bunch = 1;
    g->kend = 0;
    return TETE_OK;
}

tete_status tete_rz_step(tete_rz* g, int64_t nsteps)
{
    if (!g || nsteps < 0) return TETE_ERR_ARG;
    Guard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    const bool two = g->kernel != TETE_KERNEL_FUSED;
    for (int64_t s = 0; s < nsteps;) {
        const int ns = two && nsteps - s >= 2 ? 2 : 1;
        const bool rec = g->timing && g->ev_used < g->ev_cap;
        if (rec) RZCHK(hipEventRecord(g->ev[2 * g->ev_used], g->stream));
        RZCHK(g->fp32 ? rz_launch<float>(g, ns, g->stream) : rz_launch<double>(g, ns, g->stream));
        if (rec) {
            RZCHK(hipEventRecord(g->ev[2 * g->ev_used + 1], g->stream));
            g->ev_nst[g->ev_used] = (unsigned char)ns;
            ++g->ev_used;
        }
        g->cur = 1 - g->cur;
        g->n += ns;
        s += ns;
    }
    return TETE_OK;
}

tete_status tete_rz_set_open_pipes(tete_rz* g, int64_t start_step, int32_t kend)
{
    if (!g) return TETE_ERR_ARG;
    if (!g->has_bunch) return TETE_ERR_STATE;
    const int nr = g->d.nr, nz = g->d.nz;
    if (start_step < 0 || start_step >= nz || kend < 0 || kend > nz) return TETE_ERR_ARG;
    Guard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    int* bad = (int*)(g->scal + 6);
    RZCHK(launch_zero_bytes(bad, sizeof(int), g->stream));
    k_rz_pipe_check<<<(nr + 256) / 256, 256, 0, g->stream>>>(g->code, nr, nz, (int)start_step + 1, bad);
    RZCHK(hipGetLastError());
    int hbad = 0;
    uint8_t c0 = 0;
    Raw r0;
    const int j0 = g->b.j0;
    RZCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, g->stream));
    RZCHK(hipMemcpyAsync(&c0, g->code + (int64_t)j0 * (nz + 1), 1, hipMemcpyDeviceToHost, g->stream));
    RZCHK(hipMemcpyAsync(&r0, g->raw + j0, sizeof(Raw), hipMemcpyDeviceToHost, g->stream));
    RZCHK(hipStreamSynchronize(g->stream));
    if (hbad || (c0 & C_EZ) || !(r0.kz > 0.0)) return TETE_ERR_ARG;
    // scratch: three arrays of the other field set (each holds nr + 1 doubles)
    const int o = 1 - g->cur;
    double* phi = (double*)g->f[o][0];
    double* cw = (double*)g->f[o][1];
    double* dw = (double*)g->f[o][2];
    k_rz_pipe_solve<<<1, 64, 0, g->stream>>>(g->code, g->raw, nr, nz, g->d.dr, g->d.mode, j0, phi, cw, dw);
    RZCHK(hipGetLastError());
    // the profile of the ring current (weighted cell charges over dtau) in the
    // wake read-out area
    const int M = g->b.half_cells;
    RZCHK(launch_pipe_profile(g->wout, g->lamw, M, 1.0, g->stream));
    if (g->fp32)
        k_rz_pipe_field<float><<<512, 256, 0, g->stream>>>((float* const*)(g->dptr + 6 * g->cur), phi, g->wout,
                                                           -2 * M - 1, start_step, nr, nz, g->d.dr, g->d.mode);
    else
        k_rz_pipe_field<double><<<512, 256, 0, g->stream>>>((double* const*)(g->dptr + 6 * g->cur), phi, g->wout,
                                                            -2 * M - 1, start_step, nr, nz, g->d.dr, g->d.mode);
    RZCHK(hipGetLastError());
    RZCHK(rz_sanitize_any(g, g->cur));
    const size_t bytes = (size_t)(g->fp32 ? 4 : 8) * (size_t)(nr + 1) * (size_t)(nz + 1);
    for (int c = 0; c < 6; ++c) RZCHK(launch_zero_bytes(g->f[o][c], bytes, g->stream));
    RZCHK(launch_zero_bytes(g->acc, sizeof(double) * 4 * TETE_MAX_WAKE, g->stream));
    RZCHK(hipStreamSynchronize(g->stream));
    g->n = start_step;
    g->kend = kend;
    return TETE_OK;
}

tete_status tete_rz_steps_done(tete_rz* g, int64_t* n)
{
    if (!g || !n) return TETE_ERR_ARG;
    *n = g->n;
    return TETE_OK;
}

tete_status tete_rz_wake(tete_rz* g, double* W_par, double* W_perp, int32_t nw)
{
    if (!g || !W_par || !g->has_bunch || nw < 1 || nw > g->b.nw) return TETE_ERR_ARG;
    Guard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    const int n = g->b.nw;
    k_rz_wakes<<<1, 64, 0, g->stream>>>(g->acc, n, 1.0 / (g->b.charge_C * kEps0), g->d.dr, g->d.dz, g->wout,
                                        g->wout + 2 * n);
    RZCHK(hipGetLastError());
    RZCHK(hipMemcpyAsync(W_par, g->wout, sizeof(double) * nw, hipMemcpyDeviceToHost, g->stream));
    RZCHK(hipMemcpyAsync(W_par + nw, g->wout + n, sizeof(double) * nw, hipMemcpyDeviceToHost, g->stream));
    if (W_perp)
        RZCHK(hipMemcpyAsync(W_perp, g->wout + 2 * n, sizeof(double) * nw, hipMemcpyDeviceToHost, g->stream));
    RZCHK(hipStreamSynchronize(g->stream));
    return TETE_OK;
}

tete_status tete_rz_energy(tete_rz* g, double* W, int64_t* n)
{
    if (!g || !W) return TETE_ERR_ARG;
    Guard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    const double a = 0.5 * g->d.cdt;
    if (g->fp32)
        k_rz_energy<float><<<kRedBlocks, kRedThreads, 0, g->stream>>>(
            (const float* const*)(g->dptr + 6 * g->cur), g->code, g->raw, g->d.nr, g->d.nz, a, g->partial);
    else
        k_rz_energy<double><<<kRedBlocks, kRedThreads, 0, g->stream>>>(
            (const double* const*)(g->dptr + 6 * g->cur), g->code, g->raw, g->d.nr, g->d.nz, a, g->partial);
    RZCHK(hipGetLastError());
    k_rz_finish<<<1, kRedThreads, 0, g->stream>>>(g->partial, kRedBlocks, g->scal);
    RZCHK(hipGetLastError());
    RZCHK(hipMemcpyAsync(W, g->scal, sizeof(double), hipMemcpyDeviceToHost, g->stream));
    RZCHK(hipStreamSynchronize(g->stream));
    if (n) *n = g->n;
    return isfinite(*W) ? TETE_OK : TETE_ERR_NONFINITE;
}

tete_status tete_rz_set_tuning(tete_rz* g, int32_t kernel, int32_t chunk_rows, int32_t prefetch, int32_t order)
{
    if (!g || (kernel != TETE_KERNEL_AUTO && kernel != TETE_KERNEL_FUSED && kernel != TETE_KERNEL_FUSED2) ||
        chunk_rows < 0 || (chunk_rows > 0 && (chunk_rows < 8 || chunk_rows > 4096)) || prefetch < 0 ||
        prefetch > 4 || order < 0 || order > 2)
        return TETE_ERR_ARG;
    g->kernel = kernel;
    g->chunk_rows = chunk_rows;
    g->prefetch = prefetch;
    g->order = order;
    return TETE_OK;
}

tete_status tete_rz_set_timing(tete_rz* g, int64_t max_launches)
{
    if (!g || max_launches < 0 || max_launches > (1 << 20)) return TETE_ERR_ARG;
    Guard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    RZCHK(hipStreamSynchronize(g->stream));
    if (g->ev) {
        for (int64_t i = 0; i < 2 * g->ev_cap; ++i) (void)hipEventDestroy(g->ev[i]);
        free(g->ev);
        g->ev = nullptr;
    }
    free(g->ev_nst);
    g->ev_nst = nullptr;
    g->ev_cap = g->ev_used = 0;
    g->timing = 0;
    if (max_launches == 0) return TETE_OK;
    g->ev = (hipEvent_t*)calloc((size_t)(2 * max_launches), sizeof(hipEvent_t));
    g->ev_nst = (unsigned char*)calloc((size_t)max_launches, 1);
    if (!g->ev || !g->ev_nst) {
        free(g->ev);
        free(g->ev_nst);
        g->ev = nullptr;
        g->ev_nst = nullptr;
        return TETE_ERR_NOMEM;
    }
    for (int64_t i = 0; i < 2 * max_launches; ++i) {
        if (hipEventCreate(&g->ev[i]) != hipSuccess) {
            for (int64_t t = 0; t < i; ++t) (void)hipEventDestroy(g->ev[t]);
            free(g->ev);
            free(g->ev_nst);
            g->ev = nullptr;
            g->ev_nst = nullptr;
            return TETE_ERR_DEVICE;
        }
    }
    g->ev_cap = max_launches;
    g->timing = 1;
    return TETE_OK;
}

tete_status tete_rz_timing(tete_rz* g, double* ms, int64_t* launches, int64_t* steps)
{
    if (!g || !ms || !launches || !steps) return TETE_ERR_ARG;
    Guard dg(g->device);
    if (!dg.ok) return TETE_ERR_DEVICE;
    RZCHK(hipStreamSynchronize(g->stream));
    double sum = 0.0;
    int64_t ns = 0;
    for (int64_t i = 0; i < g->ev_used; ++i) {
        float t = 0.0f;
        RZCHK(hipEventElapsedTime(&t, g->ev[2 * i], g->ev[2 * i + 1]));
        sum += t;
        ns += g->ev_nst[i];
    }
    *ms = sum;
    *launches = g->ev_used;
    *steps = ns;
    return TETE_OK;
}

}  // extern "C"
