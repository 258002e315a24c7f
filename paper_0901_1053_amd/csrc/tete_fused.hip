// Fused explicit TE/TM step (scheme (23), the ten sub-updates of Sec. 4.2) in
// one kernel, for vacuum cells with staircase PEC codes.
//
// Work decomposition.  A workgroup owns a tile of TY rows (j) by 62 entries
// (k) of the grid and marches along x through a chunk of planes.  Each wave is
// one j-row of 64 consecutive k (lanes), the tile plus a halo of one k below
// and one above; the workgroup holds TY + 4 rows, the tile plus a halo of two
// rows below and two above.  Along k, neighbours come from lane shuffles;
// along j, from LDS; along x, from registers, because the march visits the
// planes in order.  Every value of the step is therefore computed in
// registers and each field entry is read once from HBM and written once.
//
// The ten sub-updates form a pipeline over the planes.  With old data of plane
// p loaded at iteration p, the sub-updates run at plane lags
//   S1 (h_x^n)          p        S2 (h_y^n)        p-1    S3 (e_z^{n+1/2}) p-1
//   S4 (h_x^{n+1/2})    p-2      S5 (h_y^{n+1/2})  p-2
//   S6 (e_x^{n+1/2})    p-2      S7 (e_y^{n+1/2})  p-2    S8 (h_z^{n+1})   p-3
//   S9 (e_x^{n+1})      p-4      S10 (e_y^{n+1})   p-3
// chosen so that every j-neighbour a sub-update needs was produced in an
// earlier iteration (or loaded in this one): one LDS write phase and a single
// barrier per plane suffice, with the LDS double-buffered by plane parity.
// The halo rows, halo lanes and the first planes of a chunk compute values
// that are never stored; only the tile's own entries are written.

#include <algorithm>
#include <vector>

#include "tete_dev.h"

namespace tete {
namespace {

constexpr int KT = 62;   // k entries owned per workgroup (64 lanes minus two halo lanes)

// LDS of one workgroup: six double-buffered j-exchange planes of TYH + 2 rows.
template <typename R, int TYH>
struct Lds {
    R sEZ[2][TYH + 2][64];
    R sHXN[2][TYH + 2][64];
    R sEZH[2][TYH + 2][64];
    R sHZ[2][TYH + 2][64];
    R sEXH[2][TYH + 2][64];
    R sHZN[2][TYH + 2][64];
};

// Per-entry materials (kappa_x, kappa_y, kappa_z, mu_x, mu_y, mu_z arrays,
// zero on PEC edges and outside each component's range) for the MAT instance.
template <typename R>
struct MatA {
    const R* m[6];
};

// One tile (ty, tz) and x-chunk cx of one step of the grid described by A.
// Every thread of the workgroup must call it (it contains barriers).  MAT:
// the coefficients come from the per-entry arrays of MA, loaded with the
// fields of each plane and carried to the lags where the sub-updates use them
// (kappa_z to p-1, mu_x to p-2, mu_y to p-2, kappa_y to p-3, mu_z to p-3,
// kappa_x to p-4), instead of the vacuum scalars and the PEC codes.
template <typename R, int TYH, int PD, bool MAT = false>
__device__ __forceinline__ void fused_tile(const FArgs<R>& A, const int ty, const int tz, const int cx,
                                           Lds<R, TYH>& L, const MatA<R>& MA = MatA<R>{})
{
    constexpr int TY = TYH - 4;
    auto& sEZ = L.sEZ;
    auto& sHXN = L.sHXN;
    auto& sEZH = L.sEZH;
    auto& sHZ = L.sHZ;
    auto& sEXH = L.sEXH;
    auto& sHZN = L.sHZN;
    const Geo g = A.g;

    const int kl = threadIdx.x & 63;
    const int jl = threadIdx.x >> 6;
    const int j = ty * TY - 2 + jl;
    const int k = tz * KT - 1 + kl;
    const bool jin = (unsigned)j <= (unsigned)g.ny;
    const bool kin = (unsigned)k <= (unsigned)g.nz;
    const bool node = jin && kin;
    const bool owned = node && jl >= 2 && jl < 2 + TY && kl >= 1 && kl <= KT;
    const int roff = k + j * g.sz;

    // index-range masks of the h components (x part applied per plane)
    const bool hx_jk = node && j < g.ny && k < g.nz;
    const bool hy_k = node && k < g.nz;
    const bool hz_j = node && j < g.ny;

    const int xs = cx * A.xchunk;
    const int xe = min(xs + A.xchunk, g.nx + 1);
    const int xload_end = min(xe + 1, g.nx);    // last plane whose old data is needed

    const R a = A.a, a2 = A.a + A.a;
    const bool src_row = A.src.on && j == A.src.j0;

    // carried pipeline state (see the lag table above)
    R EXm1 = 0, EXm2 = 0, pzEXm2 = 0;
    R EYm1 = 0, EYm2 = 0, pzEYm1 = 0, pzEYm2 = 0;
    R EZm1 = 0, HYm1 = 0;
    R HZm1 = 0, HZm2 = 0, HZm3 = 0;
    uint32_t cm1 = 7, cm2 = 7, cm3 = 7, cm4 = 7;   // PEC codes of planes p-1..p-4
    R hxn_m1 = 0, hxn_m2 = 0, hyn_m2 = 0, ezh_m2 = 0;
    R pztHX_m3 = 0, pztHY_m3 = 0, pztHY_m4 = 0;
    R exh_m3 = 0, exh_m4 = 0, eyh_m3 = 0, hzn_m4 = 0;

    // Loads and stores go through buffer resources built once per workgroup in
    // scalar registers, each covering the planes of the chunk (loads: from
    // plane pb = max(0, xs - 2) to xload_end; stores: xs .. xe-1).  The byte
    // offset of an entry is its in-plane offset plus the plane's offset from
    // the first covered plane; a plane outside the covered range wraps to an
    // offset past the end, and lanes outside the grid use an offset past the
    // end, so out-of-range loads return 0 and such stores are dropped.  The
    // range check needs every covered range below 2^31 bytes (the host limits
    // the chunk length accordingly).
    constexpr uint32_t RB = sizeof(R);
    constexpr uint32_t OOB = 0x80000000u;
    const uint32_t plane_bytes = (uint32_t)g.sp * RB;
    const int pb = max(0, xs - 2);
    const int nload = xload_end >= pb ? xload_end - pb + 1 : 0;
    auto mk = [](const void* base, uint32_t bytes) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
    };
    const int64_t ld0 = (int64_t)pb * g.sp;
    const auto rEX = mk(A.ex + ld0, nload * plane_bytes), rEY = mk(A.ey + ld0, nload * plane_bytes),
               rEZ = mk(A.ez + ld0, nload * plane_bytes), rHX = mk(A.hx + ld0, nload * plane_bytes),
               rHY = mk(A.hy + ld0, nload * plane_bytes), rHZ = mk(A.hz + ld0, nload * plane_bytes);
    // PEC codes (one byte per entry) are read as the aligned dword holding the
    // lane's byte: a sub-dword load would be packed with other bytes into one
    // register, which needs the load complete at once and defeats the prefetch.
    const auto rC = mk(A.code, (uint32_t)std::min<int64_t>((int64_t)g.np + 4, 0x7fffffff));
    const int64_t st0 = (int64_t)xs * g.sp;
    const uint32_t nstb = (uint32_t)(xe - xs) * plane_bytes;
    const auto sEX = mk(A.ex1 + st0, nstb), sEY = mk(A.ey1 + st0, nstb), sEZ1 = mk(A.ez1 + st0, nstb),
               sHX = mk(A.hx1 + st0, nstb), sHY = mk(A.hy1 + st0, nstb), sHZ1 = mk(A.hz1 + st0, nstb);
    const uint32_t in_ld = (uint32_t)roff * RB;
    const uint32_t cfix = node ? 0u : 7u;              // outside the grid: PEC
    // material arrays over the same planes as the fields (MAT only)
    __amdgpu_buffer_rsrc_t rM[6];
    if constexpr (MAT) {
#pragma unroll
        for (int c = 0; c < 6; ++c) rM[c] = mk(MA.m[c] + ld0, nload * plane_bytes);
    }

    auto load_plane = [&](int i, R& vex, R& vey, R& vez, R& vhx, R& vhy, R& vhz, uint32_t& vc) {
        const uint32_t po = (uint32_t)(i - pb);
        const uint32_t off = node ? in_ld + po * plane_bytes : OOB;
        vex = bload<R>(rEX, off);
        vey = bload<R>(rEY, off);
        vez = bload<R>(rEZ, off);
        vhx = bload<R>(rHX, off);
        vhy = bload<R>(rHY, off);
        vhz = bload<R>(rHZ, off);
        const uint32_t offc = node ? ((uint32_t)(roff + i * g.sp) & ~3u) : OOB;
        vc = __builtin_amdgcn_raw_buffer_load_b32(rC, offc, 0, 0);   // byte extracted when used
    };

    // Prefetch: the old data of planes p+1 .. p+PD are in flight while plane p
    // is processed.  The PD+1 plane buffers are used round-robin by a loop
    // unrolled PD+1 times, so a buffer that a load is writing is never copied
    // (a copy would have to wait for that load).
    struct PR {
        R ex, ey, ez, hx, hy, hz;
        uint32_t c;
        R m[MAT ? 6 : 1];
    };
    auto load_mat = [&](int i, PR& d) {
        if constexpr (MAT) {
            const uint32_t off = node ? in_ld + (uint32_t)(i - pb) * plane_bytes : OOB;
#pragma unroll
            for (int c = 0; c < 6; ++c) d.m[c] = bload<R>(rM[c], off);
        }
    };
    // carried coefficients of the MAT instance (index: planes behind p)
    R KXc[5] = {}, KYc[4] = {}, KZc[2] = {}, MXc[3] = {}, MYc[3] = {}, MZc[4] = {};
    PR buf[PD + 1];
#pragma unroll
    for (int d = 0; d < PD; ++d) {
        load_plane(xs - 2 + d, buf[d].ex, buf[d].ey, buf[d].ez, buf[d].hx, buf[d].hy, buf[d].hz, buf[d].c);
        load_mat(xs - 2 + d, buf[d]);
    }

    const int pend = xe + 3;
    auto body = [&](const int p, const PR& cur, PR& nxt) {
        load_plane(p + PD, nxt.ex, nxt.ey, nxt.ez, nxt.hx, nxt.hy, nxt.hz, nxt.c);
        load_mat(p + PD, nxt);
        const R EX0 = cur.ex, EY0 = cur.ey, EZ0 = cur.ez, HX0 = cur.hx, HY0 = cur.hy, HZ0 = cur.hz;
        if constexpr (MAT) {
            KXc[0] = cur.m[0]; KYc[0] = cur.m[1]; KZc[0] = cur.m[2];
            MXc[0] = cur.m[3]; MYc[0] = cur.m[4]; MZc[0] = cur.m[5];
        }
        // outside the grid, or a plane without old data: PEC on all edges
        const uint32_t c0 = ((cur.c >> (((uint32_t)(roff + p * g.sp) & 3u) * 8u)) & 7u) | cfix |
                            ((p >= pb && p <= xload_end) ? 0u : 7u);

        // j-exchange through LDS (row r of the tile is LDS row r+1).  Rows 0 and
        // TYH+1 are never written: what they hold reaches only rows 0, 1,
        // TYH-2 and TYH-1 of the tile, which are never stored.
        const int s = p & 1;
        sEZ[s][jl + 1][kl] = EZ0;
        sHXN[s][jl + 1][kl] = hxn_m1;
        sEZH[s][jl + 1][kl] = ezh_m2;
        sHZ[s][jl + 1][kl] = HZm2;
        sEXH[s][jl + 1][kl] = exh_m3;
        sHZN[s][jl + 1][kl] = hzn_m4;
        __syncthreads();
        const R EZ0_jp = sEZ[s][jl + 2][kl];
        const R hxn_m1_jm = sHXN[s][jl][kl];
        const R ezh_m2_jp = sEZH[s][jl + 2][kl];
        const R HZm2_jm = sHZ[s][jl][kl];
        const R exh_m3_jp = sEXH[s][jl + 2][kl];
        const R hzn_m4_jm = sHZN[s][jl][kl];

        // planes handled in this iteration and their x-range masks
        const int q0 = p, q1 = p - 1, q2 = p - 2, q3 = p - 3, q4 = p - 4;
        auto xin = [&](int q) { return (unsigned)q <= (unsigned)g.nx; };
        auto xlt = [&](int q) { return q >= 0 && q < g.nx; };
        R mx0, mx2, my1, my2, mz3, kz1, ky2, kx2, ky3, kx4;
        if constexpr (MAT) {
            mx0 = MXc[0]; mx2 = MXc[2]; my1 = MYc[1]; my2 = MYc[2]; mz3 = MZc[3];
            kz1 = KZc[1]; ky2 = KYc[2]; kx2 = KXc[2]; ky3 = KYc[3]; kx4 = KXc[4];
        } else {
            mx0 = (hx_jk && xin(q0)) ? A.mx : R(0);
            mx2 = (hx_jk && xin(q2)) ? A.mx : R(0);
            my1 = (hy_k && xlt(q1)) ? A.my : R(0);
            my2 = (hy_k && xlt(q2)) ? A.my : R(0);
            mz3 = (hz_j && xlt(q3)) ? A.mz : R(0);
            kz1 = (cm1 & 4u) ? R(0) : A.kz;
            ky2 = (cm2 & 2u) ? R(0) : A.ky;
            kx2 = (cm2 & 1u) ? R(0) : A.kx;
            ky3 = (cm3 & 2u) ? R(0) : A.ky;
            kx4 = (cm4 & 1u) ? R(0) : A.kx;
        }

        // S1 at q0: h_x^n = h_x^{n-1/2} + a mu_x [P_z e_y^n - P_y e_z^{n-1/2}]
        const R pzEY0 = lane_next(EY0) - EY0;
        const R hxn0 = HX0 + a * mx0 * (pzEY0 - (EZ0_jp - EZ0));
        // S2 at q1: h_y^n = h_y^{n-1/2} + a mu_y [-P_z e_x^n + P_x e_z^{n-1/2}]
        const R pzEXm1 = lane_next(EXm1) - EXm1;
        const R hyn_m1 = HYm1 + a * my1 * (-pzEXm1 + (EZ0 - EZm1));
        // S3 at q1: e_z^{n+1/2} = e_z^{n-1/2} + 2a kappa_z [P_y^T h_x^n - P_x^T h_y^n - j_z^n]
        R ezh_m1 = EZm1 + a2 * kz1 * ((hxn_m1_jm - hxn_m1) - (hyn_m2 - hyn_m1));
        if (src_row && q1 == A.src.i0 && kin && k < g.nz) {
            const int64_t m = (int64_t)k - A.src.n + A.src.M;   // cell m crosses edge k in step n
            if (m >= -A.src.M && m <= A.src.M) {
                // the current term is rounded on its own (no fused multiply-add
                // with the subtraction), as in the two-step kernel
#pragma clang fp contract(off)
                ezh_m1 -= (R)((double)kz1 * A.src.lam[m + A.src.M]);
            }
            if (owned && q1 >= xs && q1 < xe && k < A.src.kend) {
                const int64_t js = A.src.n - k - A.src.M;      // wake sample of edge k
                if (js >= A.src.jmin && js < (int64_t)A.src.jmin + A.src.nw)
                    A.src.wacc[js - A.src.jmin] += -0.5 * ((double)EZm1 + (double)ezh_m1);
            }
        }
        // S4 at q2: h_x^{n+1/2} = h_x^n + a mu_x [P_z e_y^n - P_y e_z^{n+1/2}]
        const R hxh_m2 = hxn_m2 + a * mx2 * (pzEYm2 - (ezh_m2_jp - ezh_m2));
        // S5 at q2: h_y^{n+1/2} = h_y^n + a mu_y [-P_z e_x^n + P_x e_z^{n+1/2}]
        const R hyh_m2 = hyn_m2 + a * my2 * (-pzEXm2 + (ezh_m1 - ezh_m2));
        // S7 at q2: e_y^{n+1/2} = e_y^n + a kappa_y [-P_z^T h_x^{n+1/2} + P_x^T h_z^n]
        const R pztHX_m2 = lane_prev(hxh_m2) - hxh_m2;
        const R eyh_m2 = EYm2 + a * ky2 * (-pztHX_m2 + (HZm3 - HZm2));
        // S6 at q2: e_x^{n+1/2} = e_x^n + a kappa_x [P_z^T h_y^{n+1/2} - P_y^T h_z^n]
        const R pztHY_m2 = lane_prev(hyh_m2) - hyh_m2;
        const R exh_m2 = EXm2 + a * kx2 * (pztHY_m2 - (HZm2_jm - HZm2));
        // S8 at q3: h_z^{n+1} = h_z^n + 2a mu_z [P_y e_x^{n+1/2} - P_x e_y^{n+1/2}]
        const R hzn_m3 = HZm3 + a2 * mz3 * ((exh_m3_jp - exh_m3) - (eyh_m2 - eyh_m3));
        // S9 at q4: e_x^{n+1} = e_x^{n+1/2} + a kappa_x [P_z^T h_y^{n+1/2} - P_y^T h_z^{n+1}]
        const R ex1_m4 = exh_m4 + a * kx4 * (pztHY_m4 - (hzn_m4_jm - hzn_m4));
        // S10 at q3: e_y^{n+1} = e_y^{n+1/2} + a kappa_y [-P_z^T h_x^{n+1/2} + P_x^T h_z^{n+1}]
        const R ey1_m3 = eyh_m3 + a * ky3 * (-pztHX_m3 + (hzn_m4 - hzn_m3));

        if (owned) {
            const uint32_t o1 = in_ld + (uint32_t)(q1 - xs) * plane_bytes;
            const uint32_t o2 = o1 - plane_bytes, o3 = o2 - plane_bytes, o4 = o3 - plane_bytes;
            bstore<R>(sEZ1, o1, ezh_m1);
            bstore<R>(sHX, o2, hxh_m2);
            bstore<R>(sHY, o2, hyh_m2);
            bstore<R>(sHZ1, o3, hzn_m3);
            bstore<R>(sEY, o3, ey1_m3);
            bstore<R>(sEX, o4, ex1_m4);
        }

        // rotate the pipeline registers by one plane
        EXm2 = EXm1; EXm1 = EX0; pzEXm2 = pzEXm1;
        EYm2 = EYm1; EYm1 = EY0; pzEYm2 = pzEYm1; pzEYm1 = pzEY0;
        EZm1 = EZ0; HYm1 = HY0;
        HZm3 = HZm2; HZm2 = HZm1; HZm1 = HZ0;
        cm4 = cm3; cm3 = cm2; cm2 = cm1; cm1 = c0;
        if constexpr (MAT) {
#pragma unroll
            for (int d = 4; d > 0; --d) KXc[d] = KXc[d - 1];
#pragma unroll
            for (int d = 3; d > 0; --d) { KYc[d] = KYc[d - 1]; MZc[d] = MZc[d - 1]; }
#pragma unroll
            for (int d = 2; d > 0; --d) { MXc[d] = MXc[d - 1]; MYc[d] = MYc[d - 1]; }
            KZc[1] = KZc[0];
        }
        hxn_m2 = hxn_m1; hxn_m1 = hxn0;
        hyn_m2 = hyn_m1;
        ezh_m2 = ezh_m1;
        pztHX_m3 = pztHX_m2;
        pztHY_m4 = pztHY_m3; pztHY_m3 = pztHY_m2;
        exh_m4 = exh_m3; exh_m3 = exh_m2;
        eyh_m3 = eyh_m2;
        hzn_m4 = hzn_m3;
    };

    // The trip count is rounded up to a multiple of PD+1 (no per-plane guard,
    // which would make the buffers loop phis that the back edge has to copy):
    // the extra planes lie past the chunk, where loads return 0, stores are
    // dropped and nothing is accumulated.
    for (int p = xs - 2; p <= pend; p += PD + 1) {
#pragma unroll
        for (int u = 0; u <= PD; ++u) body(p + u, buf[u], buf[(u + PD) % (PD + 1)]);
    }
}

// One step of one grid: one workgroup per (tile, x-chunk).
template <typename R, int TYH, int PD>
__global__ __launch_bounds__(64 * TYH) void k_fused(FArgs<R> A, const int* act)
{
    __shared__ Lds<R, TYH> L;
    int ty, tz, cx;
    if (act) {   // the active tiles only, as in the materials instance below
        const int t = act[xcd_remap(blockIdx.x, gridDim.x)];
        tz = t % A.nzt;
        ty = (t / A.nzt) % A.nyt;
        cx = t / (A.nzt * A.nyt);
    } else if (!tile_of(xcd_remap(blockIdx.x, A.nblk), A.order, A.nyt, A.nzt, ty, tz, cx)) {
        return;   // whole group
    }
    fused_tile<R, TYH, PD>(A, ty, tz, cx, L);
}

// The same step with per-entry materials.  act (or null): the tiles that are
// not static, (cx nyt + ty) nzt + tz in the launch's tile order
// (fused_static_tiles), one workgroup each, remapped over the XCDs.
template <typename R, int TYH, int PD>
__global__ __launch_bounds__(64 * TYH) void k_fused_mat(FArgs<R> A, MatA<R> MA, const int* act)
{
    __shared__ Lds<R, TYH> L;
    int ty, tz, cx;
    if (act) {
        const int t = act[xcd_remap(blockIdx.x, gridDim.x)];
        tz = t % A.nzt;
        ty = (t / A.nzt) % A.nyt;
        cx = t / (A.nzt * A.nyt);
    } else if (!tile_of(xcd_remap(blockIdx.x, A.nblk), A.order, A.nyt, A.nzt, ty, tz, cx)) {
        return;   // whole group
    }
    fused_tile<R, TYH, PD, true>(A, ty, tz, cx, L, MA);
}

// A tile of the materials step is static when every entry it loads (rows
// ty TY - 2 .., TYH of them, lanes tz KT - 1 .., 64 of them, planes
// max(0, xs-2) .. min(xe+1, nx)) has kappa zero on its three e edges (PEC, or
// outside the component's range): e stays zero and h constant there, and the
// step leaves every entry the tile owns unchanged.  One workgroup per tile.
// kx null: the vacuum step, static where the PEC code of every entry is 7
// (three e edges PEC or absent), so that e stays zero and h constant.
template <typename R>
__global__ __launch_bounds__(256) void k_static_mat(const R* kx, const R* ky, const R* kz, const uint8_t* code, Geo g,
                                                    int TYH, int TY, int xchunk, int nyt, int nzt, uint8_t* out)
{
    __shared__ int active;
    const int t = blockIdx.x;
    const int tz = t % nzt, ty = (t / nzt) % nyt, cx = t / (nzt * nyt);
    if (threadIdx.x == 0) active = 0;
    __syncthreads();
    const int xs = cx * xchunk, xe = min(xs + xchunk, g.nx + 1);
    const int pb = max(0, xs - 2), pe = min(xe + 1, g.nx);
    const int64_t per_plane = (int64_t)TYH * 64;
    const int64_t n = (int64_t)(pe - pb + 1) * per_plane;
    bool found = false;
    for (int64_t e = threadIdx.x; e < n && !found; e += blockDim.x) {
        const int q = pb + (int)(e / per_plane);
        const int r = (int)(e % per_plane);
        const int j = ty * TY - 2 + r / 64, k = tz * KT - 1 + r % 64;
        if (j < 0 || j > g.ny || k < 0 || k > g.nz) continue;
        const int64_t i = (int64_t)q * g.sp + (int64_t)j * g.sz + k;
        if (kx ? (kx[i] != R(0) || ky[i] != R(0) || kz[i] != R(0)) : (code[i] & 7u) != 7u) found = true;
    }
    if (found) atomicOr(&active, 1);
    __syncthreads();
    if (threadIdx.x == 0) out[t] = active ? 0 : 1;
}

// One step of every active instance of a batch, by a persistent grid: work
// item w (instance, tile, x-chunk) is taken by workgroup w mod gridDim.x in
// round w / gridDim.x.  Within a round the items are remapped over the XCDs
// like the tiles of one grid, so that neighbouring tiles share an L2.  The
// instance's step index and the ping-pong parity come from the table, which
// the host may rewrite between launches (a captured graph stays valid); this
// launch follows `flips` launches and `steps` steps of the current block.
template <typename R, int TYH, int PD>
__global__ __launch_bounds__(64 * TYH) void k_fused_batch(const BatchTable<R>* Tg, int flips, int steps)
{
    __shared__ Lds<R, TYH> L;
    // The table is read-only during the launch: reading it through the
    // constant address space makes its (uniform) fields scalar loads into
    // scalar registers instead of vector loads that would occupy VGPRs.
    typedef const __attribute__((address_space(4))) BatchTable<R>* CTable;
    typedef const __attribute__((address_space(4))) uint32_t* CWords;
    const CTable T = (CTable)Tg;
    const int total = T->total;
    const int ninst = T->ninst;
    const int parity = (T->phase + flips) & 1;
    for (int round = 0; round * (int)gridDim.x < total; ++round) {
        const int base = round * (int)gridDim.x;
        const int span = min((int)gridDim.x, total - base);
        if ((int)blockIdx.x >= span) break;
        // work item and instance are uniform over the workgroup: keep them (and
        // the instance's arguments) in scalar registers
        const int w = __builtin_amdgcn_readfirstlane(base + xcd_remap(blockIdx.x, span));
        int lo = 0, hi = ninst - 1;               // last instance whose first item is <= w
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (T->offset[mid] <= w) lo = mid;
            else hi = mid - 1;
        }
        const int inst = __builtin_amdgcn_readfirstlane(lo);
        FArgs<R> A;
        {
            const CWords src = (CWords)&T->item[inst].a[parity];
            uint32_t* dst = (uint32_t*)&A;
#pragma unroll
            for (int i = 0; i < (int)(sizeof(FArgs<R>) / 4); ++i) dst[i] = src[i];
        }
        A.src.n = T->step[inst] + steps;
        int ty, tz, cx;
        if (tile_of(w - T->offset[inst], A.order, A.nyt, A.nzt, ty, tz, cx)) fused_tile<R, TYH, PD>(A, ty, tz, cx, L);
        __syncthreads();   // the LDS is reused by the next item
    }
}

// After a block: advance every instance's step index, and the phase by the
// number of launches (each launch swaps the ping-pong sets once).
template <typename R>
__global__ void k_batch_advance(BatchTable<R>* T, int steps, int flips)
{
    const int i = threadIdx.x + blockIdx.x * blockDim.x;
    if (i < T->ninst) T->step[i] += steps;
    if (i == 0) T->phase = (T->phase + flips) & 1;
}

template <typename R, int TYH, int PD>
hipError_t launch_fused_t(const FArgs<R>& A, const int* act, int nact, hipStream_t s)
{
    if (!act) k_fused<R, TYH, PD><<<A.nblk, 64 * TYH, 0, s>>>(A, nullptr);
    else if (nact > 0) k_fused<R, TYH, PD><<<nact, 64 * TYH, 0, s>>>(A, act);
    return hipGetLastError();
}

}  // namespace

int fused_default_rows(int real_bytes) { return real_bytes == 8 ? 12 : 16; }   // FP64 at 16 rows spills

template <typename R>
bool fused_setup(FArgs<R>& A, int rows, int xchunk, int order)
{
    if (rows == 0) rows = fused_default_rows(sizeof(R));
    if (rows != 12 && rows != 16) return false;
    const int TY = rows - 4;
    A.nyt = (A.g.ny + 1 + TY - 1) / TY;
    A.nzt = (A.g.nz + 1 + KT - 1) / KT;
    const int nplanes = A.g.nx + 1;
    int xc = xchunk;
    if (xc <= 0) {
        // enough workgroups to fill the chip several times over
        const int tiles = A.nyt * A.nzt;
        int chunks = (4096 + tiles - 1) / tiles;
        chunks = std::max(1, std::min(chunks, (nplanes + 31) / 32));
        xc = (nplanes + chunks - 1) / chunks;
    }
    // every buffer range must stay below 2^31 bytes: (xchunk + 4) planes
    const int64_t plane_bytes = (int64_t)A.g.sp * sizeof(R);
    const int64_t xmax = ((int64_t(1) << 31) - 1) / plane_bytes - 4;
    if (xmax < 1) return false;
    xc = (int)std::min<int64_t>(std::max(xc, 1), xmax);
    A.xchunk = xc;
    A.nxc = (nplanes + xc - 1) / xc;
    A.order = order != 0 ? order : default_order(A.nyt, A.nzt, A.nxc);
    A.nblk = launch_tiles(A.order, A.nyt, A.nzt, A.nxc);
    return true;
}

template <typename R>
FArgs<R> fused_args(Fields<R> o, Fields<R> nf, Mat<R> M, Geo g, R alpha, Src src)
{
    FArgs<R> A;
    A.ex = o.c[0]; A.ey = o.c[1]; A.ez = o.c[2]; A.hx = o.c[3]; A.hy = o.c[4]; A.hz = o.c[5];
    A.ex1 = nf.c[0]; A.ey1 = nf.c[1]; A.ez1 = nf.c[2]; A.hx1 = nf.c[3]; A.hy1 = nf.c[4]; A.hz1 = nf.c[5];
    A.code = M.code;
    A.cls = M.cls;
    A.ctab = M.ctab;
    A.g = g;
    A.a = alpha;
    A.kx = M.k[0]; A.ky = M.k[1]; A.kz = M.k[2];
    A.mx = M.m[0]; A.my = M.m[1]; A.mz = M.m[2];
    A.src = src;
    A.nyt = A.nzt = A.nxc = A.xchunk = A.nblk = A.order = 0;
    return A;
}

template <typename R>
hipError_t launch_batch_step(BatchTable<R>* T, int rows, int depth, int grid, int flips, int steps, hipStream_t s)
{
    if (rows == 0) rows = fused_default_rows(sizeof(R));
    const int threads = 64 * rows;
    if (rows == 12) {
        if (depth == 1) k_fused_batch<R, 12, 1><<<grid, threads, 0, s>>>(T, flips, steps);
        else if (depth == 3) k_fused_batch<R, 12, 3><<<grid, threads, 0, s>>>(T, flips, steps);
        else k_fused_batch<R, 12, 2><<<grid, threads, 0, s>>>(T, flips, steps);
    } else {
        if (depth == 1) k_fused_batch<R, 16, 1><<<grid, threads, 0, s>>>(T, flips, steps);
        else if (depth == 3) k_fused_batch<R, 16, 3><<<grid, threads, 0, s>>>(T, flips, steps);
        else k_fused_batch<R, 16, 2><<<grid, threads, 0, s>>>(T, flips, steps);
    }
    return hipGetLastError();
}

template <typename R>
hipError_t launch_batch_advance(BatchTable<R>* T, int steps, int flips, hipStream_t s)
{
    k_batch_advance<R><<<(TETE_MAX_BATCH + 255) / 256, 256, 0, s>>>(T, steps, flips);
    return hipGetLastError();
}

bool fused_fits(Geo g, int real_bytes)
{
    return (int64_t)g.sp * real_bytes * 5 < (int64_t(1) << 31);
}

int64_t fused_tile_cap(Geo g)
{
    // the smallest owned shape: 8 rows (12-row tiles) by 62 entries over tiles
    // of single planes
    return (int64_t)(g.nx + 1) * ((g.ny + 1 + 7) / 8) * ((g.nz + 1 + KT - 1) / KT);
}

template <typename R>
hipError_t fused_static_tiles(const R* const kap[3], const uint8_t* code, Geo g, int rows, int xchunk, int order,
                              uint8_t* tab, int* act, int64_t cap, int64_t* ntiles, int* nact, hipStream_t s)
{
    FArgs<R> A = fused_args<R>(Fields<R>{}, Fields<R>{}, Mat<R>{}, g, R(0), Src{});
    if (kap || rows == 0) rows = fused_default_rows(sizeof(R));   // the materials instance: default shape
    if (!fused_setup<R>(A, rows, xchunk, order)) return hipErrorInvalidValue;
    const int64_t nt = (int64_t)A.nyt * A.nzt * A.nxc;
    if (nt > cap || nt > 0x7fffffff) return hipErrorInvalidValue;
    if (!kap && !code) return hipErrorInvalidValue;
    k_static_mat<R><<<(int)nt, 256, 0, s>>>(kap ? kap[0] : nullptr, kap ? kap[1] : nullptr, kap ? kap[2] : nullptr,
                                            code, g, rows, rows - 4, A.xchunk, A.nyt, A.nzt, tab);
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

template <typename R>
hipError_t launch_step_fused(Fields<R> o, Fields<R> nf, Mat<R> M, Geo g, R alpha, Src src, int rows, int xchunk,
                             int depth, int order, hipStream_t s, hipEvent_t* ev, const int* act, int nact)
{
    FArgs<R> A = fused_args<R>(o, nf, M, g, alpha, src);
    const bool mat = M.arr[0] != nullptr;   // per-entry materials: one shape, one plane prefetched
    if (rows == 0 || mat) rows = fused_default_rows(sizeof(R));
    if (!fused_setup<R>(A, rows, xchunk, order)) return hipErrorInvalidValue;
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    if (mat) {
        MatA<R> MA;
        for (int c = 0; c < 6; ++c) {
            if (!M.arr[c]) return hipErrorInvalidValue;
            MA.m[c] = M.arr[c];
        }
        constexpr int TYH = sizeof(R) == 8 ? 12 : 16;
        // with a list of active tiles, one workgroup per entry (none: every
        // tile is static and the new set already holds the result)
        if (!act) k_fused_mat<R, TYH, 1><<<A.nblk, 64 * TYH, 0, s>>>(A, MA, nullptr);
        else if (nact > 0) k_fused_mat<R, TYH, 1><<<nact, 64 * TYH, 0, s>>>(A, MA, act);
        e = hipGetLastError();
    } else if (rows == 12) {
        if (depth == 1) e = launch_fused_t<R, 12, 1>(A, act, nact, s);
        else if (depth == 3) e = launch_fused_t<R, 12, 3>(A, act, nact, s);
        else e = launch_fused_t<R, 12, 2>(A, act, nact, s);
    } else {
        if (depth == 1) e = launch_fused_t<R, 16, 1>(A, act, nact, s);
        else if (depth == 3) e = launch_fused_t<R, 16, 3>(A, act, nact, s);
        else e = launch_fused_t<R, 16, 2>(A, act, nact, s);
    }
    if (e != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    return hipSuccess;
}

#define TETE_FUSED_INST(R)                                                                                     \
    template bool fused_setup<R>(FArgs<R>&, int, int, int);                                                    \
    template FArgs<R> fused_args<R>(Fields<R>, Fields<R>, Mat<R>, Geo, R, Src);                                 \
    template hipError_t launch_batch_step<R>(BatchTable<R>*, int, int, int, int, int, hipStream_t);            \
    template hipError_t launch_batch_advance<R>(BatchTable<R>*, int, int, hipStream_t);
TETE_FUSED_INST(float)
TETE_FUSED_INST(double)

template hipError_t launch_step_fused<float>(Fields<float>, Fields<float>, Mat<float>, Geo, float, Src, int, int,
                                             int, int, hipStream_t, hipEvent_t*, const int*, int);
template hipError_t launch_step_fused<double>(Fields<double>, Fields<double>, Mat<double>, Geo, double, Src, int,
                                              int, int, int, hipStream_t, hipEvent_t*, const int*, int);
template hipError_t fused_static_tiles<float>(const float* const[3], const uint8_t*, Geo, int, int, int, uint8_t*,
                                              int*, int64_t, int64_t*, int*, hipStream_t);
template hipError_t fused_static_tiles<double>(const double* const[3], const uint8_t*, Geo, int, int, int, uint8_t*,
                                               int*, int64_t, int64_t*, int*, hipStream_t);

}  // namespace tete
