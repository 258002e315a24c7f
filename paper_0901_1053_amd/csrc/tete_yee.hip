// Yee's E/M scheme (7) as a baseline on the same grid, layout and PEC codes:
//   e^{n+1/2} = e^{n-1/2} + dtau M_eps^-1 C^T h^n,   h^{n+1} = h^n - dtau M_mu^-1 C e^{n+1/2},
// stable in vacuum up to (8).  One fused kernel per step, built like the
// fused TE/TM step: a workgroup owns a tile of rows (j) by 62 entries (k) and
// marches along x; k-neighbours come from lane shifts, j-neighbours from LDS
// (double-buffered, one barrier per plane), x-neighbours from registers.
// Plane lags: with the old data of plane p loaded at iteration p, e^{n+1/2}
// is formed at plane p (it needs h^n at p and p-1) and h^{n+1} at plane p-1
// (it needs e^{n+1/2} at p-1 and p).  Halos: e^{n+1/2} needs h^n one row and
// one lane below, h^{n+1} needs e^{n+1/2} one row and one lane above, so a
// tile of TYH rows owns rows 1 .. TYH-2 and lanes 1 .. 62.

#include <algorithm>

#include "tete_dev.h"

namespace tete {
namespace {

constexpr int KTY = 62;   // k entries owned per workgroup

template <typename R, int TYH>
struct LdsY {
    R hx[2][TYH][64];    // h_x^n, h_z^n of the current plane (read one row below)
    R hz[2][TYH][64];
    R ez[2][TYH][64];    // e_z^{n+1/2}, e_x^{n+1/2} of the previous plane (read one row above)
    R ex[2][TYH][64];
};

template <typename R, int TYH, int PD>
__device__ __forceinline__ void yee_tile(const FArgs<R>& A, const int ty, const int tz, const int cx, LdsY<R, TYH>& L)
{
    constexpr int TY = TYH - 2;
    const Geo g = A.g;
    const int kl = threadIdx.x & 63;
    const int jl = threadIdx.x >> 6;
    const int j = ty * TY - 1 + jl;
    const int k = tz * KTY - 1 + kl;
    const bool jin = (unsigned)j <= (unsigned)g.ny;
    const bool kin = (unsigned)k <= (unsigned)g.nz;
    const bool node = jin && kin;
    const bool owned = node && jl >= 1 && jl <= TY && kl >= 1 && kl <= KTY;
    const int roff = k + j * g.sz;

    const bool hx_jk = node && j < g.ny && k < g.nz;
    const bool hy_k = node && k < g.nz;
    const bool hz_j = node && j < g.ny;

    const int xs = cx * A.xchunk;
    const int xe = min(xs + A.xchunk, g.nx + 1);
    const int xload_end = min(xe, g.nx);         // last plane whose old data is needed

    const R dt = A.a + A.a;                      // dtau
    const R dkx = dt * A.kx, dky = dt * A.ky, dkz = dt * A.kz;
    const R dmx = hx_jk ? dt * A.mx : R(0), dmy = hy_k ? dt * A.my : R(0), dmz = hz_j ? dt * A.mz : R(0);

    // buffer resources over the chunk's planes (loads: pb = max(0, xs - 1) ..
    // xload_end; stores: xs .. xe-1); out-of-range loads return 0 and
    // out-of-range stores are dropped (the host keeps (xchunk + 2) planes
    // below 2^31 bytes)
    constexpr uint32_t RB = sizeof(R);
    constexpr uint32_t OOB = 0x80000000u;
    const uint32_t plane_bytes = (uint32_t)g.sp * RB;
    const int pb = max(0, xs - 1);
    const int nload = xload_end >= pb ? xload_end - pb + 1 : 0;
    auto mk = [](const void* base, uint32_t bytes) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
    };
    const int64_t ld0 = (int64_t)pb * g.sp;
    const auto rEX = mk(A.ex + ld0, nload * plane_bytes), rEY = mk(A.ey + ld0, nload * plane_bytes),
               rEZ = mk(A.ez + ld0, nload * plane_bytes), rHX = mk(A.hx + ld0, nload * plane_bytes),
               rHY = mk(A.hy + ld0, nload * plane_bytes), rHZ = mk(A.hz + ld0, nload * plane_bytes);
    const auto rC = mk(A.code, (uint32_t)std::min<int64_t>((int64_t)g.np + 4, 0x7fffffff));
    const int64_t st0 = (int64_t)xs * g.sp;
    const uint32_t nstb = (uint32_t)(xe - xs) * plane_bytes;
    const auto sEX = mk(A.ex1 + st0, nstb), sEY = mk(A.ey1 + st0, nstb), sEZ = mk(A.ez1 + st0, nstb),
               sHX = mk(A.hx1 + st0, nstb), sHY = mk(A.hy1 + st0, nstb), sHZ = mk(A.hz1 + st0, nstb);
    const uint32_t in_ld = (uint32_t)roff * RB;
    const uint32_t cfix = node ? 0u : 7u;

    struct PR {
        R ex, ey, ez, hx, hy, hz;
        uint32_t c;
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
        const uint32_t offc = node ? ((uint32_t)(roff + i * g.sp) & ~3u) : OOB;
        d.c = __builtin_amdgcn_raw_buffer_load_b32(rC, offc, 0, 0);
    };

    // carried: h^n of plane p-1, e^{n+1/2} of plane p-1
    R HXm1 = 0, HYm1 = 0, HZm1 = 0, exm1 = 0, eym1 = 0, ezm1 = 0;
    auto xlt = [&](int q) { return q >= 0 && q < g.nx; };

    PR buf[PD + 1];
#pragma unroll
    for (int d = 0; d < PD; ++d) load_plane(xs - 1 + d, buf[d]);

    auto body = [&](const int p, const PR& cur, PR& nxt) {
        load_plane(p + PD, nxt);
        const uint32_t c0 = ((cur.c >> (((uint32_t)(roff + p * g.sp) & 3u) * 8u)) & 7u) | cfix |
                            ((p >= pb && p <= xload_end) ? 0u : 7u);
        const int s = p & 1;
        L.hx[s][jl][kl] = cur.hx;
        L.hz[s][jl][kl] = cur.hz;
        L.ez[s][jl][kl] = ezm1;
        L.ex[s][jl][kl] = exm1;
        __syncthreads();
        // rows outside the tile read a neighbour inside it: such values reach
        // only halo results
        const int jm = jl > 0 ? jl - 1 : 0, jp = jl < TYH - 1 ? jl + 1 : TYH - 1;
        const R HX_jm = L.hx[s][jm][kl], HZ_jm = L.hz[s][jm][kl];
        const R ezm1_jp = L.ez[s][jp][kl], exm1_jp = L.ex[s][jp][kl];

        // e^{n+1/2} at plane p (kappa zero on PEC edges)
        const R kx = (c0 & 1u) ? R(0) : dkx, ky = (c0 & 2u) ? R(0) : dky, kz = (c0 & 4u) ? R(0) : dkz;
        const R pzt_hy = lane_prev(cur.hy) - cur.hy, pzt_hx = lane_prev(cur.hx) - cur.hx;
        const R ex0 = cur.ex + kx * (pzt_hy - (HZ_jm - cur.hz));
        const R ey0 = cur.ey + ky * (-pzt_hx + (HZm1 - cur.hz));
        const R ez0 = cur.ez + kz * ((HX_jm - cur.hx) - (HYm1 - cur.hy));

        // h^{n+1} at plane p-1 (mu masked by the component's index range)
        const int q = p - 1;
        const R my = xlt(q) ? dmy : R(0), mz = xlt(q) ? dmz : R(0);
        const R pz_ey = lane_next(eym1) - eym1, pz_ex = lane_next(exm1) - exm1;
        const R hx1 = HXm1 + dmx * (pz_ey - (ezm1_jp - ezm1));
        const R hy1 = HYm1 + my * (-pz_ex + (ez0 - ezm1));
        const R hz1 = HZm1 + mz * ((exm1_jp - exm1) - (ey0 - eym1));

        if (owned) {
            const uint32_t o0 = in_ld + (uint32_t)(p - xs) * plane_bytes, o1 = o0 - plane_bytes;
            bstore<R>(sEX, o0, ex0);
            bstore<R>(sEY, o0, ey0);
            bstore<R>(sEZ, o0, ez0);
            bstore<R>(sHX, o1, hx1);
            bstore<R>(sHY, o1, hy1);
            bstore<R>(sHZ, o1, hz1);
        }
        HXm1 = cur.hx; HYm1 = cur.hy; HZm1 = cur.hz;
        exm1 = ex0; eym1 = ey0; ezm1 = ez0;
    };

    // planes xs-1 .. xe, the trip count rounded up to a multiple of PD+1
    for (int p = xs - 1; p <= xe; p += PD + 1) {
#pragma unroll
        for (int u = 0; u <= PD; ++u) body(p + u, buf[u], buf[(u + PD) % (PD + 1)]);
    }
}

template <typename R, int TYH, int PD>
__global__ __launch_bounds__(64 * TYH) void k_yee(FArgs<R> A)
{
    __shared__ LdsY<R, TYH> L;
    int ty, tz, cx;
    if (!tile_of(xcd_remap(blockIdx.x, A.nblk), A.order, A.nyt, A.nzt, ty, tz, cx)) return;   // whole group
    yee_tile<R, TYH, PD>(A, ty, tz, cx, L);
}

// Two steps of (7) per launch, temporally blocked as the TE/TM two-step
// kernel: stage A takes (e^{n-1/2}, h^n) to e^{n+1/2} at plane p and h^{n+1}
// at p-1, stage B takes stage A's results to e^{n+3/2} at p-1 and h^{n+2} at
// p-2; only stage B's results are stored.  Each stage exchanges its
// j-neighbours through its own double-buffered LDS planes, with a barrier
// before each stage.  Two steps lose two rows and two lanes at each edge, so
// a tile of TYH rows owns rows 2 .. TYH-3 and lanes 2 .. 61.  Every
// sub-update is the expression of the single step, so two steps here equal
// two single steps bitwise.
constexpr int KTY2 = 60;   // k entries owned per workgroup of the two-step kernel

template <typename R, int TYH>
struct LdsY2 {
    LdsY<R, TYH> a, b;
};

template <typename R, int TYH, int PD>
__device__ __forceinline__ void yee2_tile(const FArgs<R>& A, const int ty, const int tz, const int cx,
                                          LdsY2<R, TYH>& L)
{
    constexpr int TY = TYH - 4;
    const Geo g = A.g;
    const int kl = threadIdx.x & 63;
    const int jl = threadIdx.x >> 6;
    const int j = ty * TY - 2 + jl;
    const int k = tz * KTY2 - 2 + kl;
    const bool jin = (unsigned)j <= (unsigned)g.ny;
    const bool kin = (unsigned)k <= (unsigned)g.nz;
    const bool node = jin && kin;
    const bool owned = node && jl >= 2 && jl <= TYH - 3 && kl >= 2 && kl <= KTY2 + 1;
    const int roff = k + j * g.sz;

    const bool hx_jk = node && j < g.ny && k < g.nz;
    const bool hy_k = node && k < g.nz;
    const bool hz_j = node && j < g.ny;

    const int xs = cx * A.xchunk;
    const int xe = min(xs + A.xchunk, g.nx + 1);
    const int xload_end = min(xe + 1, g.nx);     // last plane whose old data is needed

    const R dt = A.a + A.a;                      // dtau
    const R dkx = dt * A.kx, dky = dt * A.ky, dkz = dt * A.kz;
    const R dmx = hx_jk ? dt * A.mx : R(0), dmy = hy_k ? dt * A.my : R(0), dmz = hz_j ? dt * A.mz : R(0);

    // loads: planes pb = max(0, xs - 2) .. xload_end; stores: xs .. xe-1;
    // out-of-range loads return 0 and out-of-range stores are dropped (the
    // host keeps (xchunk + 3) planes below 2^31 bytes)
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
    const auto rC = mk(A.code, (uint32_t)std::min<int64_t>((int64_t)g.np + 4, 0x7fffffff));
    const int64_t st0 = (int64_t)xs * g.sp;
    const uint32_t nstb = (uint32_t)(xe - xs) * plane_bytes;
    const auto sEX = mk(A.ex1 + st0, nstb), sEY = mk(A.ey1 + st0, nstb), sEZ = mk(A.ez1 + st0, nstb),
               sHX = mk(A.hx1 + st0, nstb), sHY = mk(A.hy1 + st0, nstb), sHZ = mk(A.hz1 + st0, nstb);
    const uint32_t in_ld = (uint32_t)roff * RB;
    const uint32_t cfix = node ? 0u : 7u;

    struct PR {
        R ex, ey, ez, hx, hy, hz;
        uint32_t c;
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
        const uint32_t offc = node ? ((uint32_t)(roff + i * g.sp) & ~3u) : OOB;
        d.c = __builtin_amdgcn_raw_buffer_load_b32(rC, offc, 0, 0);
    };

    // stage A carries h^n and e^{n+1/2} of plane p-1; stage B h^{n+1} and
    // e^{n+3/2} of plane p-2, and the PEC code of its plane p-1
    R HXm1 = 0, HYm1 = 0, HZm1 = 0, exm1 = 0, eym1 = 0, ezm1 = 0;
    R BHXm1 = 0, BHYm1 = 0, BHZm1 = 0, bexm1 = 0, beym1 = 0, bezm1 = 0;
    uint32_t cprev = 7u;
    auto xlt = [&](int q) { return q >= 0 && q < g.nx; };
    const int jm = jl > 0 ? jl - 1 : 0, jp = jl < TYH - 1 ? jl + 1 : TYH - 1;

    PR buf[PD + 1];
#pragma unroll
    for (int d = 0; d < PD; ++d) load_plane(xs - 2 + d, buf[d]);

    auto body = [&](const int p, const PR& cur, PR& nxt) {
        load_plane(p + PD, nxt);
        const uint32_t c0 = ((cur.c >> (((uint32_t)(roff + p * g.sp) & 3u) * 8u)) & 7u) | cfix |
                            ((p >= pb && p <= xload_end) ? 0u : 7u);
        const int s = p & 1;

        // stage A: e^{n+1/2} at p, h^{n+1} at p-1
        L.a.hx[s][jl][kl] = cur.hx;
        L.a.hz[s][jl][kl] = cur.hz;
        L.a.ez[s][jl][kl] = ezm1;
        L.a.ex[s][jl][kl] = exm1;
        __syncthreads();
        const R HX_jm = L.a.hx[s][jm][kl], HZ_jm = L.a.hz[s][jm][kl];
        const R ezm1_jp = L.a.ez[s][jp][kl], exm1_jp = L.a.ex[s][jp][kl];
        const R kx = (c0 & 1u) ? R(0) : dkx, ky = (c0 & 2u) ? R(0) : dky, kz = (c0 & 4u) ? R(0) : dkz;
        const R pzt_hy = lane_prev(cur.hy) - cur.hy, pzt_hx = lane_prev(cur.hx) - cur.hx;
        const R ex0 = cur.ex + kx * (pzt_hy - (HZ_jm - cur.hz));
        const R ey0 = cur.ey + ky * (-pzt_hx + (HZm1 - cur.hz));
        const R ez0 = cur.ez + kz * ((HX_jm - cur.hx) - (HYm1 - cur.hy));
        const int q = p - 1;
        const R my = xlt(q) ? dmy : R(0), mz = xlt(q) ? dmz : R(0);
        const R pz_ey = lane_next(eym1) - eym1, pz_ex = lane_next(exm1) - exm1;
        const R hx1 = HXm1 + dmx * (pz_ey - (ezm1_jp - ezm1));
        const R hy1 = HYm1 + my * (-pz_ex + (ez0 - ezm1));
        const R hz1 = HZm1 + mz * ((exm1_jp - exm1) - (ey0 - eym1));

        // stage B on plane q = p-1, from h^{n+1}(q) and e^{n+1/2}(q): e^{n+3/2}
        // at q, h^{n+2} at q-1
        L.b.hx[s][jl][kl] = hx1;
        L.b.hz[s][jl][kl] = hz1;
        L.b.ez[s][jl][kl] = bezm1;
        L.b.ex[s][jl][kl] = bexm1;
        __syncthreads();
        const R BHX_jm = L.b.hx[s][jm][kl], BHZ_jm = L.b.hz[s][jm][kl];
        const R bezm1_jp = L.b.ez[s][jp][kl], bexm1_jp = L.b.ex[s][jp][kl];
        const R bkx = (cprev & 1u) ? R(0) : dkx, bky = (cprev & 2u) ? R(0) : dky, bkz = (cprev & 4u) ? R(0) : dkz;
        const R bpzt_hy = lane_prev(hy1) - hy1, bpzt_hx = lane_prev(hx1) - hx1;
        const R bex0 = exm1 + bkx * (bpzt_hy - (BHZ_jm - hz1));
        const R bey0 = eym1 + bky * (-bpzt_hx + (BHZm1 - hz1));
        const R bez0 = ezm1 + bkz * ((BHX_jm - hx1) - (BHYm1 - hy1));
        const int qb = p - 2;
        const R bmy = xlt(qb) ? dmy : R(0), bmz = xlt(qb) ? dmz : R(0);
        const R bpz_ey = lane_next(beym1) - beym1, bpz_ex = lane_next(bexm1) - bexm1;
        const R bhx1 = BHXm1 + dmx * (bpz_ey - (bezm1_jp - bezm1));
        const R bhy1 = BHYm1 + bmy * (-bpz_ex + (bez0 - bezm1));
        const R bhz1 = BHZm1 + bmz * ((bexm1_jp - bexm1) - (bey0 - beym1));

        if (owned) {
            const uint32_t o1 = in_ld + (uint32_t)(p - 1 - xs) * plane_bytes, o2 = o1 - plane_bytes;
            bstore<R>(sEX, o1, bex0);
            bstore<R>(sEY, o1, bey0);
            bstore<R>(sEZ, o1, bez0);
            bstore<R>(sHX, o2, bhx1);
            bstore<R>(sHY, o2, bhy1);
            bstore<R>(sHZ, o2, bhz1);
        }
        BHXm1 = hx1; BHYm1 = hy1; BHZm1 = hz1;
        bexm1 = bex0; beym1 = bey0; bezm1 = bez0;
        HXm1 = cur.hx; HYm1 = cur.hy; HZm1 = cur.hz;
        exm1 = ex0; eym1 = ey0; ezm1 = ez0;
        cprev = c0;
    };

    // planes xs-2 .. xe+1, the trip count rounded up to a multiple of PD+1
    for (int p = xs - 2; p <= xe + 1; p += PD + 1) {
#pragma unroll
        for (int u = 0; u <= PD; ++u) body(p + u, buf[u], buf[(u + PD) % (PD + 1)]);
    }
}

template <typename R, int TYH, int PD>
__global__ __launch_bounds__(64 * TYH) void k_yee2(FArgs<R> A)
{
    __shared__ LdsY2<R, TYH> L;
    int ty, tz, cx;
    if (!tile_of(xcd_remap(blockIdx.x, A.nblk), A.order, A.nyt, A.nzt, ty, tz, cx)) return;   // whole group
    yee2_tile<R, TYH, PD>(A, ty, tz, cx, L);
}

constexpr int ROWSY = 16;

}  // namespace

template <typename R>
bool yee_setup(FArgs<R>& A, int xchunk, int order)
{
    constexpr int TY = ROWSY - 2;
    A.nyt = (A.g.ny + 1 + TY - 1) / TY;
    A.nzt = (A.g.nz + 1 + KTY - 1) / KTY;
    const int nplanes = A.g.nx + 1;
    // every buffer range must stay below 2^31 bytes: (xchunk + 2) planes
    const int64_t plane_bytes = (int64_t)A.g.sp * sizeof(R);
    const int64_t xmax = ((int64_t(1) << 31) - 1) / plane_bytes - 2;
    if (xmax < 1) return false;
    int xc = xchunk;
    if (xc <= 0) {
        // as in the fused single step: enough workgroups to fill the chip
        // several times over, chunks of at least 32 planes
        const int tiles = A.nyt * A.nzt;
        int chunks = (4096 + tiles - 1) / tiles;
        chunks = std::max(1, std::min(chunks, (nplanes + 31) / 32));
        xc = (nplanes + chunks - 1) / chunks;
    }
    xc = (int)std::min<int64_t>(std::max(xc, 1), xmax);
    A.xchunk = xc;
    A.nxc = (nplanes + xc - 1) / xc;
    A.order = order != 0 ? order : default_order(A.nyt, A.nzt, A.nxc);
    A.nblk = launch_tiles(A.order, A.nyt, A.nzt, A.nxc);
    return true;
}

bool yee_fits(Geo g, int real_bytes)
{
    return (int64_t)g.sp * real_bytes * 3 < (int64_t(1) << 31);
}

template <typename R>
hipError_t launch_step_yee(Fields<R> o, Fields<R> nf, Mat<R> M, Geo g, R alpha, int xchunk, int order,
                           hipStream_t s, hipEvent_t* ev)
{
    Src none = {};
    FArgs<R> A = fused_args<R>(o, nf, M, g, alpha, none);
    if (!yee_setup<R>(A, xchunk, order)) return hipErrorInvalidValue;
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    k_yee<R, ROWSY, 2><<<A.nblk, 64 * ROWSY, 0, s>>>(A);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    return hipSuccess;
}

template <typename R>
bool yee2_setup(FArgs<R>& A, int xchunk, int order)
{
    constexpr int TY = ROWSY - 4;
    A.nyt = (A.g.ny + 1 + TY - 1) / TY;
    A.nzt = (A.g.nz + 1 + KTY2 - 1) / KTY2;
    const int nplanes = A.g.nx + 1;
    // every buffer range must stay below 2^31 bytes: (xchunk + 3) planes
    const int64_t plane_bytes = (int64_t)A.g.sp * sizeof(R);
    const int64_t xmax = ((int64_t(1) << 31) - 1) / plane_bytes - 3;
    if (xmax < 1) return false;
    int xc = xchunk;
    if (xc <= 0) {
        const int tiles = A.nyt * A.nzt;
        int chunks = (4096 + tiles - 1) / tiles;
        chunks = std::max(1, std::min(chunks, (nplanes + 31) / 32));
        xc = (nplanes + chunks - 1) / chunks;
    }
    xc = (int)std::min<int64_t>(std::max(xc, 1), xmax);
    A.xchunk = xc;
    A.nxc = (nplanes + xc - 1) / xc;
    A.order = order != 0 ? order : default_order(A.nyt, A.nzt, A.nxc);
    A.nblk = launch_tiles(A.order, A.nyt, A.nzt, A.nxc);
    return true;
}

bool yee2_fits(Geo g, int real_bytes)
{
    return (int64_t)g.sp * real_bytes * 4 < (int64_t(1) << 31);
}

template <typename R>
hipError_t launch_step_yee2(Fields<R> o, Fields<R> nf, Mat<R> M, Geo g, R alpha, int xchunk, int order,
                            hipStream_t s, hipEvent_t* ev)
{
    Src none = {};
    FArgs<R> A = fused_args<R>(o, nf, M, g, alpha, none);
    if (!yee2_setup<R>(A, xchunk, order)) return hipErrorInvalidValue;
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    // two prefetched planes in FP32 (62 VGPRs with one), one in FP64 (120)
    k_yee2<R, ROWSY, sizeof(R) == 4 ? 2 : 1><<<A.nblk, 64 * ROWSY, 0, s>>>(A);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    return hipSuccess;
}

template hipError_t launch_step_yee2<float>(Fields<float>, Fields<float>, Mat<float>, Geo, float, int, int,
                                            hipStream_t, hipEvent_t*);
template hipError_t launch_step_yee2<double>(Fields<double>, Fields<double>, Mat<double>, Geo, double, int, int,
                                             hipStream_t, hipEvent_t*);
template hipError_t launch_step_yee<float>(Fields<float>, Fields<float>, Mat<float>, Geo, float, int, int,
                                           hipStream_t, hipEvent_t*);
template hipError_t launch_step_yee<double>(Fields<double>, Fields<double>, Mat<double>, Geo, double, int, int,
                                            hipStream_t, hipEvent_t*);

}  // namespace tete
