// HIP kernels of libtete for gfx950: set-up (PEC codes, bunch table, field
// import/export), the explicit TE/TM step, and the FP64 diagnostics.
//
// The step follows scheme (23) of Dohlus & Zagorodnov as the ten sub-updates
// of Sec. 4.2: the TM-like group u = (h_x, h_y, e_z) is advanced from
// u^{n-1/2} to u^{n+1/2} with v^n, then the TE-like group v = (e_x, e_y, h_z)
// from v^n to v^{n+1} with u^{n+1/2}.  Each group is one kernel that writes a
// second (ping-pong) copy of its three arrays, so no thread ever reads a value
// another thread of the same launch writes.  The intermediate values h_x^n,
// h_y^n (S1, S2) and e_x^{n+1/2}, e_y^{n+1/2} (S6, S7) are never stored: each
// thread recomputes the ones its stencil touches.

#include <float.h>
#include <math.h>

#include <algorithm>

#include "tete_dev.h"
#include "tete_impl.h"

namespace tete {
namespace {

constexpr int TB = 256;   // threads per block of the element-wise kernels

__device__ __forceinline__ void decomp(int idx, const Geo& g, int& i, int& j, int& k)
{
    i = idx / g.sp;
    int r = idx - i * g.sp;
    j = r / g.sz;
    k = r - j * g.sz;
}

__device__ __forceinline__ bool in_nodes(const Geo& g, int i, int j, int k)
{
    return (unsigned)i <= (unsigned)g.nx && (unsigned)j <= (unsigned)g.ny && (unsigned)k <= (unsigned)g.nz;
}

__device__ __forceinline__ int lin(const Geo& g, int i, int j, int k) { return k + j * g.sz + i * g.sp; }

// Component index ranges (entries outside them hold no grid object).
__device__ __forceinline__ bool ex_ok(const Geo& g, int i, int, int) { return i < g.nx; }
__device__ __forceinline__ bool ey_ok(const Geo& g, int, int j, int) { return j < g.ny; }
__device__ __forceinline__ bool ez_ok(const Geo& g, int, int, int k) { return k < g.nz; }
__device__ __forceinline__ bool hx_ok(const Geo& g, int, int j, int k) { return j < g.ny && k < g.nz; }
__device__ __forceinline__ bool hy_ok(const Geo& g, int i, int, int k) { return i < g.nx && k < g.nz; }
__device__ __forceinline__ bool hz_ok(const Geo& g, int i, int j, int) { return i < g.nx && j < g.ny; }

__device__ __forceinline__ bool comp_ok(int c, const Geo& g, int i, int j, int k)
{
    switch (c) {
    case 0: return ex_ok(g, i, j, k);
    case 1: return ey_ok(g, i, j, k);
    case 2: return ez_ok(g, i, j, k);
    case 3: return hx_ok(g, i, j, k);
    case 4: return hy_ok(g, i, j, k);
    default: return hz_ok(g, i, j, k);
    }
}

template <typename R>
__device__ __forceinline__ R ld(const R* p, const Geo& g, int i, int j, int k)
{
    return in_nodes(g, i, j, k) ? p[lin(g, i, j, k)] : R(0);
}

// M_eps^-1 entry of e component c (0..2) at linear index id.
template <typename R>
__device__ __forceinline__ R kap(const Mat<R>& M, int c, int id)
{
    if (M.arr[c]) return M.arr[c][id];
    return ((M.code[id] >> c) & 1) ? R(0) : M.k[c];
}

// M_mu^-1 entry of h component c (0..2).
template <typename R>
__device__ __forceinline__ R muv(const Mat<R>& M, int c, int id)
{
    return M.arr[3 + c] ? M.arr[3 + c][id] : M.m[c];
}

// ---------------------------------------------------------------------------
// Set-up kernels
// ---------------------------------------------------------------------------

__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}

__global__ void k_zero16(uint4* p, int64_t n)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_fill_f64(double* p, int64_t n, double v)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}

// Staircase PEC: an edge is PEC if any of its (up to four) adjacent cells is
// PEC; cells outside the box count as PEC, so the edges tangential to the
// walls are PEC (n x E = 0).  Entries outside a component's range are marked
// too, which keeps them at zero.
__global__ void k_build_codes(uint8_t* code, const uint8_t* cells, Geo g)
{
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.np) return;
    int i, j, k;
    decomp(idx, g, i, j, k);
    auto pec = [&](int ci, int cj, int ck) -> bool {
        if (ci < 0 || cj < 0 || ck < 0 || ci >= g.nx || cj >= g.ny || ck >= g.nz) return true;
        return cells ? cells[ck + g.nz * (cj + g.ny * ci)] != 0 : false;
    };
    uint8_t c = 0;
    if (i >= g.nx || pec(i, j - 1, k - 1) || pec(i, j, k - 1) || pec(i, j - 1, k) || pec(i, j, k)) c |= 1;
    if (j >= g.ny || pec(i - 1, j, k - 1) || pec(i, j, k - 1) || pec(i - 1, j, k) || pec(i, j, k)) c |= 2;
    if (k >= g.nz || pec(i - 1, j - 1, k) || pec(i, j - 1, k) || pec(i - 1, j, k) || pec(i, j, k)) c |= 4;
    code[idx] = c;
}

// Cell charges of the truncated Gaussian: lam[m+M] = Q [Phi(b) - Phi(a)],
// a = (m-1/2) dz/sigma, b = (m+1/2) dz/sigma, written with erfc on the side
// of the mean where the difference does not cancel.
__global__ void k_lambda(double* lam, double Q, double sigma, double dz, int M)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t > 2 * M) return;
    int m = t - M;
    const double r2 = 0.70710678118654752440;   // 1/sqrt(2)
    double a = (m - 0.5) * dz / sigma, b = (m + 0.5) * dz / sigma, v;
    if (a >= 0.0)
        v = 0.5 * (erfc(a * r2) - erfc(b * r2));
    else if (b <= 0.0)
        v = 0.5 * (erfc(-b * r2) - erfc(-a * r2));
    else
        v = 1.0 - 0.5 * erfc(-a * r2) - 0.5 * erfc(b * r2);
    lam[t] = Q * v;
}

template <typename R>
__device__ __forceinline__ bool e_pec(const Mat<R>& M, int c, int id)
{
    return kap(M, c, id) == R(0);
}

template <typename R>
__global__ void k_import(Fields<R> dst, const void* s0, const void* s1, const void* s2, const void* s3,
                         const void* s4, const void* s5, int src_fp32, Mat<R> M, Geo g)
{
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.np) return;
    int i, j, k;
    decomp(idx, g, i, j, k);
    const void* src[6] = {s0, s1, s2, s3, s4, s5};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        R v = src_fp32 ? (R)((const float*)src[c])[idx] : (R)((const double*)src[c])[idx];
        bool keep = comp_ok(c, g, i, j, k) && (c >= 3 || !e_pec(M, c, idx));
        dst.c[c][idx] = keep ? v : R(0);
    }
}

template <typename R>
__global__ void k_export(void* d0, void* d1, void* d2, void* d3, void* d4, void* d5, int dst_fp32,
                         Fields<R> src, Geo g)
{
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.np) return;
    void* dst[6] = {d0, d1, d2, d3, d4, d5};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        if (dst_fp32)
            ((float*)dst[c])[idx] = (float)src.c[c][idx];
        else
            ((double*)dst[c])[idx] = (double)src.c[c][idx];
    }
}

template <typename R>
__global__ void k_import_mat(R* d0, R* d1, R* d2, R* d3, R* d4, R* d5, const void* s0, const void* s1,
                             const void* s2, const void* s3, const void* s4, const void* s5, int src_fp32,
                             Geo g)
{
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.np) return;
    int i, j, k;
    decomp(idx, g, i, j, k);
    R* dst[6] = {d0, d1, d2, d3, d4, d5};
    const void* src[6] = {s0, s1, s2, s3, s4, s5};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        R v = src_fp32 ? (R)((const float*)src[c])[idx] : (R)((const double*)src[c])[idx];
        dst[c][idx] = comp_ok(c, g, i, j, k) ? v : R(0);
    }
}

template <typename R>
__global__ void k_zero_pec(Fields<R> f, Mat<R> M, Geo g)
{
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.np) return;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        if (e_pec(M, c, idx)) f.c[c][idx] = R(0);
}

// ---------------------------------------------------------------------------
// TM-like half step: S1..S5.  One thread per node entry (i,j,k) writes
// h_x^{n+1/2}, h_y^{n+1/2}, e_z^{n+1/2} there.  The bunch current enters S3
// on the node line (i0, j0); the wake accumulator takes the time-centred
// e_z of the thread's own edge (no two threads share a sample in one step).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(TB) void k_tm(Fields<R> o, Fields<R> nf, Mat<R> M, Geo g, R a, Src src)
{
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.np) return;
    int i, j, k;
    decomp(idx, g, i, j, k);
    const R* ex = o.c[0];
    const R* ey = o.c[1];
    const R* ez = o.c[2];
    const R* hx = o.c[3];
    const R* hy = o.c[4];
    const R a2 = a + a;

    // S1: h_x^n = h_x^{n-1/2} + a mu_x [P_z e_y^n - P_y e_z^{n-1/2}]
    auto hxn = [&](int ii, int jj) -> R {
        if (!in_nodes(g, ii, jj, k) || !hx_ok(g, ii, jj, k)) return R(0);
        int id = lin(g, ii, jj, k);
        return hx[id] + a * muv(M, 0, id) * ((ld(ey, g, ii, jj, k + 1) - ey[id]) - (ld(ez, g, ii, jj + 1, k) - ez[id]));
    };
    // S2: h_y^n = h_y^{n-1/2} + a mu_y [-P_z e_x^n + P_x e_z^{n-1/2}]
    auto hyn = [&](int ii, int jj) -> R {
        if (!in_nodes(g, ii, jj, k) || !hy_ok(g, ii, jj, k)) return R(0);
        int id = lin(g, ii, jj, k);
        return hy[id] + a * muv(M, 1, id) * (-(ld(ex, g, ii, jj, k + 1) - ex[id]) + (ld(ez, g, ii + 1, jj, k) - ez[id]));
    };
    // S3: e_z^{n+1/2} = e_z^{n-1/2} + 2a kappa_z [P_y^T h_x^n - P_x^T h_y^n - j_z^n]
    auto ezh = [&](int ii, int jj) -> R {
        if (!in_nodes(g, ii, jj, k) || !ez_ok(g, ii, jj, k)) return R(0);
        int id = lin(g, ii, jj, k);
        R kp = kap(M, 2, id);
        R v = ez[id] + a2 * kp * ((hxn(ii, jj - 1) - hxn(ii, jj)) - (hyn(ii - 1, jj) - hyn(ii, jj)));
        if (src.on && ii == src.i0 && jj == src.j0) {
            int64_t m = (int64_t)k - src.n + src.M;       // charge of cell m crosses edge k in step n
            if (m >= -src.M && m <= src.M) {
                // the current term is rounded on its own, as in the fused kernels
#pragma clang fp contract(off)
                v -= (R)((double)kp * src.lam[m + src.M]);
            }
        }
        return v;
    };

    const R e0 = ezh(i, j);
    nf.c[2][idx] = e0;
    // S4: h_x^{n+1/2} = h_x^n + a mu_x [P_z e_y^n - P_y e_z^{n+1/2}]
    R hxv = R(0);
    if (hx_ok(g, i, j, k))
        hxv = hxn(i, j) + a * muv(M, 0, idx) * ((ld(ey, g, i, j, k + 1) - ey[idx]) - (ezh(i, j + 1) - e0));
    nf.c[3][idx] = hxv;
    // S5: h_y^{n+1/2} = h_y^n + a mu_y [-P_z e_x^n + P_x e_z^{n+1/2}]
    R hyv = R(0);
    if (hy_ok(g, i, j, k))
        hyv = hyn(i, j) + a * muv(M, 1, idx) * (-(ld(ex, g, i, j, k + 1) - ex[idx]) + (ezh(i + 1, j) - e0));
    nf.c[4][idx] = hyv;

    // wake: W(s_j) sample of edge k is taken in step n = k + M + j
    if (src.on && i == src.i0 && j == src.j0 && k < src.kend) {
        int64_t js = src.n - k - src.M;
        if (js >= src.jmin && js < (int64_t)src.jmin + src.nw)
            src.wacc[js - src.jmin] += -0.5 * ((double)ez[idx] + (double)e0);
    }
}

// ---------------------------------------------------------------------------
// TE-like half step: S6..S10 with u^{n+1/2} (the TM kernel's output).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(TB) void k_te(Fields<R> o, Fields<R> nf, Mat<R> M, Geo g, R a)
{
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.np) return;
    int i, j, k;
    decomp(idx, g, i, j, k);
    const R* ex = o.c[0];
    const R* ey = o.c[1];
    const R* hz = o.c[5];
    const R* hx1 = nf.c[3];
    const R* hy1 = nf.c[4];
    const R a2 = a + a;

    // S6: e_x^{n+1/2} = e_x^n + a kappa_x [P_z^T h_y^{n+1/2} - P_y^T h_z^n]
    auto exh = [&](int ii, int jj) -> R {
        if (!in_nodes(g, ii, jj, k)) return R(0);
        int id = lin(g, ii, jj, k);
        return ex[id] + a * kap(M, 0, id) * ((ld(hy1, g, ii, jj, k - 1) - hy1[id]) - (ld(hz, g, ii, jj - 1, k) - hz[id]));
    };
    // S7: e_y^{n+1/2} = e_y^n + a kappa_y [-P_z^T h_x^{n+1/2} + P_x^T h_z^n]
    auto eyh = [&](int ii, int jj) -> R {
        if (!in_nodes(g, ii, jj, k)) return R(0);
        int id = lin(g, ii, jj, k);
        return ey[id] + a * kap(M, 1, id) * (-(ld(hx1, g, ii, jj, k - 1) - hx1[id]) + (ld(hz, g, ii - 1, jj, k) - hz[id]));
    };
    // S8: h_z^{n+1} = h_z^n + 2a mu_z [P_y e_x^{n+1/2} - P_x e_y^{n+1/2}]
    auto hzn = [&](int ii, int jj) -> R {
        if (!in_nodes(g, ii, jj, k) || !hz_ok(g, ii, jj, k)) return R(0);
        int id = lin(g, ii, jj, k);
        return hz[id] + a2 * muv(M, 2, id) * ((exh(ii, jj + 1) - exh(ii, jj)) - (eyh(ii + 1, jj) - eyh(ii, jj)));
    };

    const R h0 = hzn(i, j);
    nf.c[5][idx] = h0;
    // S9: e_x^{n+1} = e_x^{n+1/2} + a kappa_x [P_z^T h_y^{n+1/2} - P_y^T h_z^{n+1}]
    nf.c[0][idx] = exh(i, j) + a * kap(M, 0, idx) * ((ld(hy1, g, i, j, k - 1) - hy1[idx]) - (hzn(i, j - 1) - h0));
    // S10: e_y^{n+1} = e_y^{n+1/2} + a kappa_y [-P_z^T h_x^{n+1/2} + P_x^T h_z^{n+1}]
    nf.c[1][idx] = eyh(i, j) + a * kap(M, 1, idx) * (-(ld(hx1, g, i, j, k - 1) - hx1[idx]) + (hzn(i - 1, j) - h0));
}

// ---------------------------------------------------------------------------
// FP64 diagnostics
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ double nan_max(double a, double b)
{
    if (a != a || b != b) return NAN;
    return a > b ? a : b;
}

__device__ __forceinline__ double wave_max(double v)
{
    for (int off = 32; off > 0; off >>= 1) v = nan_max(v, __shfl_down(v, off, 64));
    return v;
}

template <bool MAX>
__device__ __forceinline__ double block_reduce(double v)
{
    __shared__ double red[RED_THREADS / 64];
    v = MAX ? wave_max(v) : wave_sum(v);
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
    for (int t = 1; t < RED_THREADS / 64; ++t) r = MAX ? nan_max(r, red[t]) : r + red[t];
    __syncthreads();
    return r;
}

template <typename R>
__device__ __forceinline__ double ldd(const R* p, const Geo& g, int i, int j, int k)
{
    return (double)ld(p, g, i, j, k);
}

// W^{n,e} = 1/2 <Q^e y, y> (Sec. 4.4) expanded over the grid entries:
//   1/2 [sum h^2/mu + sum_{kappa>0} e^2/kappa]
//   - a^2/2 [sum_hx mu_x (P_y e_z)^2 + sum_hy mu_y (P_x e_z)^2
//            + sum_{ex,kappa>0} kappa_x (P_y^T h_z)^2 + sum_{ey,kappa>0} kappa_y (P_x^T h_z)^2]
//   + a [sum_hx h_x P_z e_y - sum_hy h_y P_z e_x]
// With rw = 0 the a^2 terms drop: the energy of the implicit scheme (16),
// whose Q = B - alpha A holds no transverse operator.
//
// Work decomposition: a work item is a tile of EN_ROWS rows (j, one wave each)
// by 63 entries (k) and a chunk of xc planes, marched along x; workgroup b
// takes items b, b + gridDim.x, ...  Each lane loads its entry's six values
// and its PEC code two planes ahead.  The k-neighbour (e_x, e_y at k+1) is the
// next lane (lane 63 only supplies it), the j-neighbours (h_z at j-1, e_z at
// j+1) come through LDS from the neighbouring waves (the tile's first and last
// rows load theirs), and the x-neighbours are the planes before and after in
// registers: every value is read from HBM about once and no index is divided
// per entry.  In vacuum 1/kappa and 1/mu are formed once.  The sums are per
// lane in plane order, then per workgroup and finished in a fixed order, so
// the result does not depend on timing.
constexpr int EN_ROWS = 8;
constexpr int EN_KT = 63;
constexpr int EN_THREADS = 64 * EN_ROWS;

template <typename R, bool ARR>
struct EnPlane {
    R ex, ey, ez, hx, hy, hz, hz_jm, ez_jp;
    uint32_t c;
    R m[ARR ? 6 : 1];   // per-entry kappa_x .. mu_z (ARR)
};

// ARR: per-entry materials, loaded with the fields (M.arr[0..5] all set);
// else vacuum coefficients and the PEC codes.
template <typename R, bool ARR>
__global__ __launch_bounds__(EN_THREADS) void k_energy(Fields<R> f, Mat<R> M, Geo g, double a, double rw, int nyt,
                                                       int nzt, int xc, int items, double* partial)
{
    // h_z and e_z of the plane being summed, in two buffers taken in turn by
    // the planes the workgroup sums, across its work items (one barrier per
    // plane: a buffer is rewritten two planes later, after the next barrier,
    // which every wave reaches only once it has read the buffer)
    __shared__ R sHZ[2][EN_ROWS][64], sEZ[2][EN_ROWS][64];
    __shared__ double red[EN_ROWS];
    const R *ex = f.c[0], *ey = f.c[1], *ez = f.c[2], *hx = f.c[3], *hy = f.c[4], *hz = f.c[5];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // vacuum reciprocals (per-entry arrays divide per entry)
    const double ik[3] = {1.0 / (double)M.k[0], 1.0 / (double)M.k[1], 1.0 / (double)M.k[2]};
    const double im[3] = {1.0 / (double)M.m[0], 1.0 / (double)M.m[1], 1.0 / (double)M.m[2]};
    const double ra2 = 0.5 * rw * a * a;
    double acc = 0.0;
    int turn = 0;   // planes summed so far by the workgroup
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int tz = it % nzt, q = it / nzt, ty = q % nyt, cx = q / nyt;
        const int j = ty * EN_ROWS + w, k = tz * EN_KT + lane;
        const bool node = j <= g.ny && k <= g.nz;
        const bool own = node && lane < EN_KT;
        const int roff = k + j * g.sz;
        const int xs = cx * xc, xe = min(xs + xc, g.nx + 1);
        // Loads of a plane, issued by every lane from a valid address (entry 0
        // outside the grid), so that no load sits in a branch and the waits
        // count only the loads they need.  Values loaded outside the grid are
        // never used: a term reads its own entry, the next lane's only when
        // k < nz, the next plane's only when i < nx, and a j-neighbour only
        // when it lies in the grid (h_z at j-1 is taken as 0 for j = 0).  The
        // waves of the tile's inner rows load their own entry again instead of
        // a j-neighbour (cache hits).
        auto load = [&](int i, EnPlane<R, ARR>& d) {
            const bool ok = node && i >= 0 && i <= g.nx;
            const int id = ok ? roff + i * g.sp : 0;
            d.ex = ex[id];
            d.ey = ey[id];
            d.ez = ez[id];
            d.hx = hx[id];
            d.hy = hy[id];
            d.hz = hz[id];
            int idm = ok && w == 0 && j >= 1 ? id - g.sz : id;
            int idp = ok && w == EN_ROWS - 1 && j < g.ny ? id + g.sz : id;
            // opaque to the compiler, so that it issues these loads instead of
            // reusing the entry's own (which would make them conditional)
            asm volatile("" : "+v"(idm), "+v"(idp));
            d.hz_jm = hz[idm];
            d.ez_jp = ez[idp];
            d.c = M.code ? (uint32_t)M.code[id] : 0u;
            if constexpr (ARR) {
#pragma unroll
                for (int c = 0; c < 6; ++c) d.m[c] = M.arr[c][id];
            }
        };
        // kappa of e component c and mu of h component c of plane d
        auto kapc = [&](int c, const EnPlane<R, ARR>& d) {
            if constexpr (ARR) return (double)d.m[c];
            else return ((d.c >> c) & 1u) ? 0.0 : (double)M.k[c];
        };
        auto muc = [&](int c, const EnPlane<R, ARR>& d) {
            if constexpr (ARR) return (double)d.m[3 + c];
            else return (double)M.m[c];
        };
        // v^2 / kappa (or / mu): the vacuum reciprocal, else a division
        auto sqk = [&](double v, double kv, int c) {
            if constexpr (ARR) return v * v / kv;
            else return v * v * ik[c];
        };
        auto sqm = [&](double v, double mv, int c) {
            if constexpr (ARR) return v * v / mv;
            else return v * v * im[c];
        };

        EnPlane<R, ARR> cur, nxt;
        load(xs, cur);
        load(xs + 1, nxt);
        R hz_im = (node && xs >= 1) ? hz[roff + (xs - 1) * g.sp] : R(0);   // h_z at plane i-1
        for (int i = xs; i < xe; ++i) {
            const int x = turn++ & 1;
            sHZ[x][w][lane] = cur.hz;
            sEZ[x][w][lane] = cur.ez;
            __syncthreads();
            const R hz_jm = w > 0 ? sHZ[x][w - 1][lane] : (j >= 1 ? cur.hz_jm : R(0));
            const R ez_jp = w < EN_ROWS - 1 ? sEZ[x][w + 1][lane] : cur.ez_jp;
            EnPlane<R, ARR> n2;
            load(i + 2, n2);
            // k-neighbours from the next lane, with every lane active
            const double eyk = (double)lane_next(cur.ey), exk = (double)lane_next(cur.ex);
            if (own) {
                double sq = 0.0, r = 0.0, lc = 0.0;
                const double kx = kapc(0, cur), ky = kapc(1, cur), kz = kapc(2, cur);
                const double hzv = (double)cur.hz;
                if (kx > 0.0) {
                    const double d = (double)hz_jm - hzv;
                    sq += sqk((double)cur.ex, kx, 0);
                    r += kx * d * d;
                }
                if (ky > 0.0) {
                    const double d = (double)hz_im - hzv;
                    sq += sqk((double)cur.ey, ky, 1);
                    r += ky * d * d;
                }
                if (kz > 0.0) sq += sqk((double)cur.ez, kz, 2);
                if (j < g.ny && k < g.nz) {                       // h_x
                    const double mu = muc(0, cur), h = (double)cur.hx;
                    if (mu > 0.0) sq += sqm(h, mu, 0);
                    const double d = (double)ez_jp - (double)cur.ez;
                    r += mu * d * d;
                    lc += h * (eyk - (double)cur.ey);
                }
                if (i < g.nx && k < g.nz) {                       // h_y
                    const double mu = muc(1, cur), h = (double)cur.hy;
                    if (mu > 0.0) sq += sqm(h, mu, 1);
                    const double d = (double)nxt.ez - (double)cur.ez;
                    r += mu * d * d;
                    lc -= h * (exk - (double)cur.ex);
                }
                if (i < g.nx && j < g.ny) {                       // h_z
                    const double mu = muc(2, cur);
                    if (mu > 0.0) sq += sqm(hzv, mu, 2);
                }
                acc += 0.5 * sq - ra2 * r + a * lc;
            }
            hz_im = cur.hz;
            cur = nxt;
            nxt = n2;
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) red[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = red[0];
        for (int t = 1; t < EN_ROWS; ++t) s += red[t];
        partial[blockIdx.x] = s;
    }
}

template <bool MAX>
__global__ __launch_bounds__(RED_THREADS) void k_finish(const double* partial, int n, int stride, double* out)
{
    double v = MAX ? 0.0 : 0.0;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        double x = partial[(int64_t)t * stride];
        v = MAX ? nan_max(v, x) : v + x;
    }
    double r = block_reduce<MAX>(v);
    if (threadIdx.x == 0) *out = r;
}

// Conserved charges (Sec. 4.5), from y^n (o) and y^{n+1} (nf):
//  q_e^{n+1/2} at nodes with six non-PEC edges, compared with the charge of the
//  bunch inside the node's dual cell at tau_{n+1/2}: lam_{k-n-1+M} on the bunch line;
//  q_h^n at every cell (must stay zero).
template <typename R>
__global__ __launch_bounds__(RED_THREADS) void k_charges(Fields<R> o, Fields<R> nf, Mat<R> M, Geo g, double a,
                                                         Src src, double* partial)
{
    double me = 0.0, mh = 0.0;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.np; idx += gridDim.x * blockDim.x) {
        int i, j, k;
        decomp(idx, g, i, j, k);
        // ---- q_e at node (i,j,k)
        if (i > 0 && j > 0 && k > 0 && i < g.nx && j < g.ny && k < g.nz) {
            int ixm = lin(g, i - 1, j, k), jym = lin(g, i, j - 1, k), kzm = lin(g, i, j, k - 1);
            double kx0 = kap(M, 0, idx), kx1 = kap(M, 0, ixm), ky0 = kap(M, 1, idx), ky1 = kap(M, 1, jym),
                   kz0 = kap(M, 2, idx), kz1 = kap(M, 2, kzm);
            if (kx0 > 0 && kx1 > 0 && ky0 > 0 && ky1 > 0 && kz0 > 0 && kz1 > 0) {
                auto dbar = [&](int c, int id, double kp) {
                    return 0.5 * ((double)o.c[c][id] + (double)nf.c[c][id]) / kp;
                };
                // dtil_z(kk) = e_z/kappa_z - a^2 (P_y^T mu_x P_y + P_x^T mu_y P_x) e_z at level kk, e_z^{n+1/2}
                auto dtil = [&](int kk, double kp) {
                    const R* e = nf.c[2];
                    int id = lin(g, i, j, kk);
                    double e0 = e[id];
                    double mxm = muv(M, 0, lin(g, i, j - 1, kk)), mxp = muv(M, 0, id);
                    double mym = muv(M, 1, lin(g, i - 1, j, kk)), myp = muv(M, 1, id);
                    double rr = mxm * (e0 - (double)e[lin(g, i, j - 1, kk)]) - mxp * ((double)e[lin(g, i, j + 1, kk)] - e0)
                              + mym * (e0 - (double)e[lin(g, i - 1, j, kk)]) - myp * ((double)e[lin(g, i + 1, j, kk)] - e0);
                    return e0 / kp - a * a * rr;
                };
                double q = dbar(0, idx, kx0) - dbar(0, ixm, kx1) + dbar(1, idx, ky0) - dbar(1, jym, ky1)
                         + dtil(k, kz0) - dtil(k - 1, kz1);
                double want = 0.0;
                if (src.on && i == src.i0 && j == src.j0) {
                    int64_t m = (int64_t)k - src.n - 1 + src.M;
                    if (m >= -src.M && m <= src.M) want = src.lam[m + src.M];
                }
                double res = fabs(q - want);
                me = nan_max(me, (res <= DBL_MAX) ? res : NAN);
            }
        }
        // ---- q_h at cell (i,j,k)
        if (i < g.nx && j < g.ny && k < g.nz) {
            auto bbar = [&](int c, int id) {
                double mu = muv(M, c - 3, id);
                return mu > 0.0 ? 0.5 * ((double)o.c[c][id] + (double)nf.c[c][id]) / mu : 0.0;
            };
            auto btil = [&](int kk) {
                const R* h = o.c[5];
                int id = lin(g, i, j, kk);
                double mu = muv(M, 2, id);
                if (!(mu > 0.0)) return 0.0;
                double h0 = h[id];
                double gxp = (double)kap(M, 0, lin(g, i, j + 1, kk)) * (h0 - ldd(h, g, i, j + 1, kk));
                double gx0 = (double)kap(M, 0, id) * (ldd(h, g, i, j - 1, kk) - h0);
                double gyp = (double)kap(M, 1, lin(g, i + 1, j, kk)) * (h0 - ldd(h, g, i + 1, j, kk));
                double gy0 = (double)kap(M, 1, id) * (ldd(h, g, i - 1, j, kk) - h0);
                return h0 / mu - a * a * ((gxp - gx0) + (gyp - gy0));
            };
            double q = bbar(3, lin(g, i + 1, j, k)) - bbar(3, idx) + bbar(4, lin(g, i, j + 1, k)) - bbar(4, idx)
                     + btil(k + 1) - btil(k);
            double res = fabs(q);
            mh = nan_max(mh, (res <= DBL_MAX) ? res : NAN);
        }
    }
    double re = block_reduce<true>(me);
    double rh = block_reduce<true>(mh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = re;
        partial[2 * blockIdx.x + 1] = rh;
    }
}

template <typename R>
__global__ void k_probes(const R* ez, const int64_t* idx, int n, double* out)
{
    int t = threadIdx.x;
    if (t < n) out[t] = (double)ez[idx[t]];
}

// The probes' e_z after one step from state o, for a two-step launch that
// never stores that state: one thread per probe evaluates S3 at its edge from
// S1 and S2 at the four h edges around it, the formulas and the order of
// operations of the TM half step (k_tm), bunch current included.
template <typename R>
__global__ void k_probes_next(Fields<R> o, Mat<R> M, Geo g, R a, Src src, const int64_t* idx, int n, double* out)
{
    const int t = threadIdx.x;
    if (t >= n) return;
    int i, j, k;
    decomp((int)idx[t], g, i, j, k);
    const R* ex = o.c[0];
    const R* ey = o.c[1];
    const R* ez = o.c[2];
    const R* hx = o.c[3];
    const R* hy = o.c[4];
    const R a2 = a + a;
    // S1 and S2 at (ii, jj, k)
    auto hxn = [&](int ii, int jj) -> R {
        if (!in_nodes(g, ii, jj, k) || !hx_ok(g, ii, jj, k)) return R(0);
        int id = lin(g, ii, jj, k);
        return hx[id] + a * muv(M, 0, id) * ((ld(ey, g, ii, jj, k + 1) - ey[id]) - (ld(ez, g, ii, jj + 1, k) - ez[id]));
    };
    auto hyn = [&](int ii, int jj) -> R {
        if (!in_nodes(g, ii, jj, k) || !hy_ok(g, ii, jj, k)) return R(0);
        int id = lin(g, ii, jj, k);
        return hy[id] + a * muv(M, 1, id) * (-(ld(ex, g, ii, jj, k + 1) - ex[id]) + (ld(ez, g, ii + 1, jj, k) - ez[id]));
    };
    R v = R(0);
    if (ez_ok(g, i, j, k)) {
        const int id = lin(g, i, j, k);
        const R kp = kap(M, 2, id);
        v = ez[id] + a2 * kp * ((hxn(i, j - 1) - hxn(i, j)) - (hyn(i - 1, j) - hyn(i, j)));
        if (src.on && i == src.i0 && j == src.j0) {
            int64_t m = (int64_t)k - src.n + src.M;
            if (m >= -src.M && m <= src.M) {
#pragma clang fp contract(off)
                v -= (R)((double)kp * src.lam[m + src.M]);
            }
        }
    }
    out[t] = (double)v;
}

// One thread per (edge k, line blockIdx.y).  Within one step the edges of a
// line feed distinct samples, so no two threads add to one accumulator.
template <typename R>
__global__ void k_witness(const R* ez_old, const R* ez_new, Witness w, int kend, int64_t n, int M, int jmin, int nw,
                          double* acc)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kend) return;
    const int64_t js = n - k - M;
    if (js < jmin || js >= (int64_t)jmin + nw) return;
    const int l = blockIdx.y;
    const int64_t o = w.base[l] + k;
    acc[(int64_t)l * TETE_MAX_WAKE + (js - jmin)] += -0.5 * ((double)ez_old[o] + (double)ez_new[o]);
}

// Two steps n, n+1 of one two-step launch, one thread per (sample, line):
// sample j takes edge k = n - j - M in step n and edge k+1 in step n+1, added
// in that order, as two single steps would add them.
template <typename R>
__global__ void k_witness2(const R* ez_old, const R* ez_mid, const R* ez_new, Witness w, int nz, int kend, int64_t n,
                           int M, int jmin, int nw, double* acc)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nw) return;
    const int l = blockIdx.y;
    const int64_t k = n - ((int64_t)jmin + t) - M;
    const R* mid = ez_mid + (int64_t)l * nz;
    double a = acc[(int64_t)l * TETE_MAX_WAKE + t];
    if (k >= 0 && k < kend) a += -0.5 * ((double)ez_old[w.base[l] + k] + (double)mid[k]);
    if (k + 1 >= 0 && k + 1 < kend) a += -0.5 * ((double)mid[k + 1] + (double)ez_new[w.base[l] + k + 1]);
    acc[(int64_t)l * TETE_MAX_WAKE + t] = a;
}

// ---------------------------------------------------------------------------
// Stability of general diagonal materials (Sec. 4.4: the scheme is stable when
// Q^e is positive definite).  In the scaled variables a = h / sqrt(mu),
// b = e / sqrt(kappa) the form 2 W^{n,e} = |u|^2 + |v|^2 - alpha^2 (<R_0 u, u>
// + <R_1 v, v>) + 2 alpha <L v, u> falls into three independent blocks:
//   e_z alone:  I - alpha^2 R_0, with R_0 the transverse mu-weighted
//               difference operator on the kappa_z-scaled e_z;
//   h_z alone:  I - alpha^2 R_1, the same with kappa_x, kappa_y on h_z;
//   (h_x, h_y, e_x, e_y):  [[I, alpha L], [alpha L^T, I]], L = the
//               z-differences between h_x and e_y, h_y and e_x.
// Each block is positive semi-definite when, in every row, the diagonal part
// subtracted from the identity plus the off-diagonal magnitudes is at most 1
// (Gershgorin).  This kernel forms those row sums for the rows of every
// entry and reduces their maximum; with vacuum coefficients it is
// max(cdt^2 (dx^-2 + dy^-2), cdt / dz) at interior rows, the bound (25).
// Entries outside a component's index range are not read; a negative or
// non-finite value in range makes the result NaN.
// ---------------------------------------------------------------------------
// Per-entry material arrays (kappa_x, kappa_y, kappa_z, mu_x, mu_y, mu_z).
template <typename S>
struct MatSrc {
    const S* c[6];
    __device__ double v(int comp, const Geo& g, int i, int j, int k) const
    {
        if (!in_nodes(g, i, j, k) || !comp_ok(comp, g, i, j, k)) return 0.0;
        return (double)c[comp][lin(g, i, j, k)];
    }
    __device__ bool bad(const Geo& g, int idx, int i, int j, int k) const
    {
        bool b = false;
#pragma unroll
        for (int comp = 0; comp < 6; ++comp) {
            if (!comp_ok(comp, g, i, j, k)) continue;
            const double x = (double)c[comp][idx];
            if (!(x >= 0.0) || x > DBL_MAX) b = true;
        }
        return b;
    }
};

// Materials by class: the table's values of the entry's class, kappa zero
// where the PEC code marks the edge (the table itself is checked on the host).
struct ClsSrc {
    const uint8_t* code;
    const uint8_t* cls;
    const double* tab;   // TETE_MAX_CLASSES x 6
    int ncls;
    __device__ double v(int comp, const Geo& g, int i, int j, int k) const
    {
        if (!in_nodes(g, i, j, k) || !comp_ok(comp, g, i, j, k)) return 0.0;
        const int id = lin(g, i, j, k);
        if (comp < 3 && ((code[id] >> comp) & 1u)) return 0.0;
        return tab[6 * (int)cls[id] + comp];
    }
    __device__ bool bad(const Geo&, int idx, int, int, int) const { return (int)cls[idx] >= ncls; }
};

template <typename SRC>
__global__ __launch_bounds__(RED_THREADS) void k_mat_bound(SRC m, Geo g, double a, double* partial)
{
    double worst = 0.0;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.np; idx += gridDim.x * blockDim.x) {
        int i, j, k;
        decomp(idx, g, i, j, k);
        if (m.bad(g, idx, i, j, k)) {
            worst = NAN;
            continue;
        }
        double s = 0.0;
        // e_z row: alpha^2 sum over its four h facets of mu (kappa_z + sqrt(kappa_z kappa_z'))
        const double kz = m.v(2, g, i, j, k);
        if (kz > 0.0) {
            const double r = m.v(3, g, i, j, k) * (kz + sqrt(kz * m.v(2, g, i, j + 1, k)))
                           + m.v(3, g, i, j - 1, k) * (kz + sqrt(kz * m.v(2, g, i, j - 1, k)))
                           + m.v(4, g, i, j, k) * (kz + sqrt(kz * m.v(2, g, i + 1, j, k)))
                           + m.v(4, g, i - 1, j, k) * (kz + sqrt(kz * m.v(2, g, i - 1, j, k)));
            s = fmax(s, a * a * r);
        }
        // h_z row: alpha^2 sum over its four e edges of kappa (mu_z + sqrt(mu_z mu_z'))
        const double mz = m.v(5, g, i, j, k);
        if (mz > 0.0) {
            const double r = m.v(0, g, i, j, k) * (mz + sqrt(mz * m.v(5, g, i, j - 1, k)))
                           + m.v(0, g, i, j + 1, k) * (mz + sqrt(mz * m.v(5, g, i, j + 1, k)))
                           + m.v(1, g, i, j, k) * (mz + sqrt(mz * m.v(5, g, i - 1, j, k)))
                           + m.v(1, g, i + 1, j, k) * (mz + sqrt(mz * m.v(5, g, i + 1, j, k)));
            s = fmax(s, a * a * r);
        }
        // rows of the L block: h_x with e_y at k, k+1; h_y with e_x at k, k+1;
        // e_y with h_x at k-1, k; e_x with h_y at k-1, k
        const double mx = m.v(3, g, i, j, k), my = m.v(4, g, i, j, k);
        const double kx = m.v(0, g, i, j, k), ky = m.v(1, g, i, j, k);
        s = fmax(s, a * sqrt(mx) * (sqrt(ky) + sqrt(m.v(1, g, i, j, k + 1))));
        s = fmax(s, a * sqrt(my) * (sqrt(kx) + sqrt(m.v(0, g, i, j, k + 1))));
        s = fmax(s, a * sqrt(ky) * (sqrt(mx) + sqrt(m.v(3, g, i, j, k - 1))));
        s = fmax(s, a * sqrt(kx) * (sqrt(my) + sqrt(m.v(4, g, i, j, k - 1))));
        worst = nan_max(worst, s);
    }
    const double r = block_reduce<true>(worst);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

// Materials by class -> the six per-entry arrays (kappa zero on PEC codes,
// every component zero outside its range).
template <typename R>
__global__ void k_expand_classes(R* d0, R* d1, R* d2, R* d3, R* d4, R* d5, const uint8_t* code,
                                 const uint8_t* cls, const double* tab, Geo g)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.np) return;
    int i, j, k;
    decomp(idx, g, i, j, k);
    R* dst[6] = {d0, d1, d2, d3, d4, d5};
    const int c0 = 6 * (int)cls[idx];
    const uint32_t pec = code[idx];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const bool zero = !comp_ok(c, g, i, j, k) || (c < 3 && ((pec >> c) & 1u));
        dst[c][idx] = zero ? R(0) : (R)tab[c0 + c];
    }
}

template <typename R>
struct Six {
    R* c[6];
};

// Classes recognised in per-entry arrays (tete_set_materials): entries with
// the same six coefficients share a class.  A table of CLS_SLOTS slots keyed
// by a 64-bit hash of the tuple's bits (open addressing, linear probing)
// collects the distinct tuples; a second pass finds each entry's slot,
// checks its tuple against the slot's bitwise (two tuples with one hash
// fail this check) and writes its class byte.  Entries outside a
// component's range hold 0 there, as imported.  flags[0]: the table
// overflowed or took more than TETE_MAX_CLASSES tuples (flags[3] counts
// them); flags[1]: an e edge that the PEC codes mark carries a nonzero kappa
// (the class kernel takes kappa 0 there from the codes); flags[2]: a tuple
// differs from its slot's.  The insert pass stops early once flags[0] or
// flags[1] is set: the arrays are then no classes whatever the rest holds.
__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    x ^= x >> 30;
    x *= 0xbf58476d1ce4e5b9ull;
    x ^= x >> 27;
    x *= 0x94d049bb133111ebull;
    x ^= x >> 31;
    return x;
}

template <typename R>
__device__ __forceinline__ uint64_t bits_of(R v)
{
    if constexpr (sizeof(R) == 4) return (uint64_t)__builtin_bit_cast(uint32_t, v);
    else return __builtin_bit_cast(uint64_t, v);
}

template <typename R>
__device__ __forceinline__ uint64_t tuple_key(const R (&v)[6])
{
    uint64_t h = 0x9e3779b97f4a7c15ull;
#pragma unroll
    for (int c = 0; c < 6; ++c) h = mix64(h ^ (bits_of(v[c]) + (uint64_t)(c + 1) * 0x632be59bd9b4e019ull));
    return h | 1ull;                      // 0 marks an empty slot
}

template <typename R>
__global__ void k_classify_insert(Six<const R> m, const uint8_t* code, Geo g, unsigned long long* keys,
                                  double* vals, int* flags)
{
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < g.np;
         idx += (int64_t)gridDim.x * blockDim.x) {
        // the arrays are no classes once flags[0] or flags[1] is set: stop
        // (a graded medium fills the table within its first entries, and every
        // later new tuple would probe all its slots)
        if (*(volatile const int*)&flags[0] | *(volatile const int*)&flags[1]) break;
        R v[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = m.c[c][idx];
        const uint32_t pec = code[idx];
        if ((((pec & 1u) && v[0] != R(0)) || ((pec & 2u) && v[1] != R(0)) || ((pec & 4u) && v[2] != R(0))))
            flags[1] = 1;
        const unsigned long long key = tuple_key(v);
        int slot = (int)((key >> 32) & (CLS_SLOTS - 1));
        bool placed = false;
        for (int t = 0; t < CLS_SLOTS && !placed; ++t) {
            // read first: after the first insertion every entry of the class
            // finds its key without an atomic
            unsigned long long cur = keys[slot];
            if (cur == 0ull) {
                cur = atomicCAS(&keys[slot], 0ull, key);
                if (cur == 0ull) {                     // this entry inserted the tuple
#pragma unroll
                    for (int c = 0; c < 6; ++c) vals[6 * slot + c] = (double)v[c];
                    // more tuples than classes: as good as an overflow
                    if (atomicAdd(&flags[3], 1) >= TETE_MAX_CLASSES) flags[0] = 1;
                    placed = true;
                    break;
                }
            }
            if (cur == key) placed = true;
            else slot = (slot + 1) & (CLS_SLOTS - 1);
        }
        if (!placed) flags[0] = 1;
    }
}

template <typename R>
__global__ void k_classify_assign(Six<const R> m, Geo g, const unsigned long long* keys, const double* vals,
                                  const int* slot_class, uint8_t* cls, int* flags)
{
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < g.np;
         idx += (int64_t)gridDim.x * blockDim.x) {
        R v[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = m.c[c][idx];
        const unsigned long long key = tuple_key(v);
        int slot = (int)((key >> 32) & (CLS_SLOTS - 1));
        int found = -1;
        for (int t = 0; t < CLS_SLOTS; ++t) {
            const unsigned long long cur = keys[slot];
            if (cur == key) { found = slot; break; }
            if (cur == 0ull) break;
            slot = (slot + 1) & (CLS_SLOTS - 1);
        }
        bool same = found >= 0 && slot_class[found] >= 0;
        if (same) {
#pragma unroll
            for (int c = 0; c < 6; ++c) same = same && bits_of((R)vals[6 * found + c]) == bits_of(v[c]);
        }
        if (!same) {
            flags[2] = 1;
            cls[idx] = 0;
        } else {
            cls[idx] = (uint8_t)slot_class[found];
        }
    }
}

// The step kernels' class table: per class the coefficients multiplied by
// their factor in the field type, as the materials step forms them from its
// arrays (a mu, 2a kappa_z, ...; a = alpha rounded to R, 2a = a + a).
template <typename R>
__global__ void k_class_table(R* ctab, const double* tab, R a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= TETE_MAX_CLASSES) return;
    const R a2 = a + a;
    const double* t = tab + 6 * c;
    R* o = ctab + CLS_STRIDE * c;
    o[CLS_AMX] = a * (R)t[3];
    o[CLS_AMY] = a * (R)t[4];
    o[CLS_A2MZ] = a2 * (R)t[5];
    o[CLS_A2KZ] = a2 * (R)t[2];
    o[CLS_AKY] = a * (R)t[1];
    o[CLS_AKX] = a * (R)t[0];
    o[CLS_KZ] = (R)t[2];
    o[7] = R(0);
}

// ---------------------------------------------------------------------------
// Streaming ceiling of the step's access pattern: six arrays and the PEC code
// byte read, six arrays written, every access a coalesced 16-byte load or
// store (four consecutive entries per thread).  out_c[i] = in_c[i], or 0
// where bit 7 of code[i] is set (never for the library's codes, but the code
// must be read).  n is a multiple of 4 handled by whole threads; the host
// copies the remainder with a second launch of this kernel at offset.
// ---------------------------------------------------------------------------

template <typename R>
__global__ __launch_bounds__(256) void k_stream(Six<R> in, Six<R> out, const uint8_t* code, int64_t n4)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n4) return;
    const uint32_t cw = ((const uint32_t*)code)[t];
    if constexpr (sizeof(R) == 4) {
        const uint32_t keep[4] = {(cw & 0x80u) ? 0u : ~0u, (cw & 0x8000u) ? 0u : ~0u, (cw & 0x800000u) ? 0u : ~0u,
                                  (cw & 0x80000000u) ? 0u : ~0u};
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            uint4 v = ((const uint4*)in.c[c])[t];
            v.x &= keep[0];
            v.y &= keep[1];
            v.z &= keep[2];
            v.w &= keep[3];
            ((uint4*)out.c[c])[t] = v;
        }
    } else {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            uint4 v0 = ((const uint4*)in.c[c])[2 * t], v1 = ((const uint4*)in.c[c])[2 * t + 1];
            if (cw & 0x80u) v0.x = v0.y = 0u;
            if (cw & 0x8000u) v0.z = v0.w = 0u;
            if (cw & 0x800000u) v1.x = v1.y = 0u;
            if (cw & 0x80000000u) v1.z = v1.w = 0u;
            ((uint4*)out.c[c])[2 * t] = v0;
            ((uint4*)out.c[c])[2 * t + 1] = v1;
        }
    }
}

template <typename R>
__global__ void k_stream_tail(Six<R> in, Six<R> out, const uint8_t* code, int64_t from, int64_t n)
{
    const int64_t i = from + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool z = (code[i] & 0x80u) != 0;
#pragma unroll
    for (int c = 0; c < 6; ++c) out.c[c][i] = z ? R(0) : in.c[c][i];
}

inline int nblocks(int64_t n, int tb) { return (int)((n + tb - 1) / tb); }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int nb = (int)std::min<int64_t>(nblocks(n, TB), 65536);
    k_fill_u8<<<nb, TB, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int nb = (int)std::min<int64_t>(nblocks(n, TB), 65536);
    k_fill_f64<<<nb, TB, 0, s>>>(p, n, v);
    return hipGetLastError();
}

hipError_t launch_zero_bytes(void* p, size_t bytes, hipStream_t s)
{
    // bulk in 16-byte stores (p is 256-byte aligned), tail bytewise
    int64_t n16 = (int64_t)(bytes / 16);
    if (n16 > 0) {
        int nb = (int)std::min<int64_t>(nblocks(n16, TB), 65536);
        k_zero16<<<nb, TB, 0, s>>>((uint4*)p, n16);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return launch_fill_u8((uint8_t*)p + n16 * 16, (int64_t)(bytes - n16 * 16), 0, s);
}

hipError_t launch_build_codes(uint8_t* code, const uint8_t* cells, Geo g, hipStream_t s)
{
    k_build_codes<<<nblocks(g.np, TB), TB, 0, s>>>(code, cells, g);
    return hipGetLastError();
}

hipError_t launch_lambda(double* lam, double Q, double sigma, double dz, int M, hipStream_t s)
{
    k_lambda<<<nblocks(2 * M + 1, TB), TB, 0, s>>>(lam, Q, sigma, dz, M);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_import(Fields<R> dst, const void* const src[6], int src_fp32, Mat<R> mat, Geo g, hipStream_t s)
{
    k_import<R><<<nblocks(g.np, TB), TB, 0, s>>>(dst, src[0], src[1], src[2], src[3], src[4], src[5], src_fp32, mat, g);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_export(void* const dst[6], int dst_fp32, Fields<R> src, Geo g, hipStream_t s)
{
    k_export<R><<<nblocks(g.np, TB), TB, 0, s>>>(dst[0], dst[1], dst[2], dst[3], dst[4], dst[5], dst_fp32, src, g);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_import_materials(R* const dst[6], const void* const src[6], int src_fp32, Geo g, hipStream_t s)
{
    k_import_mat<R><<<nblocks(g.np, TB), TB, 0, s>>>(dst[0], dst[1], dst[2], dst[3], dst[4], dst[5], src[0], src[1],
                                                     src[2], src[3], src[4], src[5], src_fp32, g);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_zero_pec(Fields<R> f, Mat<R> mat, Geo g, hipStream_t s)
{
    k_zero_pec<R><<<nblocks(g.np, TB), TB, 0, s>>>(f, mat, g);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_step(Fields<R> oldf, Fields<R> newf, Mat<R> mat, Geo g, R alpha, Src src, hipStream_t s,
                       hipEvent_t* ev)
{
    int nb = nblocks(g.np, TB);
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    k_tm<R><<<nb, TB, 0, s>>>(oldf, newf, mat, g, alpha, src);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    k_te<R><<<nb, TB, 0, s>>>(oldf, newf, mat, g, alpha);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    return hipSuccess;
}

hipError_t launch_mat_bound(const void* const src[6], int src_fp32, Geo g, double alpha, double* partial,
                            double* out, hipStream_t s)
{
    if (src_fp32) {
        MatSrc<float> m;
        for (int c = 0; c < 6; ++c) m.c[c] = (const float*)src[c];
        k_mat_bound<MatSrc<float>><<<RED_BLOCKS, RED_THREADS, 0, s>>>(m, g, alpha, partial);
    } else {
        MatSrc<double> m;
        for (int c = 0; c < 6; ++c) m.c[c] = (const double*)src[c];
        k_mat_bound<MatSrc<double>><<<RED_BLOCKS, RED_THREADS, 0, s>>>(m, g, alpha, partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_finish<true><<<1, RED_THREADS, 0, s>>>(partial, RED_BLOCKS, 1, out);
    return hipGetLastError();
}

hipError_t launch_mat_bound_cls(const uint8_t* code, const uint8_t* cls, const double* table, int ncls, Geo g,
                                double alpha, double* partial, double* out, hipStream_t s)
{
    ClsSrc m{code, cls, table, ncls};
    k_mat_bound<ClsSrc><<<RED_BLOCKS, RED_THREADS, 0, s>>>(m, g, alpha, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_finish<true><<<1, RED_THREADS, 0, s>>>(partial, RED_BLOCKS, 1, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_expand_classes(R* const dst[6], R* ctab, const uint8_t* code, const uint8_t* cls,
                                 const double* table, R alpha, Geo g, hipStream_t s)
{
    k_expand_classes<R><<<nblocks(g.np, TB), TB, 0, s>>>(dst[0], dst[1], dst[2], dst[3], dst[4], dst[5], code, cls,
                                                         table, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_class_table<R><<<1, TETE_MAX_CLASSES, 0, s>>>(ctab, table, alpha);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_classify(R* const arr[6], const uint8_t* code, Geo g, unsigned long long* keys, double* vals,
                           const int* slot_class, uint8_t* cls, int* flags, int pass, hipStream_t s)
{
    Six<const R> m;
    for (int c = 0; c < 6; ++c) m.c[c] = arr[c];
    const int nb = (int)std::min<int64_t>(nblocks(g.np, TB), 16384);
    if (pass == 0) k_classify_insert<R><<<nb, TB, 0, s>>>(m, code, g, keys, vals, flags);
    else k_classify_assign<R><<<nb, TB, 0, s>>>(m, g, keys, vals, slot_class, cls, flags);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_class_table(R* ctab, const double* table, R alpha, hipStream_t s)
{
    k_class_table<R><<<1, TETE_MAX_CLASSES, 0, s>>>(ctab, table, alpha);
    return hipGetLastError();
}

hipError_t launch_stream(void* const in[6], void* const out[6], const uint8_t* code, int64_t n, int fp32,
                         hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t n4 = n / 4;
    auto run = [&](auto tag) -> hipError_t {
        typedef decltype(tag) R;
        Six<R> a, b;
        for (int c = 0; c < 6; ++c) {
            a.c[c] = (R*)in[c];
            b.c[c] = (R*)out[c];
        }
        if (n4 > 0) k_stream<R><<<(unsigned)((n4 + 255) / 256), 256, 0, s>>>(a, b, code, n4);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (4 * n4 < n) k_stream_tail<R><<<1, 256, 0, s>>>(a, b, code, 4 * n4, n);
        return hipGetLastError();
    };
    return fp32 ? run(float(0)) : run(double(0));
}

template <typename R>
hipError_t launch_energy(Fields<R> f, Mat<R> mat, Geo g, double alpha, double rw, double* partial, double* out,
                         hipStream_t s)
{
    // tiles of EN_ROWS x EN_KT entries; chunks of at least 32 planes, short
    // enough that each workgroup takes about 16 work items
    const int nyt = (g.ny + 1 + EN_ROWS - 1) / EN_ROWS, nzt = (g.nz + 1 + EN_KT - 1) / EN_KT;
    const int64_t tiles = (int64_t)nyt * nzt, planes = g.nx + 1;
    int64_t xc = (planes * tiles + 16 * RED_BLOCKS - 1) / (16 * RED_BLOCKS);
    xc = std::min<int64_t>(std::max<int64_t>(xc, 32), planes);
    const int64_t items = tiles * ((planes + xc - 1) / xc);
    if (items > 0x7fffffff) return hipErrorInvalidValue;
    const int grid = (int)std::min<int64_t>(items, RED_BLOCKS);
    bool arr = true;
    for (int c = 0; c < 6; ++c) arr = arr && mat.arr[c] != nullptr;
    if (arr) k_energy<R, true><<<grid, EN_THREADS, 0, s>>>(f, mat, g, alpha, rw, nyt, nzt, (int)xc, (int)items, partial);
    else k_energy<R, false><<<grid, EN_THREADS, 0, s>>>(f, mat, g, alpha, rw, nyt, nzt, (int)xc, (int)items, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_finish<false><<<1, RED_THREADS, 0, s>>>(partial, grid, 1, out);
    return hipGetLastError();
}

hipError_t launch_sum(const double* part, int n, int stride, double* out, hipStream_t s)
{
    k_finish<false><<<1, RED_THREADS, 0, s>>>(part, n, stride, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_charges(Fields<R> oldf, Fields<R> newf, Mat<R> mat, Geo g, double alpha, Src src, double* partial,
                          double* out, hipStream_t s)
{
    k_charges<R><<<RED_BLOCKS, RED_THREADS, 0, s>>>(oldf, newf, mat, g, alpha, src, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_finish<true><<<1, RED_THREADS, 0, s>>>(partial, RED_BLOCKS, 2, out);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_finish<true><<<1, RED_THREADS, 0, s>>>(partial + 1, RED_BLOCKS, 2, out + 1);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_probes(const R* ez, const int64_t* idx, int nprobe, double* out, hipStream_t s)
{
    if (nprobe <= 0) return hipSuccess;
    k_probes<R><<<1, 64, 0, s>>>(ez, idx, nprobe, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_probes_next(Fields<R> o, Mat<R> mat, Geo g, R alpha, Src src, const int64_t* idx, int nprobe,
                              double* out, hipStream_t s)
{
    if (nprobe <= 0) return hipSuccess;
    if (nprobe > 64) return hipErrorInvalidValue;
    k_probes_next<R><<<1, 64, 0, s>>>(o, mat, g, alpha, src, idx, nprobe, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_witness2(const R* ez_old, const R* ez_mid, const R* ez_new, Witness w, Geo g, int64_t n, int M,
                           int jmin, int nw, int kend, double* acc, hipStream_t s)
{
    if (nw < 1 || nw > TETE_MAX_WAKE || kend < 0 || kend > g.nz) return hipErrorInvalidValue;
    for (int l = 0; l < TETE_WITNESS_LINES; ++l)   // every line inside the array
        if (w.base[l] < 0 || w.base[l] + g.nz > (int64_t)g.np) return hipErrorInvalidValue;
    k_witness2<R><<<dim3(nblocks(nw, TB), TETE_WITNESS_LINES), TB, 0, s>>>(ez_old, ez_mid, ez_new, w, g.nz, kend, n,
                                                                          M, jmin, nw, acc);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_witness(const R* ez_old, const R* ez_new, Witness w, Geo g, int64_t n, int M, int jmin, int nw,
                          int kend, double* acc, hipStream_t s)
{
    if (nw < 1 || nw > TETE_MAX_WAKE || kend < 0 || kend > g.nz) return hipErrorInvalidValue;
    for (int l = 0; l < TETE_WITNESS_LINES; ++l)   // every line inside the array
        if (w.base[l] < 0 || w.base[l] + g.nz > (int64_t)g.np) return hipErrorInvalidValue;
    k_witness<R><<<dim3(nblocks(g.nz, TB), TETE_WITNESS_LINES), TB, 0, s>>>(ez_old, ez_new, w, kend, n, M, jmin, nw,
                                                                            acc);
    return hipGetLastError();
}

#define TETE_INST(R)                                                                                              \
    template hipError_t launch_import<R>(Fields<R>, const void* const[6], int, Mat<R>, Geo, hipStream_t);          \
    template hipError_t launch_export<R>(void* const[6], int, Fields<R>, Geo, hipStream_t);                        \
    template hipError_t launch_import_materials<R>(R* const[6], const void* const[6], int, Geo, hipStream_t);      \
    template hipError_t launch_expand_classes<R>(R* const[6], R*, const uint8_t*, const uint8_t*, const double*, R, \
                                                 Geo, hipStream_t);                                              \
    template hipError_t launch_classify<R>(R* const[6], const uint8_t*, Geo, unsigned long long*, double*,         \
                                           const int*, uint8_t*, int*, int, hipStream_t);                         \
    template hipError_t launch_class_table<R>(R*, const double*, R, hipStream_t);                                  \
    template hipError_t launch_zero_pec<R>(Fields<R>, Mat<R>, Geo, hipStream_t);                                   \
    template hipError_t launch_step<R>(Fields<R>, Fields<R>, Mat<R>, Geo, R, Src, hipStream_t, hipEvent_t*);                    \
    template hipError_t launch_energy<R>(Fields<R>, Mat<R>, Geo, double, double, double*, double*, hipStream_t);           \
    template hipError_t launch_charges<R>(Fields<R>, Fields<R>, Mat<R>, Geo, double, Src, double*, double*,        \
                                          hipStream_t);                                                            \
    template hipError_t launch_probes<R>(const R*, const int64_t*, int, double*, hipStream_t);                     \
    template hipError_t launch_probes_next<R>(Fields<R>, Mat<R>, Geo, R, Src, const int64_t*, int, double*,        \
                                              hipStream_t);                                                        \
    template hipError_t launch_witness<R>(const R*, const R*, Witness, Geo, int64_t, int, int, int, int, double*,   \
                                          hipStream_t);                                                            \
    template hipError_t launch_witness2<R>(const R*, const R*, const R*, Witness, Geo, int64_t, int, int, int, int, \
                                           double*, hipStream_t);

TETE_INST(double)
TETE_INST(float)

}  // namespace tete
