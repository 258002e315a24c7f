// The implicit TE/TM scheme (16) of Sec. 4.1 as a measured comparator of the
// explicit scheme: each half step solves (I - alpha T_i) x = rhs, where T_i
// holds the transverse curls, taken at the mean of the old and new level.
//
// Solving.  Eliminating the transverse components leaves, per z-plane, one
// positive definite system for e_z (first half) and for h_z (second half):
//     (I + alpha^2 kappa_z (P_y^T mu_x P_y + P_x^T mu_y P_x)) e_z = b_e,
//     (I + alpha^2 mu_z (P_y kappa_x P_y^T + P_x kappa_y P_x^T)) h_z = b_h,
// after which h_x, h_y (e_x, e_y) follow from the new e_z (h_z).  Their
// spectra lie in [1, 1 + alpha^2 (4/dx^2 + 4/dy^2)] (Gershgorin, vacuum and
// staircase PEC), so Chebyshev iteration with these bounds converges at a known
// rate: a fixed number of iterations, no inner products, no reductions, and the
// same result for any launch shape.  Every kernel here is one grid-stride pass
// over the entries, z fastest.

#include <math.h>

#include <algorithm>
#include <vector>

#include "tete_impl.h"

namespace tete {
namespace {

constexpr int TBI = 256;
constexpr int kListChunk = 8192;   // entries counted and listed by one block

struct IGeo {
    int nx, ny, nz, sz, sp, np;
};

__device__ __forceinline__ void dec(const IGeo& g, int idx, int& i, int& j, int& k)
{
    i = idx / g.sp;
    const int r = idx - i * g.sp;
    j = r / g.sz;
    k = r - j * g.sz;
}

template <typename R>
struct ICoef {
    R kx, ky, kz, mx, my, mz;   // vacuum kappa and mu
    R a, dt;                    // alpha = dtau / 2, dtau
};

// entry values with zero outside the array (the kept-zero out-of-range
// entries of each component hold zero already)
template <typename R>
__device__ __forceinline__ R val(const R* f, const IGeo& g, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i > g.nx || j > g.ny || k > g.nz) return (R)0;
    return f[k + g.sz * j + g.sp * i];
}

// coefficients that vanish outside the component's range and on PEC edges
template <typename R>
__device__ __forceinline__ R kap_x(const uint8_t* code, const IGeo& g, const ICoef<R>& c, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= g.nx || j > g.ny || k > g.nz) return (R)0;
    return (code[k + g.sz * j + g.sp * i] & 1u) ? (R)0 : c.kx;
}
template <typename R>
__device__ __forceinline__ R kap_y(const uint8_t* code, const IGeo& g, const ICoef<R>& c, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i > g.nx || j >= g.ny || k > g.nz) return (R)0;
    return (code[k + g.sz * j + g.sp * i] & 2u) ? (R)0 : c.ky;
}
template <typename R>
__device__ __forceinline__ R kap_z(const uint8_t* code, const IGeo& g, const ICoef<R>& c, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i > g.nx || j > g.ny || k >= g.nz) return (R)0;
    return (code[k + g.sz * j + g.sp * i] & 4u) ? (R)0 : c.kz;
}
template <typename R>
__device__ __forceinline__ R mu_x(const IGeo& g, const ICoef<R>& c, int i, int j, int k)
{
    return (i < 0 || j < 0 || k < 0 || i > g.nx || j >= g.ny || k >= g.nz) ? (R)0 : c.mx;
}
template <typename R>
__device__ __forceinline__ R mu_y(const IGeo& g, const ICoef<R>& c, int i, int j, int k)
{
    return (i < 0 || j < 0 || k < 0 || i >= g.nx || j > g.ny || k >= g.nz) ? (R)0 : c.my;
}
template <typename R>
__device__ __forceinline__ R mu_z(const IGeo& g, const ICoef<R>& c, int i, int j, int k)
{
    return (i < 0 || j < 0 || k < 0 || i >= g.nx || j >= g.ny || k > g.nz) ? (R)0 : c.mz;
}

// Right-hand sides of the first half step, (I + alpha T_0) u^{n-1/2} +
// dtau (L v^n + j_u^n): r_hx, r_hy into w.hx, w.hy, r_ez into B; the initial
// iterate for e_z is e_z^{n-1/2}.
template <typename R>
__global__ void k_imp_rhs_u(Fields<R> o, Fields<R> w, R* B, const uint8_t* code, IGeo g, ICoef<R> c, Src src)
{
    const R *ex = o.c[0], *ey = o.c[1], *ez = o.c[2], *hx = o.c[3], *hy = o.c[4];
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.np; idx += gridDim.x * blockDim.x) {
        int i, j, k;
        dec(g, idx, i, j, k);
        const R mx = mu_x(g, c, i, j, k), my = mu_y(g, c, i, j, k), kz = kap_z(code, g, c, i, j, k);
        const R e0 = ez[idx];
        // h_x: -alpha mu_x P_y e_z + dtau mu_x P_z e_y
        w.c[3][idx] = mx == (R)0 ? (R)0
                                 : hx[idx] - c.a * mx * (val(ez, g, i, j + 1, k) - e0) +
                                       c.dt * mx * (val(ey, g, i, j, k + 1) - ey[idx]);
        // h_y: +alpha mu_y P_x e_z - dtau mu_y P_z e_x
        w.c[4][idx] = my == (R)0 ? (R)0
                                 : hy[idx] + c.a * my * (val(ez, g, i + 1, j, k) - e0) -
                                       c.dt * my * (val(ex, g, i, j, k + 1) - ex[idx]);
        if (kz == (R)0) {
            B[idx] = (R)0;
            w.c[2][idx] = (R)0;
            continue;
        }
        // e_z: +alpha kappa_z (P_y^T h_x - P_x^T h_y) - dtau kappa_z j_z
        R b = e0 + c.a * kz * ((val(hx, g, i, j - 1, k) - hx[idx]) - (val(hy, g, i - 1, j, k) - hy[idx]));
        if (src.on && i == src.i0 && j == src.j0) {
            const int64_t m = (int64_t)k - src.n + src.M;     // cell m crosses edge k in step n
            if (m >= -src.M && m <= src.M) {
#pragma clang fp contract(off)
                b -= (R)((double)kz * src.lam[m + src.M]);
            }
        }
        B[idx] = b;
        w.c[2][idx] = e0;
    }
}

// b_e = r_ez + alpha kappa_z (P_y^T r_hx - P_x^T r_hy), in place on B
template <typename R>
__global__ void k_imp_b_u(Fields<R> w, R* B, const uint8_t* code, IGeo g, ICoef<R> c)
{
    const R *rhx = w.c[3], *rhy = w.c[4];
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.np; idx += gridDim.x * blockDim.x) {
        int i, j, k;
        dec(g, idx, i, j, k);
        const R kz = kap_z(code, g, c, i, j, k);
        if (kz == (R)0) continue;
        B[idx] += c.a * kz * ((val(rhx, g, i, j - 1, k) - rhx[idx]) - (val(rhy, g, i - 1, j, k) - rhy[idx]));
    }
}

// (A x) of the e_z system at a free entry: x + alpha^2 kappa_z r0 x
template <typename R>
__device__ __forceinline__ R apply_e(const R* x, const uint8_t* code, const IGeo& g, const ICoef<R>& c, int i, int j,
                                     int k, int idx, R kz)
{
    const R x0 = x[idx];
    const R r = mu_x(g, c, i, j - 1, k) * (x0 - val(x, g, i, j - 1, k)) - mu_x(g, c, i, j, k) * (val(x, g, i, j + 1, k) - x0) +
                mu_y(g, c, i - 1, j, k) * (x0 - val(x, g, i - 1, j, k)) - mu_y(g, c, i, j, k) * (val(x, g, i + 1, j, k) - x0);
    return x0 + c.a * c.a * kz * r;
}

// (A x) of the h_z system at an in-range entry: x + alpha^2 mu_z r1 x
template <typename R>
__device__ __forceinline__ R apply_h(const R* x, const uint8_t* code, const IGeo& g, const ICoef<R>& c, int i, int j,
                                     int k, int idx, R mz)
{
    const R x0 = x[idx];
    const R r = kap_x(code, g, c, i, j + 1, k) * (x0 - val(x, g, i, j + 1, k)) -
                kap_x(code, g, c, i, j, k) * (val(x, g, i, j - 1, k) - x0) +
                kap_y(code, g, c, i + 1, j, k) * (x0 - val(x, g, i + 1, j, k)) -
                kap_y(code, g, c, i, j, k) * (val(x, g, i - 1, j, k) - x0);
    return x0 + c.a * c.a * mz * r;
}

// An h_z row whose four surrounding e edges are all PEC (inside the metal) is
// the identity and decoupled from every other unknown: its neighbours reach it
// only through one of those edges, whose kappa is zero.  Its solution is b.
template <typename R>
__device__ __forceinline__ bool h_coupled(const uint8_t* code, const IGeo& g, const ICoef<R>& c, int i, int j, int k)
{
    return kap_x(code, g, c, i, j + 1, k) != (R)0 || kap_x(code, g, c, i, j, k) != (R)0 ||
           kap_y(code, g, c, i + 1, j, k) != (R)0 || kap_y(code, g, c, i, j, k) != (R)0;
}

// Row lists (built once per geometry, ascending): the free e_z edges and the
// coupled h_z rows.  Chunk b of `chunk` entries is counted by block b, the
// host turns the counts into offsets, and block b writes its chunk's rows
// in order (wave ballots and a scan over the block's waves).
template <typename R>
__device__ __forceinline__ void row_flags(const uint8_t* code, const IGeo& g, const ICoef<R>& c, int idx, bool& fe,
                                          bool& fh)
{
    int i, j, k;
    dec(g, idx, i, j, k);
    fe = kap_z(code, g, c, i, j, k) != (R)0;
    fh = mu_z(g, c, i, j, k) != (R)0 && h_coupled(code, g, c, i, j, k);
}

template <typename R>
__global__ __launch_bounds__(TBI) void k_list_count(const uint8_t* code, IGeo g, ICoef<R> c, int chunk, int* cnt)
{
    __shared__ int se[TBI], sh[TBI];
    const int lo = blockIdx.x * chunk, hi = min(lo + chunk, g.np);
    int ne = 0, nh = 0;
    for (int idx = lo + (int)threadIdx.x; idx < hi; idx += TBI) {
        bool fe, fh;
        row_flags(code, g, c, idx, fe, fh);
        ne += fe;
        nh += fh;
    }
    se[threadIdx.x] = ne;
    sh[threadIdx.x] = nh;
    __syncthreads();
    for (int w = TBI / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            se[threadIdx.x] += se[threadIdx.x + w];
            sh[threadIdx.x] += sh[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cnt[2 * blockIdx.x] = se[0];
        cnt[2 * blockIdx.x + 1] = sh[0];
    }
}

template <typename R>
__global__ __launch_bounds__(TBI) void k_list_write(const uint8_t* code, IGeo g, ICoef<R> c, int chunk,
                                                    const int* off, int* le, int* lh)
{
    constexpr int NW = TBI / 64;
    __shared__ int we[NW], wh[NW];
    const int lo = blockIdx.x * chunk, hi = min(lo + chunk, g.np);
    const int wave = threadIdx.x / 64;
    const unsigned long long below = __lanemask_lt();
    int oe = off[2 * blockIdx.x], oh = off[2 * blockIdx.x + 1];
    for (int base = lo; base < hi; base += TBI) {       // same trip count for every thread
        const int idx = base + (int)threadIdx.x;
        bool fe = false, fh = false;
        if (idx < hi) row_flags(code, g, c, idx, fe, fh);
        const unsigned long long me = __ballot(fe), mh = __ballot(fh);
        if ((threadIdx.x & 63) == 0) {
            we[wave] = __popcll(me);
            wh[wave] = __popcll(mh);
        }
        __syncthreads();
        int pe = oe, ph = oh, te = 0, th = 0;
        for (int w = 0; w < NW; ++w) {
            if (w < wave) {
                pe += we[w];
                ph += wh[w];
            }
            te += we[w];
            th += wh[w];
        }
        if (fe) le[pe + __popcll(me & below)] = idx;
        if (fh) lh[ph + __popcll(mh & below)] = idx;
        oe += te;
        oh += th;
        __syncthreads();                                 // the counts are rewritten next round
    }
}

// Chebyshev start on the rows of the list: r = b - A x, d = r / theta.  Rows
// outside the list (PEC e_z edges, h_z outside its range or inside the
// metal) are not unknowns: their x is fixed (0, or h_z^n, which equals b on an
// identity row) and their directions are zero in both buffers of the
// ping-pong pair, which the e_z and h_z solves share: every solve zeroes its
// own rows in both buffers in its last iteration.
template <typename R, bool H>
__global__ void k_cheb_init(const R* X, const R* B, R* Rr, R* D, const int* list, int n, const uint8_t* code, IGeo g,
                            ICoef<R> c, R inv_theta)
{
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const int idx = list[t];
        int i, j, k;
        dec(g, idx, i, j, k);
        const R s = H ? mu_z(g, c, i, j, k) : kap_z(code, g, c, i, j, k);
        const R ax = H ? apply_h(X, code, g, c, i, j, k, idx, s) : apply_e(X, code, g, c, i, j, k, idx, s);
        const R r = B[idx] - ax;
        Rr[idx] = r;
        D[idx] = r * inv_theta;
    }
}

// One Chebyshev step: x += d; unless last: r -= A d, d' = c1 d + c2 r; in the
// last step both direction buffers are cleared on the list's rows
template <typename R, bool H>
__global__ void k_cheb_iter(R* X, R* Rr, R* D, R* Dn, const int* list, int n, const uint8_t* code, IGeo g, ICoef<R> c,
                            R c1, R c2, int last)
{
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        const int idx = list[t];
        int i, j, k;
        dec(g, idx, i, j, k);
        const R s = H ? mu_z(g, c, i, j, k) : kap_z(code, g, c, i, j, k);
        const R d = D[idx];
        X[idx] += d;
        if (last) {   // no thread reads the directions any more
            D[idx] = (R)0;
            Dn[idx] = (R)0;
            continue;
        }
        const R ad = H ? apply_h(D, code, g, c, i, j, k, idx, s) : apply_e(D, code, g, c, i, j, k, idx, s);
        const R r = Rr[idx] - ad;
        Rr[idx] = r;
        Dn[idx] = c1 * d + c2 * r;
    }
}

// h_x = r_hx - alpha mu_x P_y e_z, h_y = r_hy + alpha mu_y P_x e_z (new e_z);
// the wake takes -1/2 (e_z^{n-1/2} + e_z^{n+1/2}) on the bunch line
template <typename R>
__global__ void k_imp_back_u(Fields<R> o, Fields<R> w, const uint8_t* code, IGeo g, ICoef<R> c, Src src)
{
    const R* ez = w.c[2];
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.np; idx += gridDim.x * blockDim.x) {
        int i, j, k;
        dec(g, idx, i, j, k);
        const R mx = mu_x(g, c, i, j, k), my = mu_y(g, c, i, j, k);
        const R e0 = ez[idx];
        if (mx != (R)0) w.c[3][idx] -= c.a * mx * (val(ez, g, i, j + 1, k) - e0);
        if (my != (R)0) w.c[4][idx] += c.a * my * (val(ez, g, i + 1, j, k) - e0);
        if (src.on && i == src.i0 && j == src.j0 && k < src.kend) {
            const int64_t js = src.n - k - src.M;            // wake sample of edge k
            if (js >= src.jmin && js < (int64_t)src.jmin + src.nw)
                src.wacc[js - src.jmin] += -0.5 * ((double)o.c[2][idx] + (double)e0);
        }
    }
}

// Right-hand sides of the second half step, (I + alpha T_1) v^n - dtau L^T
// u^{n+1/2}: r_ex, r_ey into w.ex, w.ey, r_hz into B; initial iterate h_z^n.
template <typename R>
__global__ void k_imp_rhs_v(Fields<R> o, Fields<R> w, R* B, const uint8_t* code, IGeo g, ICoef<R> c)
{
    const R *ex = o.c[0], *ey = o.c[1], *hz = o.c[5], *hx1 = w.c[3], *hy1 = w.c[4];
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.np; idx += gridDim.x * blockDim.x) {
        int i, j, k;
        dec(g, idx, i, j, k);
        const R kx = kap_x(code, g, c, i, j, k), ky = kap_y(code, g, c, i, j, k), mz = mu_z(g, c, i, j, k);
        const R h0 = hz[idx];
        // e_x: -alpha kappa_x P_y^T h_z + dtau kappa_x P_z^T h_y
        w.c[0][idx] = kx == (R)0 ? (R)0
                                 : ex[idx] - c.a * kx * (val(hz, g, i, j - 1, k) - h0) +
                                       c.dt * kx * (val(hy1, g, i, j, k - 1) - hy1[idx]);
        // e_y: +alpha kappa_y P_x^T h_z - dtau kappa_y P_z^T h_x
        w.c[1][idx] = ky == (R)0 ? (R)0
                                 : ey[idx] + c.a * ky * (val(hz, g, i - 1, j, k) - h0) -
                                       c.dt * ky * (val(hx1, g, i, j, k - 1) - hx1[idx]);
        if (mz == (R)0) {
            B[idx] = (R)0;
            w.c[5][idx] = (R)0;
            continue;
        }
        // h_z: +alpha mu_z (P_y e_x - P_x e_y)
        B[idx] = h0 + c.a * mz * ((val(ex, g, i, j + 1, k) - ex[idx]) - (val(ey, g, i + 1, j, k) - ey[idx]));
        w.c[5][idx] = h0;
    }
}

// b_h = r_hz + alpha mu_z (P_y r_ex - P_x r_ey), in place on B
template <typename R>
__global__ void k_imp_b_v(Fields<R> w, R* B, IGeo g, ICoef<R> c)
{
    const R *rex = w.c[0], *rey = w.c[1];
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.np; idx += gridDim.x * blockDim.x) {
        int i, j, k;
        dec(g, idx, i, j, k);
        const R mz = mu_z(g, c, i, j, k);
        if (mz == (R)0) continue;
        B[idx] += c.a * mz * ((val(rex, g, i, j + 1, k) - rex[idx]) - (val(rey, g, i + 1, j, k) - rey[idx]));
    }
}

// e_x = r_ex - alpha kappa_x P_y^T h_z, e_y = r_ey + alpha kappa_y P_x^T h_z (new h_z)
template <typename R>
__global__ void k_imp_back_v(Fields<R> w, const uint8_t* code, IGeo g, ICoef<R> c)
{
    const R* hz = w.c[5];
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < g.np; idx += gridDim.x * blockDim.x) {
        int i, j, k;
        dec(g, idx, i, j, k);
        const R kx = kap_x(code, g, c, i, j, k), ky = kap_y(code, g, c, i, j, k);
        const R h0 = hz[idx];
        if (kx != (R)0) w.c[0][idx] -= c.a * kx * (val(hz, g, i, j - 1, k) - h0);
        if (ky != (R)0) w.c[1][idx] += c.a * ky * (val(hz, g, i - 1, j, k) - h0);
    }
}

int iblocks(int np) { return std::min(16384, std::max(1, (np + TBI - 1) / TBI)); }

// Chebyshev coefficients for spectrum [1, lmax]: (c1, c2) of each step after
// the first (Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1).
struct Cheb {
    double inv_theta;
    std::vector<double> c1, c2;
};

Cheb cheb_plan(double lmax, int iters)
{
    Cheb p;
    const double theta = 0.5 * (lmax + 1.0), delta = 0.5 * (lmax - 1.0);
    p.inv_theta = 1.0 / theta;
    const double s1 = theta / delta;
    double rho = 1.0 / s1;
    for (int t = 1; t < iters; ++t) {
        const double rn = 1.0 / (2.0 * s1 - rho);
        p.c1.push_back(rn * rho);
        p.c2.push_back(2.0 * rn / delta);
        rho = rn;
    }
    return p;
}

template <typename R, bool H>
hipError_t cheb_solve(R* X, const R* B, const ImpWork<R>& wk, const uint8_t* code, const IGeo& g, const ICoef<R>& c,
                      const Cheb& p, int iters, hipStream_t s)
{
    const int* list = H ? wk.lh : wk.le;
    const int n = H ? wk.nh : wk.ne;
    if (n == 0) return hipSuccess;   // no unknowns: x stays as set
    const int nb = iblocks(n);
    k_cheb_init<R, H><<<nb, TBI, 0, s>>>(X, B, wk.r, wk.d[0], list, n, code, g, c, (R)p.inv_theta);
    for (int t = 0; t < iters; ++t) {
        const bool last = t == iters - 1;
        const R c1 = last ? (R)0 : (R)p.c1[t], c2 = last ? (R)0 : (R)p.c2[t];
        k_cheb_iter<R, H><<<nb, TBI, 0, s>>>(X, wk.r, wk.d[t & 1], wk.d[(t + 1) & 1], list, n, code, g, c, c1, c2,
                                             last);
    }
    return hipGetLastError();
}

}  // namespace

// Largest eigenvalue bound 1 + alpha^2 (4/dx^2 + 4/dy^2) and the iterations
// that bring the Chebyshev error factor 2 ((sqrt k - 1)/(sqrt k + 1))^n below
// the precision's tolerance (1e-17 for FP64, 1e-8 for FP32).
int implicit_iters(const Geo& g, double dx, double dy, double alpha, int fp32, double* lmax_out)
{
    (void)g;
    const double lmax = 1.0 + alpha * alpha * (4.0 / (dx * dx) + 4.0 / (dy * dy));
    const double sk = sqrt(lmax), rho = (sk - 1.0) / (sk + 1.0);
    const double tol = fp32 ? 1e-8 : 1e-17;
    int n = rho > 0.0 ? (int)ceil(log(tol / 2.0) / log(rho)) : 1;
    if (lmax_out) *lmax_out = lmax;
    return std::max(1, std::min(n, 10000));
}

int implicit_list_chunks(int64_t np) { return (int)((np + kListChunk - 1) / kListChunk); }

template <typename R>
hipError_t implicit_build_lists(Mat<R> M, Geo geo, int* cnt, int* le, int* lh, int* ne, int* nh, hipStream_t s)
{
    IGeo g{geo.nx, geo.ny, geo.nz, geo.sz, geo.sp, geo.np};
    ICoef<R> c{M.k[0], M.k[1], M.k[2], M.m[0], M.m[1], M.m[2], (R)0, (R)0};
    const int nch = implicit_list_chunks(geo.np);
    hipError_t e;
    k_list_count<R><<<nch, TBI, 0, s>>>(M.code, g, c, kListChunk, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    std::vector<int> h(2 * (size_t)nch);
    if ((e = hipMemcpyAsync(h.data(), cnt, sizeof(int) * h.size(), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    int64_t te = 0, th = 0;                      // exclusive scan of the chunk counts
    for (int b = 0; b < nch; ++b) {
        const int ce = h[2 * b], chh = h[2 * b + 1];
        h[2 * b] = (int)te;
        h[2 * b + 1] = (int)th;
        te += ce;
        th += chh;
    }
    if (te > geo.np || th > geo.np) return hipErrorInvalidValue;
    if ((e = hipMemcpyAsync(cnt, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, s)) != hipSuccess) return e;
    k_list_write<R><<<nch, TBI, 0, s>>>(M.code, g, c, kListChunk, cnt, le, lh);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;   // h is released on return
    *ne = (int)te;
    *nh = (int)th;
    return hipSuccess;
}

template <typename R>
hipError_t launch_step_implicit(Fields<R> o, Fields<R> w, Mat<R> M, Geo geo, double dx, double dy, R alpha, Src src,
                                ImpWork<R> wk, hipStream_t s, hipEvent_t* ev)
{
    IGeo g{geo.nx, geo.ny, geo.nz, geo.sz, geo.sp, geo.np};
    ICoef<R> c{M.k[0], M.k[1], M.k[2], M.m[0], M.m[1], M.m[2], alpha, alpha + alpha};
    double lmax;
    const int iters = implicit_iters(geo, dx, dy, (double)alpha, sizeof(R) == 4, &lmax);
    const Cheb plan = cheb_plan(lmax, iters);
    const int nb = iblocks(g.np);
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    k_imp_rhs_u<R><<<nb, TBI, 0, s>>>(o, w, wk.b, M.code, g, c, src);
    k_imp_b_u<R><<<nb, TBI, 0, s>>>(w, wk.b, M.code, g, c);
    if ((e = cheb_solve<R, false>(w.c[2], wk.b, wk, M.code, g, c, plan, iters, s)) != hipSuccess) return e;
    k_imp_back_u<R><<<nb, TBI, 0, s>>>(o, w, M.code, g, c, src);
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
    k_imp_rhs_v<R><<<nb, TBI, 0, s>>>(o, w, wk.b, M.code, g, c);
    k_imp_b_v<R><<<nb, TBI, 0, s>>>(w, wk.b, g, c);
    if ((e = cheb_solve<R, true>(w.c[5], wk.b, wk, M.code, g, c, plan, iters, s)) != hipSuccess) return e;
    k_imp_back_v<R><<<nb, TBI, 0, s>>>(w, M.code, g, c);
    if (ev && (e = hipEventRecord(ev[2], s)) != hipSuccess) return e;
    return hipGetLastError();
}

template hipError_t implicit_build_lists<float>(Mat<float>, Geo, int*, int*, int*, int*, int*, hipStream_t);
template hipError_t implicit_build_lists<double>(Mat<double>, Geo, int*, int*, int*, int*, int*, hipStream_t);
template hipError_t launch_step_implicit<float>(Fields<float>, Fields<float>, Mat<float>, Geo, double, double, float,
                                                Src, ImpWork<float>, hipStream_t, hipEvent_t*);
template hipError_t launch_step_implicit<double>(Fields<double>, Fields<double>, Mat<double>, Geo, double, double,
                                                 double, Src, ImpWork<double>, hipStream_t, hipEvent_t*);

}  // namespace tete
