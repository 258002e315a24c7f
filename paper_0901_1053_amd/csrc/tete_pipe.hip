// Open entrance and exit pipes (the infinite pipes of the structure of Sec. 5,
// for which the paper gives no method): the bunch's own field in a uniform
// entrance pipe, written as the state a run starts from.
//
// In a pipe whose cross-section does not change along z, a bunch moving at
// v = c on the node line (i0, j0) with dtau = dz carries the field
//   e_x = -(P_x phi) F(k - n),             e_y = -(P_y phi) F(k - n),
//   h_x = (dx/dy) (P_y phi) F(k + 1 - n),  h_y = -(dy/dx) (P_x phi) F(k + 1 - n),
//   e_z = h_z = 0
// one cell per step through the ten sub-updates of scheme (23) (Sec. 4.2):
// along z each transverse edge sees the one-dimensional leapfrog at Courant
// number one; S8 keeps h_z = 0 because the transverse e is a gradient; S3
// keeps e_z = 0 because the transverse divergence of h at step n is the bunch
// current.  phi is the cross-section's potential,
//   (dy/dx)(2 phi - phi(i+1,j) - phi(i-1,j)) + (dx/dy)(2 phi - phi(i,j+1) - phi(i,j-1)) = delta_(i0,j0)
// on the nodes whose e_z edge is not PEC, phi = 0 on the others, solved here
// by conjugate gradients in FP64; F is tied to the current,
//   (F(p) + F(p+1)) / 2 = lam[p + 2M] / dtau (bunch cell p + M crosses edge
//   k in step n, p = k - n), F(p) = 0 for p > 0,
// and continues below p = -2M - 1 as the checkerboard F(p) = -F(p+1).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tete_impl.h"

namespace tete {
namespace {

constexpr int PT = 256;              // threads of the plane kernels
constexpr int PB = RED_BLOCKS;       // most blocks of a reduction pass

__host__ __device__ inline int pblocks(int64_t n) { return (int)(n / PT + 1 < PB ? n / PT + 1 : PB); }

__device__ __forceinline__ double wsum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over the block in a fixed order (waves, then the four wave sums).
__device__ __forceinline__ double bsum(double v)
{
    __shared__ double red[PT / 64];
    v = wsum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
    for (int t = 1; t < PT / 64; ++t) r += red[t];
    __syncthreads();
    return r;
}

// Free-node weight of the cross-section (1: the e_z edge of plane 0 is not
// PEC, 0: PEC), node (i, j) at t = j + (ny + 1) i.
__global__ void k_pipe_mask(double* w, const uint8_t* code, CgPlane P, int sp, int sz)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < P.n; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / (P.ny + 1)), j = (int)(t % (P.ny + 1));
        w[t] = (code[(int64_t)i * sp + (int64_t)j * sz] & 4) ? 0.0 : 1.0;
    }
}

// Cell planes 0 .. kst-1 uniform: every code of a node line repeats its
// first plane (e_z bit from plane 0, e_x and e_y bits from plane 1, as plane 0
// of e_x, e_y lies on the wall).  Any difference sets *bad.
__global__ void k_pipe_uniform(const uint8_t* code, CgPlane P, int sp, int sz, int kst, int* bad)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < P.n; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / (P.ny + 1)), j = (int)(t % (P.ny + 1));
        const uint8_t* c = code + (int64_t)i * sp + (int64_t)j * sz;
        const int z0 = c[0] & 4, t1 = c[1] & 3;
        int diff = 0;
        for (int k = 1; k < kst; ++k) diff |= ((c[k] & 4) != z0) | ((c[k] & 3) != t1);
        if (diff) *bad = 1;
    }
}

// Laplacian of the cross-section applied to p on the free nodes (0 on the
// others); partial[block] = sum of p q.
__global__ __launch_bounds__(PT) void k_cg_apply(double* q, const double* p, const double* w, CgPlane P,
                                                 double* partial)
{
    const int sy = P.ny + 1;
    double s = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < P.n; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t / sy), j = (int)(t % sy);
        double v = 0.0;
        if (w[t] != 0.0) {
            // free nodes lie strictly inside the plane (the walls are PEC), so
            // every neighbour exists; the tests keep the reads in bounds anyway
            const double pim = i > 0 ? p[t - sy] : 0.0, pip = i < P.nx ? p[t + sy] : 0.0;
            const double pjm = j > 0 ? p[t - 1] : 0.0, pjp = j < P.ny ? p[t + 1] : 0.0;
            v = P.wx * ((p[t] - pip) + (p[t] - pim)) + P.wy * ((p[t] - pjp) + (p[t] - pjm));
        }
        q[t] = v;
        s += p[t] * v;
    }
    s = bsum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Scalars of the iteration in sc: rr = |r|^2, alpha, beta, done flag, tol.
enum { CG_RR = 0, CG_ALPHA = 1, CG_BETA = 2, CG_DONE = 3, CG_TOL = 4, CG_ITER = 5 };

__global__ __launch_bounds__(PT) void k_cg_alpha(const double* partial, int nb, double* sc)
{
    double v = 0.0;
    for (int t = threadIdx.x; t < nb; t += blockDim.x) v += partial[t];
    const double pq = bsum(v);
    if (threadIdx.x == 0) sc[CG_ALPHA] = (sc[CG_DONE] != 0.0 || pq == 0.0) ? 0.0 : sc[CG_RR] / pq;
}

__global__ __launch_bounds__(PT) void k_cg_update(double* x, double* r, const double* p, const double* q,
                                                  const double* sc, CgPlane P, double* partial)
{
    const double a = sc[CG_ALPHA];
    double s = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < P.n; t += (int64_t)gridDim.x * blockDim.x) {
        x[t] += a * p[t];
        const double rv = r[t] - a * q[t];
        r[t] = rv;
        s += rv * rv;
    }
    s = bsum(s);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// New |r|^2 and beta; once |r|^2 <= tol the iteration is done and every later
// alpha and beta is 0, which freezes x at the first iterate that met tol.
__global__ __launch_bounds__(PT) void k_cg_beta(const double* partial, int nb, double* sc)
{
    double v = 0.0;
    for (int t = threadIdx.x; t < nb; t += blockDim.x) v += partial[t];
    const double rn = bsum(v);
    if (threadIdx.x == 0) {
        if (sc[CG_DONE] != 0.0) {
            sc[CG_BETA] = 0.0;
        } else {
            sc[CG_BETA] = sc[CG_RR] != 0.0 ? rn / sc[CG_RR] : 0.0;
            sc[CG_RR] = rn;
            sc[CG_ITER] += 1.0;
            if (rn <= sc[CG_TOL]) sc[CG_DONE] = 1.0;
        }
    }
}

__global__ void k_cg_dir(double* p, const double* r, const double* sc, CgPlane P)
{
    const double b = sc[CG_BETA];
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < P.n; t += (int64_t)gridDim.x * blockDim.x)
        p[t] = r[t] + b * p[t];
}

// x = 0, r = p = delta at the bunch node; sc as for a fresh iteration.
__global__ void k_cg_init(double* x, double* r, double* p, CgPlane P, int64_t src, double tol, double* sc)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < P.n; t += (int64_t)gridDim.x * blockDim.x) {
        const double v = t == src ? 1.0 : 0.0;
        x[t] = 0.0;
        r[t] = v;
        p[t] = v;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[CG_RR] = 1.0;
        sc[CG_ALPHA] = sc[CG_BETA] = 0.0;
        sc[CG_DONE] = 0.0;
        sc[CG_TOL] = tol;
        sc[CG_ITER] = 0.0;
    }
}

// Profile table of the bunch current: F[p - lo] for p = lo .. 1, lo = -2M-1,
// from the head down (one thread: the recurrence is sequential).
__global__ void k_pipe_profile(double* F, const double* lam, int M, double dtau)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int lo = -2 * M - 1;
    F[1 - lo] = 0.0;
    for (int q = 0; q >= lo; --q) {
        const double cur = q >= -2 * M ? lam[q + 2 * M] / dtau : 0.0;
        F[q - lo] = 2.0 * cur - F[q + 1 - lo];
    }
}

__device__ __forceinline__ double prof(const double* F, int lo, int64_t p)
{
    if (p > 0) return 0.0;
    if (p >= lo) return F[p - lo];
    return ((lo - p) & 1) ? -F[0] : F[0];
}

// The state y^{n0} of the field above, every entry of the six arrays (e_z,
// h_z, out-of-range entries and PEC edges 0).
template <typename R>
__global__ void k_pipe_field(Fields<R> f, const uint8_t* code, const double* phi, const double* F, int lo, int64_t n0,
                             double rxy, double ryx, Geo g)
{
    const int sy = g.ny + 1;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < g.np;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(idx / g.sp), j = (int)((idx / g.sz) % sy), k = (int)(idx % g.sz);
        const uint8_t c = code[idx];
        const double fe = prof(F, lo, (int64_t)k - n0), fh = prof(F, lo, (int64_t)k + 1 - n0);
        const double* ph = phi + (int64_t)i * sy + j;
        // Ex = -(P_x phi), Ey = -(P_y phi) at this entry's x- and y-edges
        const double Ex = i < g.nx ? -(ph[sy] - ph[0]) : 0.0;
        const double Ey = j < g.ny ? -(ph[1] - ph[0]) : 0.0;
        f.c[0][idx] = (c & 1) ? R(0) : (R)(Ex * fe);
        f.c[1][idx] = (c & 2) ? R(0) : (R)(Ey * fe);
        f.c[2][idx] = R(0);
        f.c[3][idx] = (j < g.ny && k < g.nz) ? (R)((-rxy * Ey) * fh) : R(0);
        f.c[4][idx] = (i < g.nx && k < g.nz) ? (R)((ryx * Ex) * fh) : R(0);
        f.c[5][idx] = R(0);
    }
}

}  // namespace

hipError_t launch_pipe_check(double* w, const uint8_t* code, Geo g, CgPlane P, int kst, int* bad, hipStream_t s)
{
    if (kst < 1 || kst > g.nz) return hipErrorInvalidValue;
    const int nb = pblocks(P.n);
    k_pipe_mask<<<nb, PT, 0, s>>>(w, code, P, g.sp, g.sz);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_pipe_uniform<<<nb, PT, 0, s>>>(code, P, g.sp, g.sz, kst, bad);
    return hipGetLastError();
}

hipError_t launch_cg_init(CgWork W, CgPlane P, int64_t src, double tol, hipStream_t s)
{
    if (src < 0 || src >= P.n) return hipErrorInvalidValue;
    k_cg_init<<<pblocks(P.n), PT, 0, s>>>(W.x, W.r, W.p, P, src, tol, W.sc);
    return hipGetLastError();
}

hipError_t launch_cg_iterations(CgWork W, CgPlane P, int iters, hipStream_t s)
{
    const int nb = pblocks(P.n);
    for (int it = 0; it < iters; ++it) {
        k_cg_apply<<<nb, PT, 0, s>>>(W.q, W.p, W.w, P, W.partial);
        k_cg_alpha<<<1, PT, 0, s>>>(W.partial, nb, W.sc);
        k_cg_update<<<nb, PT, 0, s>>>(W.x, W.r, W.p, W.q, W.sc, P, W.partial);
        k_cg_beta<<<1, PT, 0, s>>>(W.partial, nb, W.sc);
        k_cg_dir<<<nb, PT, 0, s>>>(W.p, W.r, W.sc, P);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_pipe_profile(double* F, const double* lam, int M, double dtau, hipStream_t s)
{
    k_pipe_profile<<<1, 64, 0, s>>>(F, lam, M, dtau);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_pipe_field(Fields<R> f, const uint8_t* code, const double* phi, const double* F, int M, int64_t n0,
                             double rxy, double ryx, Geo g, hipStream_t s)
{
    const int64_t nb = (int64_t)g.np / PT + 1;
    k_pipe_field<R><<<(int)(nb < 65536 ? nb : 65536), PT, 0, s>>>(f, code, phi, F, -2 * M - 1, n0, rxy, ryx, g);
    return hipGetLastError();
}

template hipError_t launch_pipe_field<float>(Fields<float>, const uint8_t*, const double*, const double*, int, int64_t,
                                             double, double, Geo, hipStream_t);
template hipError_t launch_pipe_field<double>(Fields<double>, const uint8_t*, const double*, const double*, int,
                                              int64_t, double, double, Geo, hipStream_t);

}  // namespace tete
