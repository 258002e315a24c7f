// Device helpers shared by the fused step kernels: raw buffer loads and
// stores, whole-wave lane shifts, the XCD-aware workgroup remap and the tile
// schedule.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

#include "tete_impl.h"

namespace tete {
namespace {

// Raw buffer load of one field value at byte offset off (vector) + soff
// (scalar); a lane whose off is past the buffer's size reads 0.
template <typename R>
__device__ __forceinline__ R bload(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff = 0);
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
}
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
template <typename R>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, R v);
template <>
__device__ __forceinline__ void bstore<float>(__amdgpu_buffer_rsrc_t r, uint32_t off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
template <>
__device__ __forceinline__ void bstore<double>(__amdgpu_buffer_rsrc_t r, uint32_t off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

// Neighbours along k are the neighbouring lanes of the wave: DPP whole-wave
// shifts by one lane (lane 0 / lane 63 receive 0; both are halo lanes).  The
// bound control writes the 0, so no register has to be cleared first.
__device__ __forceinline__ int dpp_prev(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_next(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ float lane_prev(float v) { return __builtin_bit_cast(float, dpp_prev(__builtin_bit_cast(int, v))); }
__device__ __forceinline__ float lane_next(float v) { return __builtin_bit_cast(float, dpp_next(__builtin_bit_cast(int, v))); }
typedef int i32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double lane_prev(double v)
{
    i32x2 w = __builtin_bit_cast(i32x2, v);
    w.x = dpp_prev(w.x);
    w.y = dpp_prev(w.y);
    return __builtin_bit_cast(double, w);
}
__device__ __forceinline__ double lane_next(double v)
{
    i32x2 w = __builtin_bit_cast(i32x2, v);
    w.x = dpp_next(w.x);
    w.y = dpp_next(w.y);
    return __builtin_bit_cast(double, w);
}

// Logical tile of a workgroup.  Consecutive hardware workgroups are spread
// round-robin over the eight XCDs; the remap gives each XCD a contiguous range
// of logical tiles so that neighbouring j-tiles (which share halo rows) run on
// the same XCD and share its L2.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int nx = 8;
    int x = b % nx, r = b / nx;
    int base = n / nx, extra = n % nx;
    return x < extra ? x * (base + 1) + r : extra * (base + 1) + (x - extra) * base + r;
}

// Tile (ty, tz) and x-chunk cx of logical workgroup lb.  order 2: k-tiles
// fastest, so the tiles of one band of rows, which together cover whole
// contiguous rows, run together; order 1: j-tiles fastest; orders 3-6: blocks
// of BZ k-tiles by BY j-tiles (8 x 4, 16 x 2, 4 x 8, 2 x 16: 32 workgroups, one
// XCD's worth) fastest, so that neighbouring row bands, which share halo rows,
// also run together and share the XCD's L2.  Order 0 is resolved on the host
// before launch.  Returns false for the padding workgroups of the blocked
// orders.
__host__ __device__ __forceinline__ bool blocked_order(int order) { return order >= 3 && order <= 6; }
__host__ __device__ __forceinline__ int block_z(int order)
{
    return order == 3 ? 8 : order == 4 ? 16 : order == 5 ? 4 : 2;
}
__host__ __device__ __forceinline__ int block_y(int order) { return 32 / block_z(order); }
// Workgroups of one launch: tiles (padded to whole blocks for the blocked
// orders) times x-chunks.
__host__ __device__ __forceinline__ int launch_tiles(int order, int nyt, int nzt, int nxc)
{
    if (!blocked_order(order)) return nyt * nzt * nxc;
    const int BZ = block_z(order), BY = block_y(order);
    return ((nzt + BZ - 1) / BZ) * ((nyt + BY - 1) / BY) * BZ * BY * nxc;
}
// Default tile order: 16 x 2 blocks (order 4) where a block row is filled
// and the launch spans at least eight rounds of 256 workgroups, so that the
// padding of partial blocks averages out over the rounds; otherwise k-tiles
// first (order 2).
inline int default_order(int nyt, int nzt, int nxc)
{
    const bool fill = nzt >= block_z(4) && nyt >= block_y(4);
    return fill && (int64_t)nyt * nzt * nxc >= 8 * 256 ? 4 : 2;
}
__host__ __device__ __forceinline__ bool tile_of(int lb, int order, int nyt, int nzt, int& ty, int& tz, int& cx)
{
    if (order == 2) {
        tz = lb % nzt;
        ty = (lb / nzt) % nyt;
        cx = lb / (nzt * nyt);
        return true;
    }
    if (blocked_order(order)) {
        const int BZ = block_z(order), BY = block_y(order);
        const int nbz = (nzt + BZ - 1) / BZ, nby = (nyt + BY - 1) / BY;
        const int w = lb % (BZ * BY), b = lb / (BZ * BY);
        tz = (b % nbz) * BZ + w % BZ;
        ty = ((b / nbz) % nby) * BY + w / BZ;
        cx = b / (nbz * nby);
        return tz < nzt && ty < nyt;
    }
    ty = lb % nyt;
    tz = (lb / nyt) % nzt;
    cx = lb / (nyt * nzt);
    return true;
}

}  // namespace
}  // namespace tete
