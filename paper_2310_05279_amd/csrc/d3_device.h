// Device helpers shared by the HIP translation units (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace d3 {

// DPP controls of the GFX9 family
constexpr int DPP_QUAD_1032 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_2301 = 0x4E;  // quad_perm [2,3,0,1]
constexpr int DPP_ROW_ROR4 = 0x124;  // row_ror:4
constexpr int DPP_ROW_ROR8 = 0x128;  // row_ror:8
constexpr int DPP_ROW_BCAST15 = 0x142;
constexpr int DPP_ROW_BCAST31 = 0x143;

// v from the lane the DPP control selects; lanes the row mask excludes get
// an undefined value (the sums below only read lane 63, whose inputs are
// always selected)
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, ROW_MASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sums over the 64 lanes of a wave of N values at once; the results are
// wave-uniform.  Every lane of a row gets the row sum from quad permutes
// and row rotations, then row broadcasts 15 and 31 carry the partial sums
// into lane 63, which is read back.  The N values go through each step
// together, so their DPP wait states overlap.
template <int N>
__device__ __forceinline__ void wave_sums(double (&v)[N])
{
#pragma unroll
    for (int c = 0; c < N; c++) v[c] += dpp_f64<DPP_QUAD_1032, 0xF>(v[c]);
#pragma unroll
    for (int c = 0; c < N; c++) v[c] += dpp_f64<DPP_QUAD_2301, 0xF>(v[c]);
#pragma unroll
    for (int c = 0; c < N; c++) v[c] += dpp_f64<DPP_ROW_ROR4, 0xF>(v[c]);
#pragma unroll
    for (int c = 0; c < N; c++) v[c] += dpp_f64<DPP_ROW_ROR8, 0xF>(v[c]);
#pragma unroll
    for (int c = 0; c < N; c++) v[c] += dpp_f64<DPP_ROW_BCAST15, 0xA>(v[c]);
#pragma unroll
    for (int c = 0; c < N; c++) v[c] += dpp_f64<DPP_ROW_BCAST31, 0xC>(v[c]);
#pragma unroll
    for (int c = 0; c < N; c++) {
        const int lo = __builtin_amdgcn_readlane(__double2loint(v[c]), 63);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(v[c]), 63);
        v[c] = __hiloint2double(hi, lo);
    }
}

// Sum over each DPP row (16 lanes): quad permutes then row rotations by 4
// and 8.  Every lane of a row ends with the row sum, added in a lane-
// dependent order; callers that need one value per row broadcast a lane.
__device__ __forceinline__ double row_sum(double v)
{
    v += dpp_f64<DPP_QUAD_1032, 0xF>(v);
    v += dpp_f64<DPP_QUAD_2301, 0xF>(v);
    v += dpp_f64<DPP_ROW_ROR4, 0xF>(v);
    v += dpp_f64<DPP_ROW_ROR8, 0xF>(v);
    return v;
}

__device__ __forceinline__ double row_min(double v)
{
    v = fmin(v, dpp_f64<DPP_QUAD_1032, 0xF>(v));
    v = fmin(v, dpp_f64<DPP_QUAD_2301, 0xF>(v));
    v = fmin(v, dpp_f64<DPP_ROW_ROR4, 0xF>(v));
    v = fmin(v, dpp_f64<DPP_ROW_ROR8, 0xF>(v));
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
    double a[1] = {v};
    wave_sums(a);
    return a[0];
}

__device__ __forceinline__ float wave_sum(float v)
{
    int b = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_mov_dpp(b, DPP_QUAD_1032, 0xF, 0xF, false));
    b = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_mov_dpp(b, DPP_QUAD_2301, 0xF, 0xF, false));
    b = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_mov_dpp(b, DPP_ROW_ROR4, 0xF, 0xF, false));
    b = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_mov_dpp(b, DPP_ROW_ROR8, 0xF, 0xF, false));
    b = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_mov_dpp(b, DPP_ROW_BCAST15, 0xA, 0xF, false));
    b = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_mov_dpp(b, DPP_ROW_BCAST31, 0xC, 0xF, false));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

}  // namespace d3

#include "d3_internal.h"

namespace d3 {

constexpr int IMG_LDS = 128;   // image translations cached in LDS

__device__ __forceinline__ int zbits(double w) { return __double2loint(w); }

// the value of the first lane of this lane's row
__device__ __forceinline__ double row_first(double v)
{
    const int src = (int)(threadIdx.x & (WAVE - 16));
    const int lo = __shfl(__double2loint(v), src, WAVE);
    const int hi = __shfl(__double2hiint(v), src, WAVE);
    return __hiloint2double(hi, lo);
}

// logical workgroup index: logical blocks [x G/8, (x+1) G/8) run on XCD x
// (workgroups are dispatched round-robin over the 8 XCDs)
__device__ __forceinline__ int xcd_block()
{
    const int g = gridDim.x, b = blockIdx.x;
    return (b & 7) * (g >> 3) + (b >> 3);
}

// Atoms of one wave in the per-atom passes: the atoms are cut into 8
// contiguous slabs, one per XCD; inside a slab the XCD's waves take atoms
// round-robin, so the atoms in flight on one XCD at any moment form a
// compact window whose neighbours stay in that XCD's L2.
struct Walk {
    int first, step, end;
};

__device__ __forceinline__ Walk atom_walk(int n)
{
    const int per = gridDim.x >> 3;
    const int lb = xcd_block();
    const int x = lb / per;
    const int v = (lb - x * per) * WAVES_PER_BLOCK + (int)(threadIdx.x / WAVE);
    const int s0 = (int)((long long)n * x / 8), s1 = (int)((long long)n * (x + 1) / 8);
    Walk wk;
    wk.first = __builtin_amdgcn_readfirstlane(s0 + v);
    wk.step = per * WAVES_PER_BLOCK;
    wk.end = __builtin_amdgcn_readfirstlane(s1);
    return wk;
}

// image translation k from LDS (IN_LDS) or global memory
template <bool IN_LDS>
__device__ __forceinline__ double4 image(const double4* s_img, const double4* __restrict__ img_tab,
                                         uint32_t k)
{
    if constexpr (IN_LDS) return s_img[k];
    else return img_tab[k];
}

template <bool IN_LDS>
__device__ __forceinline__ void load_images(double4* s_img, const double4* __restrict__ img_tab,
                                            int n_img)
{
    if constexpr (IN_LDS)
        for (int k = threadIdx.x; k < n_img; k += blockDim.x) s_img[k] = img_tab[k];
}

// list code k of an atom's row (cap entries), 0 beyond the count: a load
// with a valid address in every lane, so loads need no branch
__device__ __forceinline__ uint32_t list_code(const uint32_t* __restrict__ row, int k, int cnt,
                                              int cap)
{
    const uint32_t c = row[k < cap ? k : cap - 1];
    return k < cnt ? c : 0u;
}

// Fixed-order reduction of the waves' partial sums of one workgroup:
// vals[0..6] per lane -> part[logical block * 8 + c].
__device__ __forceinline__ void block_partials(const double* vals, double* __restrict__ part)
{
    __shared__ double red[WAVES_PER_BLOCK][8];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    double t[7];
#pragma unroll
    for (int c = 0; c < 7; c++) t[c] = vals[c];
    wave_sums(t);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < 7; c++) red[wv][c] = t[c];
    __syncthreads();
    if (threadIdx.x < 7) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < WAVES_PER_BLOCK; w++) t += red[w][threadIdx.x];
        part[(size_t)xcd_block() * 8 + threadIdx.x] = t;
    }
}

__device__ __forceinline__ void virial_add(double* v, double h, double dx, double dy, double dz)
{
    const double hx = h * dx, hy = h * dy;
    v[0] = fma(hx, dx, v[0]);
    v[1] = fma(hx, dy, v[1]);
    v[2] = fma(hx, dz, v[2]);
    v[3] = fma(hy, dy, v[3]);
    v[4] = fma(hy, dz, v[4]);
    v[5] = fma(h * dz, dz, v[5]);
}

}  // namespace d3
