// Coordination numbers (Eq. 4) and the normalised Gaussian weights of
// Eq. 3 for every atom.
//
// One wavefront treats four atoms at a time, one per DPP row of 16 lanes:
// a row walks its atom's R_cn list 16 entries per step and sums the
// counting function with a row reduction.  The weights
// w_a = L_a / sum_b L_b, L_a = exp(-4 (n - n_ref,a)^2 + shift), with the
// largest exponent shifted to zero (an exact identity that keeps the sums
// representable), and their CN derivatives w'_a are then formed by the
// row's first K lanes, one reference each, in FP64 in every mode.
#include "d3_device.h"

namespace d3 {

constexpr int ROW = 16;  // lanes per atom

template <bool F32, bool IMG>
__global__ void __launch_bounds__(BLOCK)
k_cn(int n, const double4* __restrict__ pos_s, const double4* __restrict__ img_tab, int n_img,
     int img_bits, const uint32_t* __restrict__ list_c, const int* __restrict__ cnt_c, int cap_c,
     const ElemTab* __restrict__ tab, double rc2, double* __restrict__ cn, double* __restrict__ w,
     double* __restrict__ wd, double* __restrict__ W, float* __restrict__ Wf)
{
    __shared__ double4 s_img[IMG ? IMG_LDS : 1];
    __shared__ double s_rcov[MAXELEM];
    __shared__ double s_cnref[MAXELEM * MAXREF];
    __shared__ int s_nref[MAXELEM];
    load_images<IMG>(s_img, img_tab, n_img);
    if (threadIdx.x < MAXELEM) {
        s_rcov[threadIdx.x] = tab->rcov[threadIdx.x];
        s_nref[threadIdx.x] = tab->n_ref[threadIdx.x];
    }
    if (threadIdx.x < MAXELEM * MAXREF) s_cnref[threadIdx.x] = tab->cn_ref[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1);
    const int rl = lane & (ROW - 1);  // lane within the row
    const uint32_t img_mask = (1u << img_bits) - 1u;
    const int ngroups = (n + WAVE / ROW - 1) / (WAVE / ROW);
    const Walk wk = atom_walk(ngroups);
    for (int gi = wk.first; gi < wk.end; gi += wk.step) {
        const int i = gi * (WAVE / ROW) + lane / ROW;
        const bool live = i < n;
        const int ic = live ? i : n - 1;
        const double4 pi = pos_s[ic];
        const int zi = zbits(pi.w);
        const double rci = s_rcov[zi];
        const int cnt = live ? min(cnt_c[ic], cap_c) : 0;
        const uint32_t* lc = list_c + (size_t)ic * cap_c;
        // steps: the longest of the four lists
        int mc = max(cnt, __shfl_xor(cnt, ROW, WAVE));
        mc = __builtin_amdgcn_readfirstlane(max(mc, __shfl_xor(mc, 2 * ROW, WAVE)));
        double sum = 0.0;
        for (int k0 = 0; k0 < mc; k0 += ROW) {
            const int k = k0 + rl;
            const uint32_t code = list_code(lc, k, cnt, cap_c);
            const double4 pj = pos_s[code >> img_bits];
            const double4 T = image<IMG>(s_img, img_tab, code & img_mask);
            const double dx = pj.x + T.x - pi.x;
            const double dy = pj.y + T.y - pi.y;
            const double dz = pj.z + T.z - pi.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const bool in = k < cnt && r2 < rc2;
            const double rs = rci + s_rcov[zbits(pj.w)];
            double f;
            if (F32) {
                const float r = __fsqrt_rn((float)r2);
                const float e = __expf(-16.0f * ((float)rs * __frcp_rn(r) - 1.0f));
                f = (double)__frcp_rn(1.0f + e);
            } else {
                const double r = sqrt(r2);
                const double e = exp(-16.0 * (rs / r - 1.0));
                f = 1.0 / (1.0 + e);
            }
            sum += in ? f : 0.0;
        }
        const double ni = row_first(row_sum(sum));
        // Gaussian weights of Eq. 3: lane a < K of the row takes reference a
        const int K = s_nref[zi];
        const bool ref = rl < K;
        const double dl = ni - s_cnref[zi * MAXREF + (rl < MAXREF ? rl : MAXREF - 1)];
        const double m = row_min(ref ? dl * dl : 1e300);
        const double L = ref ? exp(-4.0 * (dl * dl - m)) : 0.0;
        const double wl = L / row_first(row_sum(L));
        const double s = row_first(row_sum(wl * dl));
        const double wdl = ref ? -8.0 * wl * (dl - s) : 0.0;
        if (live) {
            if (rl == 0) cn[i] = ni;
            if (rl < MAXREF) {
                w[(size_t)i * MAXREF + rl] = wl;
                wd[(size_t)i * MAXREF + rl] = wdl;
            }
            // the atom's pieces for the dispersion pass: lanes 0..4 the
            // weights, lanes 5..7 the position, lane 8 (FP32) the species
            const double pv = rl == 5 ? pi.x : (rl == 6 ? pi.y : pi.z);
            if (F32) {
                float* p0 = Wf + piece_at(NPIECEF, PBLKF, 0, i) * 4;  // x, y
                float* p1 = Wf + piece_at(NPIECEF, PBLKF, 1, i) * 4;  // z, w0, w1
                float* p2 = Wf + piece_at(NPIECEF, PBLKF, 2, i) * 4;  // w2, w3, w4, species
                if (rl < 2) p1[2 + rl] = (float)wl;
                else if (rl < MAXREF) p2[rl - 2] = (float)wl;
                else if (rl < 7) ((double*)p0)[rl - 5] = pv;
                else if (rl == 7) *(double*)p1 = pv;
                else if (rl == 8) ((int*)p2)[3] = zi;
            } else {
                // slot (x, y, z, w0..w4 = 0..7) is double slot % 4 of piece slot / 4
                const int slot = rl < MAXREF ? 3 + rl : rl - 5;
                const double v = rl < MAXREF ? (((zi >> rl) & 1) && rl < 4 ? -wl : wl) : pv;
                if (rl < 8) W[piece_at(NPIECE, PBLK, slot >> 2, i) * 4 + (slot & 3)] = v;
            }
        }
    }
}

void launch_cn(int mode, int n, const double4* pos_s, const double4* img_tab, int n_img,
               int img_bits, const uint32_t* list_c, const int* cnt_c, int cap_c,
               const ElemTab* tab, double rc2, double* cn, double* w, double* wd, double* W,
               float* Wf, hipStream_t s)
{
    if (n <= 0) return;
    const int groups = (n + WAVE / ROW - 1) / (WAVE / ROW);
    const bool lds = n_img <= IMG_LDS;
#define D3_CN(F, I)                                                                             \
    hipLaunchKernelGGL((k_cn<F, I>), dim3(pass_blocks((const void*)&k_cn<F, I>, groups)),       \
                       dim3(BLOCK), 0, s, n, pos_s, img_tab, n_img, img_bits, list_c, cnt_c,    \
                       cap_c, tab, rc2, cn, w, wd, W, Wf)
    if (mode == D3_MODE_PREC_F32) {
        if (lds) D3_CN(true, true);
        else D3_CN(true, false);
    } else {
        if (lds) D3_CN(false, true);
        else D3_CN(false, false);
    }
#undef D3_CN
}

}  // namespace d3
