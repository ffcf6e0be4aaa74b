// Coordination numbers (Eq. 4) and the normalised Gaussian weights of
// Eq. 3 for every atom.
//
// One wavefront treats one atom at a time: its lanes walk the atom's
// R_cn list (one 64-entry chunk covers a typical list), the counting
// function is summed with a DPP wave reduction, and the weights
// w_a = L_a / sum_b L_b, L_a = exp(-4 (n - n_ref,a)^2 + shift), with the
// largest exponent shifted to zero (an exact identity that keeps the sums
// representable), and their CN derivatives w'_a are formed in FP64 in
// every mode.
#include "d3_device.h"

namespace d3 {

template <bool F32, bool IMG>
__global__ void __launch_bounds__(BLOCK)
k_cn(int n, const double4* __restrict__ pos_s, const double4* __restrict__ img_tab, int n_img,
     int img_bits, const uint32_t* __restrict__ list_c, const int* __restrict__ cnt_c, int cap_c,
     const ElemTab* __restrict__ tab, double rc2, double* __restrict__ cn, double* __restrict__ w,
     double* __restrict__ wd, double* __restrict__ W, float* __restrict__ Wf)
{
    __shared__ double4 s_img[IMG ? IMG_LDS : 1];
    __shared__ double s_rcov[MAXELEM];
    load_images<IMG>(s_img, img_tab, n_img);
    if (threadIdx.x < MAXELEM) s_rcov[threadIdx.x] = tab->rcov[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1);
    const uint32_t img_mask = (1u << img_bits) - 1u;
    const Walk wk = atom_walk(n);
    for (int i = wk.first; i < wk.end; i += wk.step) {
        const double4 pi = pos_s[i];
        const int zi = __builtin_amdgcn_readfirstlane(zbits(pi.w));
        const double rci = s_rcov[zi];
        const int cnt = min(cnt_c[i], cap_c);
        const uint32_t* lc = list_c + (size_t)i * cap_c;
        double sum = 0.0;
        for (int k0 = 0; k0 < cnt; k0 += WAVE) {
            const int k = k0 + lane;
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
        const double ni = wave_sum(sum);
        // Gaussian weights of Eq. 3 for atom i, normalised after shifting
        // every exponent by the largest one (FP64 in every mode)
        const int K = tab->n_ref[zi];
        double dl[MAXREF], wl[MAXREF], wdl[MAXREF];
        double m = 1e300;
#pragma unroll
        for (int a = 0; a < MAXREF; a++) {
            dl[a] = ni - tab->cn_ref[zi * MAXREF + a];
            if (a < K) m = fmin(m, dl[a] * dl[a]);
        }
        double z = 0.0;
#pragma unroll
        for (int a = 0; a < MAXREF; a++) {
            wl[a] = (a < K) ? exp(-4.0 * (dl[a] * dl[a] - m)) : 0.0;
            z += wl[a];
        }
        const double iz = 1.0 / z;
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < MAXREF; a++) {
            wl[a] *= iz;
            s += wl[a] * dl[a];
        }
#pragma unroll
        for (int a = 0; a < MAXREF; a++) wdl[a] = (a < K) ? -8.0 * wl[a] * (dl[a] - s) : 0.0;
        if (lane == 0) cn[i] = ni;
        if (lane < 8) {
            double wv = 0.0, wdv = 0.0;
#pragma unroll
            for (int a = 0; a < MAXREF; a++)
                if (lane == a) {
                    wv = wl[a];
                    wdv = wdl[a];
                }
            if (lane < MAXREF) {
                w[(size_t)i * MAXREF + lane] = wv;
                wd[(size_t)i * MAXREF + lane] = wdv;
            }
            if (F32) Wf[(size_t)i * WROWF + lane] = (float)wv;
            else if (lane < WROW) W[(size_t)i * WROW + lane] = wv;
        }
    }
}

void launch_cn(int mode, int n, const double4* pos_s, const double4* img_tab, int n_img,
               int img_bits, const uint32_t* list_c, const int* cnt_c, int cap_c,
               const ElemTab* tab, double rc2, double* cn, double* w, double* wd, double* W,
               float* Wf, hipStream_t s)
{
    if (n <= 0) return;
    const dim3 grid(split_blocks(n)), block(BLOCK);
    const bool lds = n_img <= IMG_LDS;
#define D3_CN(F, I)                                                                          \
    hipLaunchKernelGGL((k_cn<F, I>), grid, block, 0, s, n, pos_s, img_tab, n_img, img_bits,  \
                       list_c, cnt_c, cap_c, tab, rc2, cn, w, wd, W, Wf)
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
