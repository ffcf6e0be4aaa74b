// The chain pass through the coordination numbers (the many-body part of
// Eqs. 5-7): per entry within R_cn, F_i += (G_i + G_j) f'(r) r_vec / r and
// the matching virial, with f the counting function of Eq. 4 and
// G = dE/dn from the dispersion pass; then the total force (and, if asked,
// the per-atom virial and heat current of Eqs. 7-8) is written in the
// caller's atom order.  The energy (Eq. 1) and virial totals are
// summed afterwards from the workgroup partials of both passes in a fixed
// order.
#include "d3_device.h"

namespace d3 {

constexpr int ROW = 16;  // lanes per atom: four atoms per wave, one per DPP row

// AV: also each atom's virial (Eq. 7): the chain part of its entries added
// to the direct part Vp from the dispersion pass, written as a 3x3 tensor
// in the caller's order, and if heat_current is set the heat current of
// Eq. 8, J_i = W_i v_i, with v in the caller's order.
template <bool F32, bool IMG, bool AV>
__global__ void __launch_bounds__(BLOCK)
k_chain(int n, const double4* __restrict__ pos_s, const double4* __restrict__ img_tab, int n_img,
        int img_bits, const uint32_t* __restrict__ list_c, const int* __restrict__ cnt_c,
        int cap_c, const ElemTab* __restrict__ tab, double rc2, const double* __restrict__ G,
        const double* __restrict__ Fp, const double* __restrict__ U, const int* __restrict__ perm,
        double* __restrict__ forces, double* __restrict__ atom_energy, const double* __restrict__ Vp,
        const double* __restrict__ vel, double* __restrict__ atom_virial,
        double* __restrict__ heat_current, int accumulate, double* __restrict__ part)
{
    __shared__ double4 s_img[IMG ? IMG_LDS : 1];
    __shared__ double s_rcov[MAXELEM];
    load_images<IMG>(s_img, img_tab, n_img);
    if (threadIdx.x < MAXELEM) s_rcov[threadIdx.x] = tab->rcov[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1);
    const int rl = lane & (ROW - 1);  // lane within the row
    const uint32_t img_mask = (1u << img_bits) - 1u;
    double vir[6] = {0, 0, 0, 0, 0, 0};
    const int ngroups = (n + WAVE / ROW - 1) / (WAVE / ROW);
    const Walk wk = atom_walk(ngroups);
    for (int gi_ = wk.first; gi_ < wk.end; gi_ += wk.step) {
        const int i0 = gi_ * (WAVE / ROW) + lane / ROW;
        const bool live = i0 < n;
        const int i = live ? i0 : n - 1;
        const double4 pi = pos_s[i];
        const int zi = zbits(pi.w);
        const double rci = s_rcov[zi];
        const double gi = G[i];
        const int cnt = live ? min(cnt_c[i], cap_c) : 0;
        const uint32_t* lc = list_c + (size_t)i * cap_c;
        // steps: the longest of the four lists
        int mc = max(cnt, __shfl_xor(cnt, ROW, WAVE));
        mc = __builtin_amdgcn_readfirstlane(max(mc, __shfl_xor(mc, 2 * ROW, WAVE)));
        double fx = 0.0, fy = 0.0, fz = 0.0;
        double av[6] = {0, 0, 0, 0, 0, 0};  // this atom's chain virial (AV only)
        for (int k0 = 0; k0 < mc; k0 += ROW) {
            const int k = k0 + rl;
            const uint32_t code = list_code(lc, k, cnt, cap_c);
            const uint32_t j = code >> img_bits;
            const double4 pj = pos_s[j];
            const double gj = G[j];
            const double4 T = image<IMG>(s_img, img_tab, code & img_mask);
            const double dx = pj.x + T.x - pi.x;
            const double dy = pj.y + T.y - pi.y;
            const double dz = pj.z + T.z - pi.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const bool in = k < cnt && r2 < rc2;
            const double rs = rci + s_rcov[zbits(pj.w)];
            const double gs = in ? gi + gj : 0.0;
            if (F32) {
                // masked lanes may see r = 0: keep their factor finite
                const float q2 = in ? (float)r2 : 1.0f;
                const float r = __fsqrt_rn(q2);
                const float e = __expf(-16.0f * ((float)rs * __frcp_rn(r) - 1.0f));
                const float ope = 1.0f + e;
                // f'(r)/r = -16 Rs e / (r^3 (1+e)^2)
                const float dfr = -16.0f * (float)rs * e * __frcp_rn(q2 * r * ope * ope);
                const float coef = (float)gs * dfr;
                const float x = (float)dx, y = (float)dy, zz = (float)dz;
                fx += (double)(coef * x);
                fy += (double)(coef * y);
                fz += (double)(coef * zz);
                const float h = -0.5f * coef;
                const float hx = h * x, hy = h * y;
                vir[0] += (double)(hx * x);
                vir[1] += (double)(hx * y);
                vir[2] += (double)(hx * zz);
                vir[3] += (double)(hy * y);
                vir[4] += (double)(hy * zz);
                vir[5] += (double)(h * zz * zz);
                if constexpr (AV) {
                    av[0] += (double)(hx * x);
                    av[1] += (double)(hx * y);
                    av[2] += (double)(hx * zz);
                    av[3] += (double)(hy * y);
                    av[4] += (double)(hy * zz);
                    av[5] += (double)(h * zz * zz);
                }
            } else {
                const double q2 = in ? r2 : 1.0;
                const double r = sqrt(q2);
                const double e = exp(-16.0 * (rs / r - 1.0));
                const double ope = 1.0 + e;
                const double coef = gs * (-16.0 * rs * e / (q2 * r * ope * ope));
                fx = fma(coef, dx, fx);
                fy = fma(coef, dy, fy);
                fz = fma(coef, dz, fz);
                virial_add(vir, -0.5 * coef, dx, dy, dz);
                if constexpr (AV) virial_add(av, -0.5 * coef, dx, dy, dz);
            }
        }
        fx = row_sum(fx);
        fy = row_sum(fy);
        fz = row_sum(fz);
        if constexpr (AV) {
#pragma unroll
            for (int c = 0; c < 6; c++) av[c] = row_sum(av[c]);
        }
        if (live && rl == 0) {
            const size_t o = (size_t)perm[i];
            const double f0 = Fp[3 * (size_t)i] + fx;
            const double f1 = Fp[3 * (size_t)i + 1] + fy;
            const double f2 = Fp[3 * (size_t)i + 2] + fz;
            if (forces) {
                if (accumulate) {
                    forces[3 * o] += f0;
                    forces[3 * o + 1] += f1;
                    forces[3 * o + 2] += f2;
                } else {
                    forces[3 * o] = f0;
                    forces[3 * o + 1] = f1;
                    forces[3 * o + 2] = f2;
                }
            }
            if (atom_energy) {
                if (accumulate) atom_energy[o] += U[i];
                else atom_energy[o] = U[i];
            }
            if constexpr (AV) {
                double t[6];
#pragma unroll
                for (int c = 0; c < 6; c++) t[c] = Vp[6 * (size_t)i + c] + av[c];
                // symmetric: xx xy xz yy yz zz
                const double m[9] = {t[0], t[1], t[2], t[1], t[3], t[4], t[2], t[4], t[5]};
                if (atom_virial) {
                    double* wo = atom_virial + 9 * o;
#pragma unroll
                    for (int c = 0; c < 9; c++) wo[c] = accumulate ? wo[c] + m[c] : m[c];
                }
                if (heat_current) {
                    const double v0 = vel[3 * o], v1 = vel[3 * o + 1], v2 = vel[3 * o + 2];
                    const double j[3] = {m[0] * v0 + m[1] * v1 + m[2] * v2,
                                         m[3] * v0 + m[4] * v1 + m[5] * v2,
                                         m[6] * v0 + m[7] * v1 + m[8] * v2};
                    double* jo = heat_current + 3 * o;
#pragma unroll
                    for (int c = 0; c < 3; c++) jo[c] = accumulate ? jo[c] + j[c] : j[c];
                }
            }
        }
    }
    const double vals[7] = {0.0, vir[0], vir[1], vir[2], vir[3], vir[4], vir[5]};
    block_partials(vals, part);
}

// Energy (Eq. 1) and virial from the workgroup partials of the passes
// (dispersion a, chain b, and the three-body pass c when nc > 0), summed in
// a fixed order by one workgroup.
__global__ void __launch_bounds__(1024)
k_final(int na, const double* __restrict__ part_a, int nb, const double* __restrict__ part_b,
        int nc, const double* __restrict__ part_c, double* __restrict__ energy,
        double* __restrict__ virial, int accumulate)
{
    __shared__ double fin[1024 / WAVE][8];
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    const int nmax = na > nb ? na : nb;
    // four rows of partials per thread and pass, loaded before any is used;
    // rows past a pass's count load its last row and are weighted by zero
    for (int b0 = threadIdx.x; b0 < nmax; b0 += 4 * 1024) {
        double4 a0[4], a1[4], c0[4], c1[4];
        double sa[4], sb[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int b = b0 + r * 1024;
            const int ba = b < na ? b : na - 1, bb = b < nb ? b : nb - 1;
            sa[r] = b < na ? 1.0 : 0.0;
            sb[r] = b < nb ? 1.0 : 0.0;
            const double4* pa = (const double4*)(part_a + (size_t)ba * 8);
            const double4* pb = (const double4*)(part_b + (size_t)bb * 8);
            a0[r] = pa[0];
            a1[r] = pa[1];
            c0[r] = pb[0];
            c1[r] = pb[1];
        }
#pragma unroll
        for (int r = 0; r < 4; r++) {
            acc[0] += sa[r] * a0[r].x + sb[r] * c0[r].x;
            acc[1] += sa[r] * a0[r].y + sb[r] * c0[r].y;
            acc[2] += sa[r] * a0[r].z + sb[r] * c0[r].z;
            acc[3] += sa[r] * a0[r].w + sb[r] * c0[r].w;
            acc[4] += sa[r] * a1[r].x + sb[r] * c1[r].x;
            acc[5] += sa[r] * a1[r].y + sb[r] * c1[r].y;
            acc[6] += sa[r] * a1[r].z + sb[r] * c1[r].z;
        }
    }
    for (int b = threadIdx.x; b < nc; b += 1024) {
        const double4* p = (const double4*)(part_c + (size_t)b * 8);
        const double4 x0 = p[0], x1 = p[1];
        acc[0] += x0.x;
        acc[1] += x0.y;
        acc[2] += x0.z;
        acc[3] += x0.w;
        acc[4] += x1.x;
        acc[5] += x1.y;
        acc[6] += x1.z;
    }
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    wave_sums(acc);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < 7; c++) fin[wv][c] = acc[c];
    __syncthreads();
    if (threadIdx.x < 7) {
        double t = 0.0;
        for (int w = 0; w < 1024 / WAVE; w++) t += fin[w][threadIdx.x];
        fin[0][threadIdx.x] = t;  // wave 0 is the only reader below
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double* f = fin[0];
        const double e = f[0];
        const double v[9] = {f[1], f[2], f[3], f[2], f[4], f[5], f[3], f[5], f[6]};
        if (accumulate) {
            energy[0] += e;
            if (virial)
                for (int c = 0; c < 9; c++) virial[c] += v[c];
        } else {
            energy[0] = e;
            if (virial)
                for (int c = 0; c < 9; c++) virial[c] = v[c];
        }
    }
}

__global__ void __launch_bounds__(BLOCK)
k_scatter_out(int n, const double* __restrict__ src, const int* __restrict__ perm,
              double* __restrict__ dst)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[perm[k]] = src[k];
}

int launch_chain(int mode, int n, const double4* pos_s, const double4* img_tab, int n_img,
                 int img_bits, const uint32_t* list_c, const int* cnt_c, int cap_c,
                 const ElemTab* tab, double rc2, const double* G, const double* Fp,
                 const double* U, const int* perm, double* forces, double* atom_energy,
                 const double* Vp, const double* vel, double* atom_virial, double* heat_current,
                 int accumulate, double* part, hipStream_t s)
{
    if (n <= 0) return 0;
    const int groups = (n + WAVE / ROW - 1) / (WAVE / ROW);
    const bool lds = n_img <= IMG_LDS;
    int nblk = 0;
#define D3_CHAIN(F, I, A)                                                                       \
    {                                                                                           \
        nblk = pass_blocks((const void*)&k_chain<F, I, A>, groups);                             \
        hipLaunchKernelGGL((k_chain<F, I, A>), dim3(nblk), dim3(BLOCK), 0, s, n, pos_s,         \
                           img_tab, n_img, img_bits, list_c, cnt_c, cap_c, tab, rc2, G, Fp, U,  \
                           perm, forces, atom_energy, Vp, vel, atom_virial, heat_current,      \
                           accumulate, part);                                                   \
    }
    const bool prec = mode == D3_MODE_PREC_F32;
    if (Vp) {
        if (prec) {
            if (lds) D3_CHAIN(true, true, true)
            else D3_CHAIN(true, false, true)
        } else {
            if (lds) D3_CHAIN(false, true, true)
            else D3_CHAIN(false, false, true)
        }
    } else {
        if (prec) {
            if (lds) D3_CHAIN(true, true, false)
            else D3_CHAIN(true, false, false)
        } else {
            if (lds) D3_CHAIN(false, true, false)
            else D3_CHAIN(false, false, false)
        }
    }
#undef D3_CHAIN
    return nblk;
}

void launch_final(int na, const double* part_a, int nb, const double* part_b, int nc,
                  const double* part_c, double* energy, double* virial, int accumulate,
                  hipStream_t s)
{
    hipLaunchKernelGGL(k_final, dim3(1), dim3(1024), 0, s, na, part_a, nb, part_b, nc, part_c,
                       energy, virial, accumulate);
}

void launch_scatter_out(int n, const double* src, const int* perm, double* dst, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scatter_out, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, n, src,
                       perm, dst);
}

}  // namespace d3
