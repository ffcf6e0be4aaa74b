// The three-body (Axilrod-Teller-Muto) term of D3, the variant the paper
// names and sets aside (Sec. II A, before Eq. 1), as defined by the D3
// reference it cites (Grimme et al., J. Chem. Phys. 132, 154104 (2010)):
// over every triangle of atom images whose three sides are below r_atm,
//   E_ABC = s9 sqrt(C6_AB C6_BC C6_CA) (1 + 3 cos A cos B cos C)
//           / (r_AB r_BC r_CA)^3 f3,
//   f3 = 1 / (1 + 6 (rbar / (4/3 R0bar))^-16),
// rbar and R0bar the geometric means of the three sides and of the three
// pair radii R0 = sqrt(3 r2r4 r2r4), each C6 from Eq. 3 at the atoms'
// coordination numbers.  With squared sides a = r_AB^2, b = r_BC^2,
// c = r_CA^2 the cosine product is (a + c - b)(a + b - c)(b + c - a) / (8abc)
// (law of cosines), so E is a function of a, b, c and the three C6.
//
// One wavefront treats one atom A: its lanes walk the pairs (B, C) of A's
// R_cn-list entries (r_atm <= R_cn), 64 pairs per step, decoding a pair
// index into its two entries.  A triangle is found once from each of its
// vertices; atom A takes a third of its energy and virial, its whole force
// on A, -dE/dr_A = 2 dE/da d_AB + 2 dE/dc d_AC (d the vectors from A), and
// dE/dn_A = E/2 (dC6_AB/dn_A / C6_AB + dC6_AC/dn_A / C6_AC), which the chain
// pass turns into forces like the two-body dE/dn.  Every sum is gathered
// onto A: no atomics.  FP64 in every mode, with C6 from the factorised
// weights (exact Eq. 3) also in the surrogate mode.
#include "d3_device.h"

namespace d3 {

constexpr int ATM_M_LDS_ELEM = 8;  // C6 reference table in LDS up to 8 elements
constexpr double ATM_SR3 = 4.0 / 3.0;

__device__ __forceinline__ double atm_recip(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// geometry and damping of one triangle: returns g = (1 + 3 cosA cosB cosC)
// / (abc)^(3/2) f3 and its derivatives in the squared sides a, b, c
struct AtmG {
    double g, ga, gb, gc;
};
__device__ __forceinline__ AtmG atm_geometry(double a, double b, double c, double r0prod)
{
    const double u = a * b * c;
    const double x = a + c - b, y = a + b - c, z = b + c - a;
    const double P = x * y * z;
    const double iu = atm_recip(u);
    const double rr = sqrt(u);                 // r_AB r_BC r_CA
    const double u15 = iu * atm_recip(rr);     // (abc)^(-3/2)
    const double ang = 1.0 + 0.375 * P * iu;
    // (rbar / (4/3 R0bar))^-16 = X^(16/3), X = (4/3)^3 R0_AB R0_BC R0_CA / (r r r)
    const double X = ATM_SR3 * ATM_SR3 * ATM_SR3 * r0prod * atm_recip(rr);
    const double X2 = X * X;
    const double q = X2 * X2 * X * cbrt(X);
    const double f3 = atm_recip(1.0 + 6.0 * q);
    const double dP[3] = {y * z + x * z - x * y, x * z - y * z + x * y, y * z - x * z + x * y};
    const double du[3] = {b * c, a * c, a * b};
    double d[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const double dang = 0.375 * (dP[k] - P * du[k] * iu) * iu;
        const double dlog = du[k] * iu;  // d(log u)
        // d(u^-3/2) = -3/2 u^-3/2 dlog;  df3 = 16 f3^2 q dlog
        d[k] = u15 * f3 * (dang + ang * dlog * (16.0 * f3 * q - 1.5));
    }
    AtmG o;
    o.g = ang * u15 * f3;
    o.ga = d[0];
    o.gb = d[1];
    o.gc = d[2];
    return o;
}

// the pair index p of the strict upper triangle, enumerated as
// (0,1), (0,2), (1,2), (0,3), ...: entries e1 < e2 with p = e2 (e2-1)/2 + e1
__device__ __forceinline__ void pair_of(int p, int& e1, int& e2)
{
    int t = (int)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
    if (t * (t - 1) / 2 > p) t--;
    if ((t + 1) * t / 2 <= p) t++;
    e2 = t;
    e1 = p - t * (t - 1) / 2;
}

template <bool IMG, bool AV>
__global__ void __launch_bounds__(BLOCK)
k_atm(int n, const double4* __restrict__ pos_s, const double4* __restrict__ img_tab, int n_img,
      int img_bits, const uint32_t* __restrict__ list_c, const int* __restrict__ cnt_c, int cap_c,
      const ElemTab* __restrict__ tab, const double* __restrict__ c6ref,
      const double4* __restrict__ pc, double s9, double ra2, const double* __restrict__ w,
      const double* __restrict__ wd, double* __restrict__ Fp, double* __restrict__ U,
      double* __restrict__ G, double* __restrict__ Vp, double* __restrict__ part)
{
    __shared__ double4 s_img[IMG ? IMG_LDS : 1];
    __shared__ double s_r0[MAXELEM * MAXELEM];
    __shared__ double s_M[ATM_M_LDS_ELEM * ATM_M_LDS_ELEM * MAXREF * MAXREF];
    __shared__ double s_u[WAVES_PER_BLOCK][2][MAXELEM * MAXREF];
    const int ne = tab->n_elem;
    const bool m_lds = ne <= ATM_M_LDS_ELEM;
    load_images<IMG>(s_img, img_tab, n_img);
    for (int k = threadIdx.x; k < MAXELEM * MAXELEM; k += blockDim.x) s_r0[k] = sqrt(pc[k].z);
    if (m_lds)
        for (int k = threadIdx.x; k < ne * ne * MAXREF * MAXREF; k += blockDim.x) {
            const int e = k / (ne * MAXREF * MAXREF), r = k - e * ne * MAXREF * MAXREF;
            s_M[k] = c6ref[(size_t)e * MAXELEM * MAXREF * MAXREF + r];
        }
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const uint32_t img_mask = (1u << img_bits) - 1u;
    const double* u = &s_u[wv][0][0];
    const double* ud = &s_u[wv][1][0];
    double vir[6] = {0, 0, 0, 0, 0, 0};
    double esum = 0.0;
    const Walk wk = atom_walk(n);
    for (int i = wk.first; i < wk.end; i += wk.step) {
        const double4 pi = pos_s[i];
        const int zi = __builtin_amdgcn_readfirstlane(zbits(pi.w));
        const int cnt = min(cnt_c[i], cap_c);
        const uint32_t* lc = list_c + (size_t)i * cap_c;
        // u_f = w_A^T M[zA][f], u'_f = w_A'^T M[zA][f] (this wave's LDS rows)
        for (int idx = lane; idx < 2 * ne * MAXREF; idx += WAVE) {
            const int which = idx >= ne * MAXREF ? 1 : 0;
            const int q = idx - which * ne * MAXREF;
            const int f = q / MAXREF, b = q - f * MAXREF;
            double v = 0.0;
#pragma unroll
            for (int a = 0; a < MAXREF; a++) {
                const double mab = m_lds ? s_M[((zi * ne + f) * MAXREF + a) * MAXREF + b]
                                         : c6ref[((size_t)(zi * MAXELEM + f) * MAXREF + a) * MAXREF + b];
                v = fma(which ? wd[(size_t)i * MAXREF + a] : w[(size_t)i * MAXREF + a], mab, v);
            }
            s_u[wv][which][q] = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int npair = cnt * (cnt - 1) / 2;
        double fx = 0.0, fy = 0.0, fz = 0.0, ue = 0.0, g = 0.0;
        double av[6] = {0, 0, 0, 0, 0, 0};
        for (int p0 = 0; p0 < npair; p0 += WAVE) {
            const int p = p0 + lane;
            int e1 = 0, e2 = 1;
            if (p < npair) pair_of(p, e1, e2);
            const uint32_t k1 = list_code(lc, e1, cnt, cap_c), k2 = list_code(lc, e2, cnt, cap_c);
            const uint32_t j1 = k1 >> img_bits, j2 = k2 >> img_bits;
            const double4 pb = pos_s[j1], pcc = pos_s[j2];
            const double4 T1 = image<IMG>(s_img, img_tab, k1 & img_mask);
            const double4 T2 = image<IMG>(s_img, img_tab, k2 & img_mask);
            const double d1x = pb.x + T1.x - pi.x, d1y = pb.y + T1.y - pi.y, d1z = pb.z + T1.z - pi.z;
            const double d2x = pcc.x + T2.x - pi.x, d2y = pcc.y + T2.y - pi.y,
                         d2z = pcc.z + T2.z - pi.z;
            const double bx = d2x - d1x, by = d2y - d1y, bz = d2z - d1z;
            double a = d1x * d1x + d1y * d1y + d1z * d1z;
            double c = d2x * d2x + d2y * d2y + d2z * d2z;
            double b = bx * bx + by * by + bz * bz;
            const bool in = p < npair && a < ra2 && b < ra2 && c < ra2;
            // masked lanes evaluate a harmless unit triangle
            a = in ? a : 1.0;
            b = in ? b : 1.0;
            c = in ? c : 1.0;
            const int zb = zbits(pb.w), zc = zbits(pcc.w);
            double wb[MAXREF], wc[MAXREF];
#pragma unroll
            for (int r = 0; r < MAXREF; r++) {
                wb[r] = w[(size_t)j1 * MAXREF + r];
                wc[r] = w[(size_t)j2 * MAXREF + r];
            }
            double cab = 0.0, dab = 0.0, cac = 0.0, dac = 0.0, cbc = 0.0;
#pragma unroll
            for (int r = 0; r < MAXREF; r++) {
                cab = fma(u[zb * MAXREF + r], wb[r], cab);
                dab = fma(ud[zb * MAXREF + r], wb[r], dab);
                cac = fma(u[zc * MAXREF + r], wc[r], cac);
                dac = fma(ud[zc * MAXREF + r], wc[r], dac);
            }
#pragma unroll
            for (int ra = 0; ra < MAXREF; ra++) {
                double t = 0.0;
#pragma unroll
                for (int rb = 0; rb < MAXREF; rb++) {
                    const double mab =
                        m_lds ? s_M[((zb * ne + zc) * MAXREF + ra) * MAXREF + rb]
                              : c6ref[((size_t)(zb * MAXELEM + zc) * MAXREF + ra) * MAXREF + rb];
                    t = fma(mab, wc[rb], t);
                }
                cbc = fma(wb[ra], t, cbc);
            }
            if (!in) {
                cab = cac = cbc = 1.0;
                dab = dac = 0.0;
            }
            const double r0prod = s_r0[zi * MAXELEM + zb] * s_r0[zb * MAXELEM + zc] *
                                  s_r0[zc * MAXELEM + zi];
            const AtmG q = atm_geometry(a, b, c, r0prod);
            const double cc = in ? s9 * sqrt(cab * cbc * cac) : 0.0;
            const double E = cc * q.g;
            ue = fma(E, 1.0 / 3.0, ue);
            g = fma(0.5 * E, dab * atm_recip(cab) + dac * atm_recip(cac), g);
            const double ha = 2.0 * cc * q.ga, hc = 2.0 * cc * q.gc;
            fx += ha * d1x + hc * d2x;
            fy += ha * d1y + hc * d2y;
            fz += ha * d1z + hc * d2z;
            // a third of -2 sum over the sides of dE/d(side^2) side (x) side
            const double wa = -ha / 3.0, wbb = -2.0 * cc * q.gb / 3.0, wcc = -hc / 3.0;
            virial_add(vir, wa, d1x, d1y, d1z);
            virial_add(vir, wbb, bx, by, bz);
            virial_add(vir, wcc, d2x, d2y, d2z);
            if constexpr (AV) {
                virial_add(av, wa, d1x, d1y, d1z);
                virial_add(av, wbb, bx, by, bz);
                virial_add(av, wcc, d2x, d2y, d2z);
            }
        }
        if constexpr (AV) {
            double t[11] = {fx, fy, fz, ue, g, av[0], av[1], av[2], av[3], av[4], av[5]};
            wave_sums(t);
            fx = t[0];
            fy = t[1];
            fz = t[2];
            ue = t[3];
            g = t[4];
            if (lane == 0)
#pragma unroll
                for (int k = 0; k < 6; k++) Vp[6 * (size_t)i + k] += t[5 + k];
        } else {
            double t[5] = {fx, fy, fz, ue, g};
            wave_sums(t);
            fx = t[0];
            fy = t[1];
            fz = t[2];
            ue = t[3];
            g = t[4];
        }
        esum += ue;
        if (lane == 0) {
            Fp[3 * (size_t)i] += fx;
            Fp[3 * (size_t)i + 1] += fy;
            Fp[3 * (size_t)i + 2] += fz;
            U[i] += ue;
            G[i] += g;
        }
        // the next atom rewrites u: every lane has finished reading it
        __builtin_amdgcn_wave_barrier();
    }
    const double vals[7] = {lane == 0 ? esum : 0.0, vir[0], vir[1], vir[2], vir[3], vir[4], vir[5]};
    block_partials(vals, part);
}

int launch_atm(int n, const double4* pos_s, const double4* img_tab, int n_img, int img_bits,
               const uint32_t* list_c, const int* cnt_c, int cap_c, const ElemTab* tab,
               const double* c6ref, const double4* pc, double s9, double ra2, const double* w,
               const double* wd, double* Fp, double* U, double* G, double* Vp, double* part,
               hipStream_t s)
{
    if (n <= 0) return 0;
    const bool lds = n_img <= IMG_LDS;
    int nblk = 0;
#define D3_ATM(I, A)                                                                          \
    {                                                                                         \
        nblk = pass_blocks((const void*)&k_atm<I, A>, n);                                     \
        hipLaunchKernelGGL((k_atm<I, A>), dim3(nblk), dim3(BLOCK), 0, s, n, pos_s, img_tab,   \
                           n_img, img_bits, list_c, cnt_c, cap_c, tab, c6ref, pc, s9, ra2, w, \
                           wd, Fp, U, G, Vp, part);                                           \
    }
    if (Vp) {
        if (lds) D3_ATM(true, true)
        else D3_ATM(false, true)
    } else {
        if (lds) D3_ATM(true, false)
        else D3_ATM(false, false)
    }
#undef D3_ATM
    return nblk;
}

}  // namespace d3
