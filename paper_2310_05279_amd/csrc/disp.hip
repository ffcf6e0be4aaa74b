// The BJ-damped dispersion pass (Eq. 2): per neighbour entry within R_pot,
// C6 from Eq. 3, the direct force at fixed C6, the site energy U_i, the
// derivative G_i = dE/dn_i and the virial.
//
// One wavefront treats one atom i at a time; its 64 lanes walk i's list,
// 64 entries per step.  Every sum is a gather onto i (each unordered pair
// is evaluated from both ends), so no floating-point atomics are used and
// the results do not depend on scheduling.
//
// C6 factorises: the Gaussian weight of Eq. 3 is a product over the two
// atoms and so is its normaliser, hence C6_ij = w_i^T M_{Zi Zj} w_j with
// w the normalised per-atom weights.  When a wave takes atom i it forms in
// LDS the row vectors u_f = w_i^T M_{Zi f} and u'_f = w_i'^T M_{Zi f} for
// every element f, so a neighbour costs one gather of its position,
// species and weights (64 bytes, laid out in blocks written by the CN pass)
// and C6 = u_{Zj} . w_j, dC6/dn_i = u'_{Zj} . w_j.  The pair constants (Rd^6,
// Rd^8, s8 R0^2) of every element pair sit in LDS too.  List codes are
// fetched two chunks ahead of the arithmetic and neighbour data is handed
// on one chunk ahead (the compiler turns that hand-on into a load at the top
// of the next step, which measured faster than any way of keeping it);
// every lane loads a valid address (entries past the count read atom 0 and
// are masked), so the loads carry no branches.
//
// Precision form (D3_MODE_PREC_F32): distances and cutoff tests in FP64,
// then the pair arithmetic in FP32 (hardware rcp) on FP32 weights, with
// every per-lane and per-atom sum accumulated in FP64.
#include <type_traits>

#include "d3_device.h"

namespace d3 {

constexpr int M_LDS_ELEM = 8;  // C6 reference table staged in LDS up to 8 elements

// 1/x for the positive, normal denominators of Eq. 2 (r^6 + Rd^6 times
// r^8 + Rd^8): the hardware estimate refined by two Newton-Raphson steps
// y <- y + y (1 - x y), each written with fused multiply-adds; the result
// is within an ulp of 1/x.
__device__ __forceinline__ double recip(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// The damped pair energy of one entry in FP64 at fixed C6: phi = -C6 gg,
// and dphi_r = phi'(r) / r.  With x = r^2:
//  Becke-Johnson (Eq. 2), c = (Rd^6, Rd^8, R0^2, s8 R0^2):
//    gg = s6 / (x^3 + Rd^6) + s8 R0^2 / (x^4 + Rd^8);
//  zero damping, c = (K6, K8, R0^2, s8 R0^2), K6 = 6 (rs6 R0)^14,
//  K8 = 6 (rs8 R0)^16: f_n / r^n = x^4 / (x^(n/2+4) + K_n), so
//    gg = x^4 (s6 / (x^7 + K6) + s8 R0^2 / (x^8 + K8)) and
//    dphi_r = -2 C6 x^3 (s6 t6^2 (4 K6 - 3 x^7) + s8 R0^2 t8^2 (4 K8 - 4 x^8)).
// Both denominators come from one reciprocal of their product.
struct BJ {
    double gg, dphi_r;
};
template <bool ZERO>
__device__ __forceinline__ BJ damp_f64(double c6, double r2, const double4& c, double s6)
{
    const double r4 = r2 * r2, r6 = r4 * r2, r8 = r4 * r4;
    BJ o;
    if constexpr (ZERO) {
        const double x7 = r8 * r6, x8 = r8 * r8;
        const double A = x7 + c.x, B = x8 + c.y;
        const double inv = recip(A * B);
        const double t6 = B * inv, t8 = A * inv;
        const double a6 = s6 * t6, a8 = c.w * t8;
        o.gg = r8 * (a6 + a8);
        o.dphi_r = -2.0 * c6 * r6 *
                   (a6 * t6 * (4.0 * c.x - 3.0 * x7) + a8 * t8 * (4.0 * c.y - 4.0 * x8));
    } else {
        const double A = r6 + c.x, B = r8 + c.y;
        const double inv = recip(A * B);
        const double t6 = B * inv, t8 = A * inv;
        const double a6 = s6 * t6, a8 = c.w * t8;
        o.gg = a6 + a8;
        o.dphi_r = c6 * (6.0 * a6 * r4 * t6 + 8.0 * a8 * r6 * t8);
    }
    return o;
}

// One neighbour's position, weights and species (see piece_at).
template <bool F32>
struct Nbr;
template <>
struct Nbr<false> {
    double4 a;  // x, y, z, w0
    double4 b;  // w1..w4
};
template <>
struct Nbr<true> {
    double2 xy;
    double2 zw;  // z, (w0, w1)
    float4 b;    // w2, w3, w4, species
};

template <bool F32>
__device__ __forceinline__ void fetch(Nbr<F32>& nb, uint32_t code, int img_bits,
                                      const double* __restrict__ W, const float* __restrict__ Wf)
{
    const uint32_t j = code >> img_bits;
    if constexpr (F32) {
        const float4* r = (const float4*)Wf + piece_at(NPIECEF, PBLKF, 0, j);
        nb.xy = __builtin_bit_cast(double2, r[0]);
        nb.zw = __builtin_bit_cast(double2, r[PBLKF]);
        nb.b = r[2 * PBLKF];
    } else {
        const double4* r = (const double4*)W + piece_at(NPIECE, PBLK, 0, j);
        nb.a = r[0];
        nb.b = r[PBLK];
    }
}

// species of an FP64-form neighbour: bit k in the sign of w_k
__device__ __forceinline__ int rec_species(const Nbr<false>& nb)
{
    const uint32_t h0 = (uint32_t)__double2hiint(nb.a.w), h1 = (uint32_t)__double2hiint(nb.b.x);
    const uint32_t h2 = (uint32_t)__double2hiint(nb.b.y), h3 = (uint32_t)__double2hiint(nb.b.z);
    return (int)((h0 >> 31) | ((h1 >> 31) << 1) | ((h2 >> 31) << 2) | ((h3 >> 31) << 3));
}

// AV: also the direct part of each atom's virial (Eq. 7), the six
// components of sum over its entries of -1/2 phi'(r) r (x) r / r, to Vp.
template <bool F32, bool IMG, bool AV, bool ZERO>
__global__ void __launch_bounds__(BLOCK)
k_pair(int n, const double4* __restrict__ pos_s, const double4* __restrict__ img_tab, int n_img,
       int img_bits, const uint32_t* __restrict__ list_p, const int* __restrict__ cnt_p, int cap_p,
       const ElemTab* __restrict__ tab, const double* __restrict__ c6ref,
       const double4* __restrict__ pc, PairScal sc, const double* __restrict__ w,
       const double* __restrict__ wd, const double* __restrict__ W, const float* __restrict__ Wf,
       double* __restrict__ Fp, double* __restrict__ U, double* __restrict__ G,
       double* __restrict__ Vp, double* __restrict__ part)
{
    typedef typename std::conditional<F32, float, double>::type real;
    __shared__ double4 s_img[IMG ? IMG_LDS : 1];
    __shared__ double4 s_pc[MAXELEM * MAXELEM];
    __shared__ double s_M[M_LDS_ELEM * M_LDS_ELEM * MAXREF * MAXREF];
    __shared__ real s_u[WAVES_PER_BLOCK][2][MAXELEM * MAXREF];
    const int ne = tab->n_elem;
    const bool m_lds = ne <= M_LDS_ELEM;
    load_images<IMG>(s_img, img_tab, n_img);
    for (int k = threadIdx.x; k < MAXELEM * MAXELEM; k += blockDim.x) s_pc[k] = pc[k];
    if (m_lds)
        for (int k = threadIdx.x; k < ne * ne * MAXREF * MAXREF; k += blockDim.x) {
            const int e = k / (ne * MAXREF * MAXREF), r = k - e * ne * MAXREF * MAXREF;
            s_M[k] = c6ref[(size_t)e * MAXELEM * MAXREF * MAXREF + r];
        }
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const uint32_t img_mask = (1u << img_bits) - 1u;
    real* u = &s_u[wv][0][0];
    real* ud = &s_u[wv][1][0];
    double vir[6] = {0, 0, 0, 0, 0, 0};
    double esum = 0.0;
    const Walk wk = atom_walk(n);
    for (int i = wk.first; i < wk.end; i += wk.step) {
        const double4 pi = pos_s[i];
        const int zi = __builtin_amdgcn_readfirstlane(zbits(pi.w));
        const int cnt = min(cnt_p[i], cap_p);
        const uint32_t* lp = list_p + (size_t)i * cap_p;
        // list codes of the first two chunks go out first
        uint32_t code_c = list_code(lp, lane, cnt, cap_p);
        uint32_t code_n = list_code(lp, WAVE + lane, cnt, cap_p);
        // u_f = w_i^T M[zi][f] and u'_f = w_i'^T M[zi][f], this wave's LDS
        double wi[MAXREF], wdi[MAXREF];
#pragma unroll
        for (int a = 0; a < MAXREF; a++) {
            wi[a] = w[(size_t)i * MAXREF + a];
            wdi[a] = wd[(size_t)i * MAXREF + a];
        }
        for (int idx = lane; idx < 2 * ne * MAXREF; idx += WAVE) {
            const int which = idx >= ne * MAXREF ? 1 : 0;
            const int q = idx - which * ne * MAXREF;
            const int f = q / MAXREF, b = q - f * MAXREF;
            double v = 0.0;
#pragma unroll
            for (int a = 0; a < MAXREF; a++) {
                const double mab = m_lds ? s_M[((zi * ne + f) * MAXREF + a) * MAXREF + b]
                                         : c6ref[((size_t)(zi * MAXELEM + f) * MAXREF + a) * MAXREF + b];
                v = fma(which ? wdi[a] : wi[a], mab, v);
            }
            s_u[wv][which][q] = (real)v;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        Nbr<F32> nb_c;
        fetch<F32>(nb_c, code_c, img_bits, W, Wf);
        double fx = 0.0, fy = 0.0, fz = 0.0, ue = 0.0, g = 0.0;
        double av[6] = {0, 0, 0, 0, 0, 0};  // this atom's virial (AV only)
        for (int k0 = 0; k0 < cnt; k0 += WAVE) {
            const int k = k0 + lane;
            // codes two chunks ahead; neighbour data handed on to the next step
            const uint32_t code_nn = list_code(lp, k + 2 * WAVE, cnt, cap_p);
            Nbr<F32> nb_n;
            fetch<F32>(nb_n, code_n, img_bits, W, Wf);
            const double4 T = image<IMG>(s_img, img_tab, code_c & img_mask);
            double px, py, pz;
            if constexpr (F32) {
                px = nb_c.xy.x;
                py = nb_c.xy.y;
                pz = nb_c.zw.x;
            } else {
                px = nb_c.a.x;
                py = nb_c.a.y;
                pz = nb_c.a.z;
            }
            const double dx = px + T.x - pi.x;
            const double dy = py + T.y - pi.y;
            const double dz = pz + T.z - pi.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const bool in = k < cnt && r2 < sc.rp2;
            int zj;
            if constexpr (F32) zj = __float_as_int(nb_c.b.w);
            else zj = rec_species(nb_c);
            const real* uz = u + zj * MAXREF;
            const real* udz = ud + zj * MAXREF;
            const double4 c = s_pc[zi * MAXELEM + zj];  // Rd^6, Rd^8, R0^2, s8 R0^2
            if constexpr (!F32) {
                const double wj[MAXREF] = {fabs(nb_c.a.w), fabs(nb_c.b.x), fabs(nb_c.b.y),
                                           fabs(nb_c.b.z), nb_c.b.w};
                double c6 = 0.0, dc6 = 0.0;
#pragma unroll
                for (int b = 0; b < MAXREF; b++) {
                    c6 = fma(uz[b], wj[b], c6);
                    dc6 = fma(udz[b], wj[b], dc6);
                }
                c6 = in ? c6 : 0.0;
                dc6 = in ? dc6 : 0.0;
                const BJ q = damp_f64<ZERO>(c6, r2, c, sc.s6);
                ue = fma(-0.5 * c6, q.gg, ue);
                g = fma(-q.gg, dc6, g);
                fx = fma(q.dphi_r, dx, fx);
                fy = fma(q.dphi_r, dy, fy);
                fz = fma(q.dphi_r, dz, fz);
                virial_add(vir, -0.5 * q.dphi_r, dx, dy, dz);
                if constexpr (AV) virial_add(av, -0.5 * q.dphi_r, dx, dy, dz);
            } else {
                const float2 w01 = __builtin_bit_cast(float2, nb_c.zw.y);
                const float wj[MAXREF] = {w01.x, w01.y, nb_c.b.x, nb_c.b.y, nb_c.b.z};
                float c6 = 0.0f, dc6 = 0.0f;
#pragma unroll
                for (int b = 0; b < MAXREF; b++) {
                    c6 = fmaf(uz[b], wj[b], c6);
                    dc6 = fmaf(udz[b], wj[b], dc6);
                }
                c6 = in ? c6 : 0.0f;
                dc6 = in ? dc6 : 0.0f;
                const float x = (float)dx, y = (float)dy, zz = (float)dz;
                float gg, dphi_r;
                if constexpr (ZERO) {
                    // in powers of 1/r^2 (no overflow of r^16 in FP32): with
                    // q_n = ((rs_n R0)^2 / r^2)^(n/2+4) and f_n = 1 / (1 + 6 q_n),
                    // gg = s6 f6 / r^6 + s8 R0^2 f8 / r^8 and
                    // dphi_r = -2 C6 [s6 f6 (42 f6 q6 - 3) / r^8
                    //                 + s8 R0^2 f8 (48 f8 q8 - 4) / r^10]
                    const float iy = __frcp_rn(in ? (float)r2 : 1.0f);
                    const float b6 = (float)(sc.rs6sq * c.z) * iy, b8 = (float)(sc.rs8sq * c.z) * iy;
                    const float b62 = b6 * b6, b82 = b8 * b8, b84 = b82 * b82;
                    const float q6 = b62 * b62 * b62 * b6, q8 = b84 * b84;
                    const float f6 = __frcp_rn(1.0f + 6.0f * q6), f8 = __frcp_rn(1.0f + 6.0f * q8);
                    const float y2 = iy * iy, y3 = y2 * iy, y4 = y2 * y2;
                    const float a6 = (float)sc.s6 * f6, a8 = (float)c.w * f8;
                    gg = a6 * y3 + a8 * y4;
                    dphi_r = -2.0f * c6 *
                             (a6 * y4 * (42.0f * f6 * q6 - 3.0f) + a8 * y4 * iy * (48.0f * f8 * q8 - 4.0f));
                } else {
                    const float q2 = (float)r2;
                    const float r4 = q2 * q2, r6 = r4 * q2, r8 = r4 * r4;
                    const float t6 = __frcp_rn(r6 + (float)c.x), t8 = __frcp_rn(r8 + (float)c.y);
                    const float a6 = (float)sc.s6 * t6, a8 = (float)c.w * t8;
                    gg = a6 + a8;
                    dphi_r = c6 * (6.0f * a6 * r4 * t6 + 8.0f * a8 * r6 * t8);
                }
                ue += (double)(-0.5f * c6 * gg);
                g += (double)(-gg * dc6);
                fx += (double)(dphi_r * x);
                fy += (double)(dphi_r * y);
                fz += (double)(dphi_r * zz);
                const float h = -0.5f * dphi_r;
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
            }
            code_c = code_n;
            code_n = code_nn;
            nb_c = nb_n;
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
                for (int c = 0; c < 6; c++) Vp[6 * (size_t)i + c] = t[5 + c];
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
            Fp[3 * (size_t)i] = fx;
            Fp[3 * (size_t)i + 1] = fy;
            Fp[3 * (size_t)i + 2] = fz;
            U[i] = ue;
            G[i] = g;
        }
        // the next atom rewrites u: every lane has finished reading it
        __builtin_amdgcn_wave_barrier();
    }
    // energy enters once per wave (esum is wave-uniform), virial per lane
    const double vals[7] = {lane == 0 ? esum : 0.0, vir[0], vir[1], vir[2], vir[3], vir[4], vir[5]};
    block_partials(vals, part);
}

// The dispersion pass with C6 from Eq. 3 as printed (D3_MODE_LITERAL): for
// every entry the Gaussian weight of each reference pair (a, b),
// exp(-4 ((n_i - n_a)^2 + (n_j - n_b)^2)), K_i K_j exponentials, and the
// weighted mean of the reference C6 values.  The exponents are shifted by
// their largest value before exponentiation, an exact identity of the ratio
// that keeps it finite.  dC6/dn_i = (S' - C6 Z') / Z with Z = sum of the
// weights, S = sum of weight x C6_ref and ' the derivative in n_i.  It
// reads the CNs, not the factorised weights, and is otherwise the FP64
// dispersion pass (one wave per atom, sums gathered onto the atom).
template <bool IMG, bool AV, bool ZERO>
__global__ void __launch_bounds__(BLOCK)
k_pair_lit(int n, const double4* __restrict__ pos_s, const double4* __restrict__ img_tab,
           int n_img, int img_bits, const uint32_t* __restrict__ list_p,
           const int* __restrict__ cnt_p, int cap_p, const ElemTab* __restrict__ tab,
           const double* __restrict__ c6ref, const double4* __restrict__ pc, PairScal sc,
           const double* __restrict__ cn, double* __restrict__ Fp, double* __restrict__ U,
           double* __restrict__ G, double* __restrict__ Vp, double* __restrict__ part)
{
    __shared__ double4 s_img[IMG ? IMG_LDS : 1];
    __shared__ double4 s_pc[MAXELEM * MAXELEM];
    __shared__ double s_cnref[MAXELEM * MAXREF];
    __shared__ int s_nref[MAXELEM];
    load_images<IMG>(s_img, img_tab, n_img);
    for (int k = threadIdx.x; k < MAXELEM * MAXELEM; k += blockDim.x) s_pc[k] = pc[k];
    if (threadIdx.x < MAXELEM * MAXREF) s_cnref[threadIdx.x] = tab->cn_ref[threadIdx.x];
    if (threadIdx.x < MAXELEM) s_nref[threadIdx.x] = tab->n_ref[threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1);
    const uint32_t img_mask = (1u << img_bits) - 1u;
    double vir[6] = {0, 0, 0, 0, 0, 0};
    double esum = 0.0;
    const Walk wk = atom_walk(n);
    for (int i = wk.first; i < wk.end; i += wk.step) {
        const double4 pi = pos_s[i];
        const int zi = __builtin_amdgcn_readfirstlane(zbits(pi.w));
        const int Ki = __builtin_amdgcn_readfirstlane(s_nref[zi]);
        const double ni = cn[i];
        const int cnt = min(cnt_p[i], cap_p);
        const uint32_t* lp = list_p + (size_t)i * cap_p;
        double da[MAXREF];
#pragma unroll
        for (int a = 0; a < MAXREF; a++) da[a] = ni - s_cnref[zi * MAXREF + a];
        double fx = 0.0, fy = 0.0, fz = 0.0, ue = 0.0, g = 0.0;
        double av[6] = {0, 0, 0, 0, 0, 0};
        for (int k0 = 0; k0 < cnt; k0 += WAVE) {
            const int k = k0 + lane;
            const uint32_t code = list_code(lp, k, cnt, cap_p);
            const uint32_t j = code >> img_bits;
            const double4 pj = pos_s[j];
            const double nj = cn[j];
            const double4 T = image<IMG>(s_img, img_tab, code & img_mask);
            const double dx = pj.x + T.x - pi.x;
            const double dy = pj.y + T.y - pi.y;
            const double dz = pj.z + T.z - pi.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const bool in = k < cnt && r2 < sc.rp2;
            const int zj = zbits(pj.w);
            const int Kj = s_nref[zj];
            const double* M = c6ref + (size_t)(zi * MAXELEM + zj) * MAXREF * MAXREF;
            double db[MAXREF];
#pragma unroll
            for (int b = 0; b < MAXREF; b++) db[b] = nj - s_cnref[zj * MAXREF + b];
            // largest exponent over the reference pairs
            double emax = -1e300;
            for (int a = 0; a < Ki; a++)
#pragma unroll
                for (int b = 0; b < MAXREF; b++)
                    if (b < Kj) emax = fmax(emax, -4.0 * (da[a] * da[a] + db[b] * db[b]));
            double Z = 0.0, S = 0.0, Zd = 0.0, Sd = 0.0;
            for (int a = 0; a < Ki; a++) {
                const double ta = -8.0 * da[a];  // d(exponent)/dn_i
#pragma unroll
                for (int b = 0; b < MAXREF; b++) {
                    if (b < Kj) {
                        const double L = exp(-4.0 * (da[a] * da[a] + db[b] * db[b]) - emax);
                        const double LC = L * M[a * MAXREF + b];
                        Z += L;
                        S += LC;
                        Zd = fma(L, ta, Zd);
                        Sd = fma(LC, ta, Sd);
                    }
                }
            }
            double c6 = S / Z;
            double dc6 = (Sd - c6 * Zd) / Z;
            c6 = in ? c6 : 0.0;
            dc6 = in ? dc6 : 0.0;
            const BJ q = damp_f64<ZERO>(c6, r2, s_pc[zi * MAXELEM + zj], sc.s6);
            ue = fma(-0.5 * c6, q.gg, ue);
            g = fma(-q.gg, dc6, g);
            fx = fma(q.dphi_r, dx, fx);
            fy = fma(q.dphi_r, dy, fy);
            fz = fma(q.dphi_r, dz, fz);
            virial_add(vir, -0.5 * q.dphi_r, dx, dy, dz);
            if constexpr (AV) virial_add(av, -0.5 * q.dphi_r, dx, dy, dz);
        }
        if constexpr (AV) {
            wave_sums(av);
            if (lane == 0)
#pragma unroll
                for (int c = 0; c < 6; c++) Vp[6 * (size_t)i + c] = av[c];
        }
        double t5[5] = {fx, fy, fz, ue, g};
        wave_sums(t5);
        esum += t5[3];
        if (lane == 0) {
            Fp[3 * (size_t)i] = t5[0];
            Fp[3 * (size_t)i + 1] = t5[1];
            Fp[3 * (size_t)i + 2] = t5[2];
            U[i] = t5[3];
            G[i] = t5[4];
        }
    }
    const double vals[7] = {lane == 0 ? esum : 0.0, vir[0], vir[1], vir[2], vir[3], vir[4], vir[5]};
    block_partials(vals, part);
}

int launch_pair_lit(int n, const double4* pos_s, const double4* img_tab, int n_img, int img_bits,
                    const uint32_t* list_p, const int* cnt_p, int cap_p, const ElemTab* tab,
                    const double* c6ref, const double4* pc, PairScal sc, const double* cn,
                    double* Fp, double* U, double* G, double* Vp, double* part, hipStream_t s)
{
    if (n <= 0) return 0;
    const bool lds = n_img <= IMG_LDS;
    int nblk = 0;
#define D3_LIT(I, A, Z)                                                                        \
    {                                                                                          \
        nblk = pass_blocks((const void*)&k_pair_lit<I, A, Z>, n);                              \
        hipLaunchKernelGGL((k_pair_lit<I, A, Z>), dim3(nblk), dim3(BLOCK), 0, s, n, pos_s,     \
                           img_tab, n_img, img_bits, list_p, cnt_p, cap_p, tab, c6ref, pc, sc, \
                           cn, Fp, U, G, Vp, part);                                            \
    }
#define D3_LIT_Z(I, A)          \
    if (sc.zero) D3_LIT(I, A, true) \
    else D3_LIT(I, A, false)
    if (Vp) {
        if (lds) D3_LIT_Z(true, true)
        else D3_LIT_Z(false, true)
    } else {
        if (lds) D3_LIT_Z(true, false)
        else D3_LIT_Z(false, false)
    }
#undef D3_LIT_Z
#undef D3_LIT
    return nblk;
}

int launch_pair(int mode, int n, const double4* pos_s, const double4* img_tab, int n_img,
                int img_bits, const uint32_t* list_p, const int* cnt_p, int cap_p,
                const ElemTab* tab, const double* c6ref, const double4* pc, PairScal sc,
                const double* w, const double* wd, const double* W, const float* Wf, double* Fp,
                double* U, double* G, double* Vp, double* part, hipStream_t s)
{
    if (n <= 0) return 0;
    const bool lds = n_img <= IMG_LDS;
    int nblk = 0;
#define D3_PAIR_(F, I, A, Z)                                                                    \
    {                                                                                           \
        nblk = pass_blocks((const void*)&k_pair<F, I, A, Z>, n);                                \
        hipLaunchKernelGGL((k_pair<F, I, A, Z>), dim3(nblk), dim3(BLOCK), 0, s, n, pos_s,       \
                           img_tab, n_img, img_bits, list_p, cnt_p, cap_p, tab, c6ref, pc, sc,  \
                           w, wd, W, Wf, Fp, U, G, Vp, part);                                   \
    }
#define D3_PAIR(F, I, A)              \
    if (sc.zero) D3_PAIR_(F, I, A, true) \
    else D3_PAIR_(F, I, A, false)
    const bool prec = mode == D3_MODE_PREC_F32;
    if (Vp) {
        if (prec) {
            if (lds) D3_PAIR(true, true, true)
            else D3_PAIR(true, false, true)
        } else {
            if (lds) D3_PAIR(false, true, true)
            else D3_PAIR(false, false, true)
        }
    } else {
        if (prec) {
            if (lds) D3_PAIR(true, true, false)
            else D3_PAIR(true, false, false)
        } else {
            if (lds) D3_PAIR(false, true, false)
            else D3_PAIR(false, false, false)
        }
    }
#undef D3_PAIR
#undef D3_PAIR_
    return nblk;
}

}  // namespace d3
