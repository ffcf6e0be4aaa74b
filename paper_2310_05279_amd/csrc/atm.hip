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
// One wavefront treats one atom A.  A's R_cn-list entries are taken in raw
// blocks of 64: the entries of a block that lie within r_atm of A are
// compacted into LDS with everything a triangle needs from them (the
// displacement from A, its square a, 1/a, a^(-1/6), C6 with A and its
// CN derivative over C6, the weights and the species).  The lanes then walk
// the pairs of cached entries, 64 at a time: the pairs inside a block, then
// those between it and every later block (loaded into a second LDS half),
// so lists of any length are covered without global loads in the pair loop.
// A triangle is found once from each of its vertices; atom A takes a third
// of its energy and virial, its whole force on A, -dE/dr_A = 2 dE/da d_AB +
// 2 dE/dc d_AC (d the vectors from A), and dE/dn_A = E/2 (dC6_AB/dn_A /
// C6_AB + dC6_AC/dn_A / C6_AC), which the chain pass turns into forces like
// the two-body dE/dn.  Every sum is gathered onto A: no atomics.  FP64 in
// every mode, with C6 from the factorised weights (exact Eq. 3) also in the
// surrogate mode.
//
// The geometry needs no cube or square root per triangle beyond one sixth
// root: with t = (abc)^(-1/6) = a^(-1/6) b^(-1/6) c^(-1/6), (abc)^(-1/2) = t^3,
// (abc)^(-3/2) = t^9, and (rbar / (4/3 R0bar))^-16 = (4/3 t R0c)^16, where
// R0c = (R0_AB R0_BC R0_CA)^(1/3) is a product of per-element-pair sixth
// roots of R0^2.
#include "d3_device.h"

namespace d3 {

constexpr int ATM_M_LDS_ELEM = 8;  // C6 reference table in LDS up to 8 elements
constexpr int ATM_BS = 32;          // raw list entries per block
constexpr int ATM_SLOTS = 2 * ATM_BS;
constexpr int ATM_Q = 128;          // queued triangles per wave (a ring)
static_assert(ATM_BS <= WAVE, "one lane per raw entry of a block");
constexpr double ATM_SR3 = 4.0 / 3.0;

__device__ __forceinline__ double atm_recip(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

// x^(-1/6) for x > 0: an FP32 estimate from the hardware base-2 logarithm
// and exponential (relative error ~1e-7), then two Newton steps in FP64 for
// y^-6 = x, y <- y (7 - x y^6) / 6 (error e -> -3.5 e^2 each)
__device__ __forceinline__ double rsixth(double x)
{
    const float xf = (float)x;
    double y = (double)__builtin_amdgcn_exp2f(-0.16666667f * __builtin_amdgcn_logf(xf));
#pragma unroll
    for (int it = 0; it < 2; it++) {
        const double y2 = y * y;
        const double y6 = y2 * y2 * y2;
        y = y * fma(-x, y6, 7.0) * (1.0 / 6.0);
    }
    return y;
}

// the pair index p of the strict upper triangle, enumerated as
// (0,1), (0,2), (1,2), (0,3), ...: entries e1 < e2 with p = e2 (e2-1)/2 + e1
__device__ __forceinline__ void pair_of(int p, int& e1, int& e2)
{
    int t = (int)((1.0f + __builtin_sqrtf(1.0f + 8.0f * (float)p)) * 0.5f);
    if (t * (t - 1) / 2 > p) t--;
    if ((t + 1) * t / 2 <= p) t++;
    e2 = t;
    e1 = p - t * (t - 1) / 2;
}

// cached entries of one wave (structure of arrays: consecutive lanes read
// consecutive slots)
struct AtmCache {
    double dx[ATM_SLOTS], dy[ATM_SLOTS], dz[ATM_SLOTS];
    double a[ATM_SLOTS], ia[ATM_SLOTS], s[ATM_SLOTS];  // r^2, 1/r^2, r^(-1/3)
    double c6[ATM_SLOTS], g[ATM_SLOTS];                // C6 with A, dC6/dn_A / C6
    double w[MAXREF][ATM_SLOTS];
    int z[ATM_SLOTS];
};

// per-lane sums of the atom being treated
template <bool AV>
struct AtmAcc {
    double fx = 0.0, fy = 0.0, fz = 0.0, ue = 0.0, g = 0.0;
    double vir[6] = {0, 0, 0, 0, 0, 0};
    double av[AV ? 6 : 1] = {0};
};

// One triangle A, B = slot e1, C = slot e2 (both within r_atm of A); its
// third side is tested here.  A lane without a pair passes in = false.
template <bool AV, bool MLDS>
__device__ __forceinline__ void atm_pair(const AtmCache& ce, int e1, int e2, bool in, int zi,
                                         int ne, const double* s_M,
                                         const double* __restrict__ c6ref, const double* s_r0c,
                                         double s9, double ra2, AtmAcc<AV>& acc)
{
    const double d1x = ce.dx[e1], d1y = ce.dy[e1], d1z = ce.dz[e1];
    const double d2x = ce.dx[e2], d2y = ce.dy[e2], d2z = ce.dz[e2];
    const double bx = d2x - d1x, by = d2y - d1y, bz = d2z - d1z;
    double b = bx * bx + by * by + bz * bz;
    in = in && b < ra2;
    b = in ? b : 1.0;  // a harmless side for lanes without a triangle
    const double a = ce.a[e1], c = ce.a[e2];
    const double ia = ce.ia[e1], ic = ce.ia[e2];
    const int zb = ce.z[e1], zc = ce.z[e2];
    // C6 between B and C: w_B^T M[zB][zC] w_C, with M from LDS (MLDS) or
    // global memory, chosen at compile time so that the loads are LDS or
    // global ones rather than generic ones
    const double* M = MLDS ? s_M + (zb * ne + zc) * MAXREF * MAXREF
                           : c6ref + (size_t)(zb * MAXELEM + zc) * MAXREF * MAXREF;
    double cbc = 0.0;
#pragma unroll
    for (int ra = 0; ra < MAXREF; ra++) {
        double t = 0.0;
#pragma unroll
        for (int rb = 0; rb < MAXREF; rb++) t = fma(M[ra * MAXREF + rb], ce.w[rb][e2], t);
        cbc = fma(ce.w[ra][e1], t, cbc);
    }
    const double sb = rsixth(b);
    const double ib = (sb * sb) * (sb * sb) * (sb * sb);  // 1/b
    const double t = ce.s[e1] * ce.s[e2] * sb;             // (abc)^(-1/6)
    const double t3 = t * t * t;                            // (abc)^(-1/2)
    const double iu = t3 * t3;                              // 1/(abc)
    const double u15 = iu * t3;                             // (abc)^(-3/2)
    const double x = a + c - b, y = a + b - c, z = b + c - a;
    const double P = x * y * z;
    const double ang = 1.0 + 0.375 * P * iu;
    const double X = ATM_SR3 * t * s_r0c[zi * MAXELEM + zb] * s_r0c[zb * MAXELEM + zc] *
                     s_r0c[zc * MAXELEM + zi];
    const double X2 = X * X, X4 = X2 * X2, X8 = X4 * X4;
    const double q = X8 * X8;  // (rbar / (4/3 R0bar))^-16
    const double f3 = atm_recip(fma(6.0, q, 1.0));
    const double uf = u15 * f3;
    const double k16 = ang * fma(16.0 * f3, q, -1.5);
    // dg/da, dg/db, dg/dc of g = ang (abc)^(-3/2) f3
    const double ga = uf * (0.375 * (y * z + x * z - x * y - P * ia) * iu + k16 * ia);
    const double gb = uf * (0.375 * (x * z - y * z + x * y - P * ib) * iu + k16 * ib);
    const double gc = uf * (0.375 * (y * z - x * z + x * y - P * ic) * iu + k16 * ic);
    const double cab = ce.c6[e1], cac = ce.c6[e2];
    const double cc = in ? s9 * sqrt(cab * cbc * cac) : 0.0;
    const double E = cc * (ang * uf);
    constexpr double THIRD_E = 1.0 / 3.0;
    acc.ue = fma(E, THIRD_E, acc.ue);
    acc.g = fma(0.5 * E, ce.g[e1] + ce.g[e2], acc.g);
    const double ha = 2.0 * cc * ga, hc = 2.0 * cc * gc;
    acc.fx += ha * d1x + hc * d2x;
    acc.fy += ha * d1y + hc * d2y;
    acc.fz += ha * d1z + hc * d2z;
    // a third of -2 sum over the sides of dE/d(side^2) side (x) side
    constexpr double THIRD = 1.0 / 3.0;
    const double wa = -ha * THIRD, wbb = -2.0 * THIRD * cc * gb, wcc = -hc * THIRD;
    virial_add(acc.vir, wa, d1x, d1y, d1z);
    virial_add(acc.vir, wbb, bx, by, bz);
    virial_add(acc.vir, wcc, d2x, d2y, d2z);
    if constexpr (AV) {
        virial_add(acc.av, wa, d1x, d1y, d1z);
        virial_add(acc.av, wbb, bx, by, bz);
        virial_add(acc.av, wcc, d2x, d2y, d2z);
    }
}

// the LDS writes of this wave are complete and visible to its lanes
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool IMG, bool AV, bool MLDS>
__global__ void __launch_bounds__(BLOCK)
k_atm(int n, const double4* __restrict__ pos_s, const double4* __restrict__ img_tab, int n_img,
      int img_bits, const uint32_t* __restrict__ list_c, const int* __restrict__ cnt_c, int cap_c,
      const ElemTab* __restrict__ tab, const double* __restrict__ c6ref,
      const double4* __restrict__ pc, double s9, double ra2, const double* __restrict__ w,
      const double* __restrict__ wd, double* __restrict__ Fp, double* __restrict__ U,
      double* __restrict__ G, double* __restrict__ Vp, double* __restrict__ part)
{
    __shared__ double4 s_img[IMG ? IMG_LDS : 1];
    __shared__ double s_r0c[MAXELEM * MAXELEM];
    __shared__ double s_M[MLDS ? ATM_M_LDS_ELEM * ATM_M_LDS_ELEM * MAXREF * MAXREF : 1];
    __shared__ double s_u[WAVES_PER_BLOCK][2][MAXELEM * MAXREF];
    __shared__ AtmCache s_e[WAVES_PER_BLOCK];
    __shared__ uint16_t s_q[WAVES_PER_BLOCK][ATM_Q];
    const int ne = tab->n_elem;
    load_images<IMG>(s_img, img_tab, n_img);
    // (R0^2)^(1/6) per element pair: R0c of a triangle is the product of three
    for (int k = threadIdx.x; k < MAXELEM * MAXELEM; k += blockDim.x)
        s_r0c[k] = pc[k].z > 0.0 ? 1.0 / rsixth(pc[k].z) : 0.0;
    if constexpr (MLDS)
        for (int k = threadIdx.x; k < ne * ne * MAXREF * MAXREF; k += blockDim.x) {
            const int e = k / (ne * MAXREF * MAXREF), r = k - e * ne * MAXREF * MAXREF;
            s_M[k] = c6ref[(size_t)e * MAXELEM * MAXREF * MAXREF + r];
        }
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const uint32_t img_mask = (1u << img_bits) - 1u;
    const double* u = &s_u[wv][0][0];
    const double* ud = &s_u[wv][1][0];
    AtmCache& ce = s_e[wv];
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
            const double* M = MLDS ? s_M + (zi * ne + f) * MAXREF * MAXREF
                                   : c6ref + (size_t)(zi * MAXELEM + f) * MAXREF * MAXREF;
            const double* wa = (which ? wd : w) + (size_t)i * MAXREF;
            double v = 0.0;
#pragma unroll
            for (int a = 0; a < MAXREF; a++) v = fma(wa[a], M[a * MAXREF + b], v);
            s_u[wv][which][q] = v;
        }
        wave_lds_sync();
        // raw block k of the list -> the slots from base on; returns how many
        // of its entries lie within r_atm
        auto load_block = [&](int k, int base) -> int {
            const int e = k * ATM_BS + lane;
            double dx = 0.0, dy = 0.0, dz = 0.0, a = 2.0 * ra2;
            int j = 0, zj = 0;
            if (lane < ATM_BS && e < cnt) {
                const uint32_t code = lc[e];
                j = (int)(code >> img_bits);
                const double4 pj = pos_s[j];
                zj = zbits(pj.w);
                const double4 T = image<IMG>(s_img, img_tab, code & img_mask);
                dx = pj.x + T.x - pi.x;
                dy = pj.y + T.y - pi.y;
                dz = pj.z + T.z - pi.z;
                a = dx * dx + dy * dy + dz * dz;
            }
            const bool in = a < ra2;
            const unsigned long long m = __ballot(in);
            if (in) {
                const int slot = base + (int)__builtin_amdgcn_mbcnt_hi(
                                            (uint32_t)(m >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                double wj[MAXREF];
#pragma unroll
                for (int r = 0; r < MAXREF; r++) wj[r] = w[(size_t)j * MAXREF + r];
                double c6 = 0.0, dc6 = 0.0;
#pragma unroll
                for (int r = 0; r < MAXREF; r++) {
                    c6 = fma(u[zj * MAXREF + r], wj[r], c6);
                    dc6 = fma(ud[zj * MAXREF + r], wj[r], dc6);
                }
                const double sa = rsixth(a);
                ce.dx[slot] = dx;
                ce.dy[slot] = dy;
                ce.dz[slot] = dz;
                ce.a[slot] = a;
                ce.ia[slot] = (sa * sa) * (sa * sa) * (sa * sa);
                ce.s[slot] = sa;
                ce.c6[slot] = c6;
                ce.g[slot] = dc6 * atm_recip(c6);
#pragma unroll
                for (int r = 0; r < MAXREF; r++) ce.w[r][slot] = wj[r];
                ce.z[slot] = zj;
            }
            wave_lds_sync();
            return (int)__popcll(m);
        };
        AtmAcc<AV> acc;
        // Pairs of cached entries go through two steps: a cheap one that
        // tests the third side and queues the pairs that close a triangle
        // (about half of them) in this wave's LDS ring, and the full triangle
        // evaluation, 64 queued pairs at a time.  Queued pairs name cache
        // slots, so the queue is emptied before a block load overwrites any.
        int qhead = 0, qn = 0;  // wave-uniform
        auto run_batch = [&](int k) {
            const uint32_t it = s_q[wv][(qhead + (lane < k ? lane : 0)) & (ATM_Q - 1)];
            atm_pair<AV, MLDS>(ce, (int)(it & 0xFFu), (int)(it >> 8), lane < k, zi, ne, s_M,
                               c6ref, s_r0c, s9, ra2, acc);
            qhead = (qhead + k) & (ATM_Q - 1);
            qn -= k;
            __builtin_amdgcn_wave_barrier();
        };
        auto enqueue = [&](int e1, int e2, bool valid) {
            const double bx = ce.dx[e2] - ce.dx[e1], by = ce.dy[e2] - ce.dy[e1],
                         bz = ce.dz[e2] - ce.dz[e1];
            const bool in = valid && bx * bx + by * by + bz * bz < ra2;
            const unsigned long long m = __ballot(in);
            if (in)
                s_q[wv][(qhead + qn + (int)__builtin_amdgcn_mbcnt_hi(
                                          (uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))) &
                        (ATM_Q - 1)] = (uint16_t)(e1 | (e2 << 8));
            qn += (int)__popcll(m);
            wave_lds_sync();
            if (qn >= WAVE) run_batch(WAVE);
        };
        auto flush = [&]() {
            if (qn > 0) run_batch(qn);
        };
        const int nblk = (cnt + ATM_BS - 1) / ATM_BS;
        if (nblk <= 2) {
            // both blocks stay in the cache: one triangle over all their entries
            const int m0 = load_block(0, 0);
            const int m1 = nblk == 2 ? load_block(1, ATM_BS) : 0;
            const int m = m0 + m1;
            const int ntri = m * (m - 1) / 2;
            for (int p0 = 0; p0 < ntri; p0 += WAVE) {
                const int p = p0 + lane;
                int v1 = 0, v2 = 1;
                if (p < ntri) pair_of(p, v1, v2);
                const int e1 = v1 < m0 ? v1 : ATM_BS + (v1 - m0);
                const int e2 = v2 < m0 ? v2 : ATM_BS + (v2 - m0);
                enqueue(e1, e2, p < ntri);
            }
            flush();
        } else {
            for (int bi = 0; bi < nblk; bi++) {
                flush();
                const int mi = load_block(bi, 0);
                // pairs inside block bi
                const int ntri = mi * (mi - 1) / 2;
                for (int p0 = 0; p0 < ntri; p0 += WAVE) {
                    const int p = p0 + lane;
                    int e1 = 0, e2 = 1;
                    if (p < ntri) pair_of(p, e1, e2);
                    enqueue(e1, e2, p < ntri);
                }
                // pairs between block bi and every later block
                for (int bj = bi + 1; bj < nblk && mi > 0; bj++) {
                    flush();
                    const int mj = load_block(bj, ATM_BS);
                    const int nrect = mi * mj;
                    const float inv = 1.0f / (float)(mj > 0 ? mj : 1);
                    for (int p0 = 0; p0 < nrect; p0 += WAVE) {
                        const int p = p0 + lane;
                        int e1 = (int)((float)p * inv);
                        if (e1 * mj > p) e1--;
                        if ((e1 + 1) * mj <= p) e1++;
                        const bool ok = p < nrect;
                        e1 = ok ? e1 : 0;
                        const int e2 = ok ? ATM_BS + (p - e1 * mj) : ATM_BS;
                        enqueue(e1, e2, ok);
                    }
                }
            }
            flush();
        }
        double fx, fy, fz, ue, g;
        if constexpr (AV) {
            double t[11] = {acc.fx, acc.fy, acc.fz, acc.ue, acc.g, acc.av[0], acc.av[1],
                            acc.av[2], acc.av[3], acc.av[4], acc.av[5]};
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
            double t[5] = {acc.fx, acc.fy, acc.fz, acc.ue, acc.g};
            wave_sums(t);
            fx = t[0];
            fy = t[1];
            fz = t[2];
            ue = t[3];
            g = t[4];
        }
#pragma unroll
        for (int k = 0; k < 6; k++) vir[k] += acc.vir[k];
        esum += ue;
        if (lane == 0) {
            Fp[3 * (size_t)i] += fx;
            Fp[3 * (size_t)i + 1] += fy;
            Fp[3 * (size_t)i + 2] += fz;
            U[i] += ue;
            G[i] += g;
        }
        // the next atom rewrites u and the cache: every lane has finished
        // reading them
        __builtin_amdgcn_wave_barrier();
    }
    const double vals[7] = {lane == 0 ? esum : 0.0, vir[0], vir[1], vir[2], vir[3], vir[4], vir[5]};
    block_partials(vals, part);
}

int launch_atm(int n, const double4* pos_s, const double4* img_tab, int n_img, int img_bits,
               const uint32_t* list_c, const int* cnt_c, int cap_c, const ElemTab* tab,
               int n_elem, const double* c6ref, const double4* pc, double s9, double ra2,
               const double* w, const double* wd, double* Fp, double* U, double* G, double* Vp,
               double* part, hipStream_t s)
{
    if (n <= 0) return 0;
    const bool lds = n_img <= IMG_LDS;
    const bool mlds = n_elem <= ATM_M_LDS_ELEM;
    int nblk = 0;
#define D3_ATM(I, A, M)                                                                        \
    {                                                                                          \
        nblk = pass_blocks((const void*)&k_atm<I, A, M>, n);                                   \
        hipLaunchKernelGGL((k_atm<I, A, M>), dim3(nblk), dim3(BLOCK), 0, s, n, pos_s, img_tab, \
                           n_img, img_bits, list_c, cnt_c, cap_c, tab, c6ref, pc, s9, ra2, w,  \
                           wd, Fp, U, G, Vp, part);                                            \
    }
#define D3_ATM_M(I, A)            \
    if (mlds) D3_ATM(I, A, true)  \
    else D3_ATM(I, A, false)
    if (Vp) {
        if (lds) D3_ATM_M(true, true)
        else D3_ATM_M(false, true)
    } else {
        if (lds) D3_ATM_M(true, false)
        else D3_ATM_M(false, false)
    }
#undef D3_ATM_M
#undef D3_ATM
    return nblk;
}

}  // namespace d3
