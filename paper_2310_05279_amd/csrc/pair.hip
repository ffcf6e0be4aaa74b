// Coordination numbers (Eq. 4), Gaussian weights and C6 projections
// (Eq. 3), the BJ-damped dispersion pass (Eq. 2 with its direct force,
// dE/dn and virial), the chain pass through the coordination numbers
// (the many-body part of Eqs. 5-7) and the FP64 reductions (Eq. 1).
//
// One wavefront owns one atom i at a time (grid-stride over cell-sorted
// atoms); its 64 lanes walk i's neighbour list, 64 entries per step.
// Every sum is a gather onto i (each unordered pair is evaluated from both
// ends), so no floating-point atomics are used and the results do not
// depend on scheduling.  Per-atom sums close with a butterfly reduction
// across the wave; the virial stays in registers across all atoms a wave
// owns and is reduced once per wave.
//
// C6 factorises: the Gaussian weight of Eq. 3 is a product over the two
// atoms and so is its normaliser, hence C6_ij = w_i^T M_{Zi Zj} w_j with
// w the normalised per-atom weights.  The CN pass stores, for every atom j
// and every element e, P_e(j) = M_{e Zj} w_j; the pair pass then needs
// only C6 = w_i . P_Zi(j) and dC6/dn_i = w_i' . P_Zi(j) (K_i FMAs each,
// with w_i wave-uniform).
//
// Precision form (D3_MODE_PREC_F32): distances and cutoff tests in FP64,
// then the pair arithmetic in FP32 (hardware exp/rcp), with every per-lane
// and per-atom sum accumulated in FP64; weights stay FP64.
#include "d3_internal.h"

namespace d3 {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

__device__ __forceinline__ int zbits(double w) { return __double2loint(w); }

// Waves launched by the per-atom passes: one per atom up to a cap, then a
// grid-stride loop; always a whole number of workgroups, so every launched
// wave owns a virial slot.
int pass_waves(int n)
{
    const int max_waves = 256 * 4 * 16;  // 256 CUs x 4 SIMDs x 16 waves
    int w = n < max_waves ? (n > 0 ? n : 1) : max_waves;
    return (w + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK * WAVES_PER_BLOCK;
}

static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

// ------------------------------------------------------------- CN pass --

template <bool F32>
__global__ void __launch_bounds__(BLOCK)
k_cn(int n, const double4* __restrict__ pos_s, const double4* __restrict__ img_tab,
     int img_bits, const uint32_t* __restrict__ list_c, const int* __restrict__ cnt_c,
     int cap_c, const ElemTab* __restrict__ tab, const double* __restrict__ c6ref,
     double rc2, double* __restrict__ cn, double* __restrict__ w,
     double* __restrict__ wd, double* __restrict__ P, float* __restrict__ Pf,
     float* __restrict__ cnf)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
    const int nwaves = (gridDim.x * blockDim.x) / WAVE;
    const uint32_t img_mask = (1u << img_bits) - 1u;
    const int ne = tab->n_elem;
    for (int i = wave; i < n; i += nwaves) {
        const double4 pi = pos_s[i];
        const int zi = __builtin_amdgcn_readfirstlane(zbits(pi.w));
        const double rci = tab->rcov[zi];
        const int cnt = cnt_c[i];
        const uint32_t* lc = list_c + (size_t)i * cap_c;
        double sum = 0.0;
        for (int k0 = 0; k0 < cnt; k0 += WAVE) {
            const int k = k0 + lane;
            if (k < cnt) {
                const uint32_t code = lc[k];
                const int j = (int)(code >> img_bits);
                const double4 pj = pos_s[j];
                const double4 T = img_tab[code & img_mask];
                const double dx = pj.x + T.x - pi.x;
                const double dy = pj.y + T.y - pi.y;
                const double dz = pj.z + T.z - pi.z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < rc2) {
                    const double rs = rci + tab->rcov[zbits(pj.w)];
                    if (F32) {
                        const float r = sqrtf((float)r2);
                        const float e = __expf(-16.0f * ((float)rs / r - 1.0f));
                        sum += (double)(1.0f / (1.0f + e));
                    } else {
                        const double r = sqrt(r2);
                        const double e = exp(-16.0 * (rs / r - 1.0));
                        sum += 1.0 / (1.0 + e);
                    }
                }
            }
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
        if (lane == 0) {
            cn[i] = ni;
            if (F32) cnf[i] = (float)ni;
        }
        if (lane < MAXREF) {
            double wv = wl[0], wdv = wdl[0];
#pragma unroll
            for (int a = 1; a < MAXREF; a++)
                if (lane == a) { wv = wl[a]; wdv = wdl[a]; }
            w[(size_t)i * MAXREF + lane] = wv;
            wd[(size_t)i * MAXREF + lane] = wdv;
        }
        // projections P_e(i)[a] = sum_b M[e][zi][a][b] w_b
        for (int idx = lane; idx < ne * MAXREF; idx += WAVE) {
            const int e = idx / MAXREF, a = idx - e * MAXREF;
            const double* M = c6ref + ((size_t)(e * MAXELEM + zi) * MAXREF + a) * MAXREF;
            double v = 0.0;
#pragma unroll
            for (int b = 0; b < MAXREF; b++) v = fma(M[b], wl[b], v);
            if (a >= tab->n_ref[e]) v = 0.0;
            const size_t o = ((size_t)e * n + i) * MAXREF + a;
            if (F32) Pf[o] = (float)v;
            else P[o] = v;
        }
    }
}

// ----------------------------------------------------- dispersion pass --

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

template <bool F32>
__global__ void __launch_bounds__(BLOCK)
k_pair(int n, const double4* __restrict__ pos_s, const double4* __restrict__ img_tab,
       int img_bits, const uint32_t* __restrict__ list_p, const int* __restrict__ cnt_p,
       int cap_p, const ElemTab* __restrict__ tab, const double4* __restrict__ pc,
       PairScal sc, const double* __restrict__ w, const double* __restrict__ wd,
       const double* __restrict__ P, const float* __restrict__ Pf,
       double* __restrict__ Fp, double* __restrict__ U, double* __restrict__ G,
       double* __restrict__ vpart)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
    const int nwaves = (gridDim.x * blockDim.x) / WAVE;
    const uint32_t img_mask = (1u << img_bits) - 1u;
    double vir[6] = {0, 0, 0, 0, 0, 0};
    for (int i = wave; i < n; i += nwaves) {
        const double4 pi = pos_s[i];
        const int zi = __builtin_amdgcn_readfirstlane(zbits(pi.w));
        const int K = tab->n_ref[zi];
        double wi[MAXREF], wdi[MAXREF];
#pragma unroll
        for (int a = 0; a < MAXREF; a++) {
            wi[a] = w[(size_t)i * MAXREF + a];
            wdi[a] = wd[(size_t)i * MAXREF + a];
        }
        const double4* pcz = pc + zi * MAXELEM;
        const int cnt = cnt_p[i];
        const uint32_t* lp = list_p + (size_t)i * cap_p;
        double fx = 0.0, fy = 0.0, fz = 0.0, u = 0.0, g = 0.0;
        for (int k0 = 0; k0 < cnt; k0 += WAVE) {
            const int k = k0 + lane;
            if (k < cnt) {
                const uint32_t code = lp[k];
                const int j = (int)(code >> img_bits);
                const double4 pj = pos_s[j];
                const double4 T = img_tab[code & img_mask];
                const double dx = pj.x + T.x - pi.x;
                const double dy = pj.y + T.y - pi.y;
                const double dz = pj.z + T.z - pi.z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < sc.rp2) {
                    const double4 c = pcz[zbits(pj.w)];  // Rd^6, Rd^8, R0^2
                    if (!F32) {
                        const double* Pr = P + ((size_t)zi * n + j) * MAXREF;
                        double c6 = 0.0, dc6 = 0.0;
#pragma unroll
                        for (int a = 0; a < MAXREF; a++)
                            if (a < K) {
                                const double p = Pr[a];
                                c6 = fma(wi[a], p, c6);
                                dc6 = fma(wdi[a], p, dc6);
                            }
                        const double r4 = r2 * r2, r6 = r4 * r2, r8 = r4 * r4;
                        const double A = r6 + c.x, B = r8 + c.y;
                        const double inv = 1.0 / (A * B);
                        const double t6 = B * inv, t8 = A * inv;
                        const double a6 = sc.s6 * t6, a8 = sc.s8 * c.z * t8;
                        const double gg = a6 + a8;  // -dphi/dC6
                        const double dphi_r = c6 * (6.0 * a6 * r4 * t6 + 8.0 * a8 * r6 * t8);
                        u = fma(-0.5 * c6, gg, u);
                        g = fma(-gg, dc6, g);
                        fx = fma(dphi_r, dx, fx);
                        fy = fma(dphi_r, dy, fy);
                        fz = fma(dphi_r, dz, fz);
                        virial_add(vir, -0.5 * dphi_r, dx, dy, dz);
                    } else {
                        const float* Pr = Pf + ((size_t)zi * n + j) * MAXREF;
                        float c6 = 0.0f, dc6 = 0.0f;
#pragma unroll
                        for (int a = 0; a < MAXREF; a++)
                            if (a < K) {
                                const float p = Pr[a];
                                c6 = fmaf((float)wi[a], p, c6);
                                dc6 = fmaf((float)wdi[a], p, dc6);
                            }
                        const float fx2 = (float)dx, fy2 = (float)dy, fz2 = (float)dz;
                        const float q2 = (float)r2;
                        const float r4 = q2 * q2, r6 = r4 * q2, r8 = r4 * r4;
                        const float A = r6 + (float)c.x, B = r8 + (float)c.y;
                        const float t6 = __frcp_rn(A), t8 = __frcp_rn(B);
                        const float a6 = (float)sc.s6 * t6;
                        const float a8 = (float)(sc.s8 * c.z) * t8;
                        const float gg = a6 + a8;
                        const float dphi_r = c6 * (6.0f * a6 * r4 * t6 + 8.0f * a8 * r6 * t8);
                        u += (double)(-0.5f * c6 * gg);
                        g += (double)(-gg * dc6);
                        fx += (double)(dphi_r * fx2);
                        fy += (double)(dphi_r * fy2);
                        fz += (double)(dphi_r * fz2);
                        const float h = -0.5f * dphi_r;
                        const float hx = h * fx2, hy = h * fy2;
                        vir[0] += (double)(hx * fx2);
                        vir[1] += (double)(hx * fy2);
                        vir[2] += (double)(hx * fz2);
                        vir[3] += (double)(hy * fy2);
                        vir[4] += (double)(hy * fz2);
                        vir[5] += (double)(h * fz2 * fz2);
                    }
                }
            }
        }
        fx = wave_sum(fx);
        fy = wave_sum(fy);
        fz = wave_sum(fz);
        u = wave_sum(u);
        g = wave_sum(g);
        if (lane == 0) {
            Fp[3 * (size_t)i] = fx;
            Fp[3 * (size_t)i + 1] = fy;
            Fp[3 * (size_t)i + 2] = fz;
            U[i] = u;
            G[i] = g;
        }
    }
#pragma unroll
    for (int c = 0; c < 6; c++) {
        const double v = wave_sum(vir[c]);
        if (lane == 0) vpart[(size_t)wave * 6 + c] = v;
    }
}

// ---------------------------------------------------------- chain pass --

template <bool F32>
__global__ void __launch_bounds__(BLOCK)
k_chain(int n, const double4* __restrict__ pos_s, const double4* __restrict__ img_tab,
        int img_bits, const uint32_t* __restrict__ list_c, const int* __restrict__ cnt_c,
        int cap_c, const ElemTab* __restrict__ tab, double rc2,
        const double* __restrict__ G, const double* __restrict__ Fp,
        const double* __restrict__ U, const int* __restrict__ perm,
        double* __restrict__ forces, double* __restrict__ atom_energy,
        int accumulate, double* __restrict__ vpart)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
    const int nwaves = (gridDim.x * blockDim.x) / WAVE;
    const uint32_t img_mask = (1u << img_bits) - 1u;
    double vir[6] = {0, 0, 0, 0, 0, 0};
    for (int i = wave; i < n; i += nwaves) {
        const double4 pi = pos_s[i];
        const int zi = __builtin_amdgcn_readfirstlane(zbits(pi.w));
        const double rci = tab->rcov[zi];
        const double gi = G[i];
        const int cnt = cnt_c[i];
        const uint32_t* lc = list_c + (size_t)i * cap_c;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int k0 = 0; k0 < cnt; k0 += WAVE) {
            const int k = k0 + lane;
            if (k < cnt) {
                const uint32_t code = lc[k];
                const int j = (int)(code >> img_bits);
                const double4 pj = pos_s[j];
                const double4 T = img_tab[code & img_mask];
                const double dx = pj.x + T.x - pi.x;
                const double dy = pj.y + T.y - pi.y;
                const double dz = pj.z + T.z - pi.z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < rc2) {
                    const double rs = rci + tab->rcov[zbits(pj.w)];
                    const double gs = gi + G[j];
                    if (F32) {
                        const float q2 = (float)r2;
                        const float r = sqrtf(q2);
                        const float e = __expf(-16.0f * ((float)rs / r - 1.0f));
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
                    } else {
                        const double r = sqrt(r2);
                        const double e = exp(-16.0 * (rs / r - 1.0));
                        const double ope = 1.0 + e;
                        const double coef = gs * (-16.0 * rs * e / (r2 * r * ope * ope));
                        fx = fma(coef, dx, fx);
                        fy = fma(coef, dy, fy);
                        fz = fma(coef, dz, fz);
                        virial_add(vir, -0.5 * coef, dx, dy, dz);
                    }
                }
            }
        }
        fx = wave_sum(fx);
        fy = wave_sum(fy);
        fz = wave_sum(fz);
        if (lane == 0) {
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
        }
    }
#pragma unroll
    for (int c = 0; c < 6; c++) {
        const double v = wave_sum(vir[c]);
        if (lane == 0) vpart[(size_t)wave * 6 + c] = v;
    }
}

// ---------------------------------------------------------- reductions --

__global__ void __launch_bounds__(1024)
k_reduce(int n, const double* __restrict__ U, int nparts,
         const double* __restrict__ vpart, const double* __restrict__ vpart2,
         double* __restrict__ energy, double* __restrict__ virial, int accumulate)
{
    __shared__ double sh[7][1024];
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < n; i += 1024) acc[0] += U[i];
    for (int p = threadIdx.x; p < nparts; p += 1024)
        for (int c = 0; c < 6; c++) acc[1 + c] += vpart[(size_t)p * 6 + c] + vpart2[(size_t)p * 6 + c];
    for (int c = 0; c < 7; c++) sh[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int c = 0; c < 7; c++) sh[c][threadIdx.x] += sh[c][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double e = sh[0][0];
        const double v[9] = {sh[1][0], sh[2][0], sh[3][0], sh[2][0], sh[4][0],
                             sh[5][0], sh[3][0], sh[5][0], sh[6][0]};
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

// ----------------------------------------------------------- launchers --

void launch_cn(int mode, int n, const double4* pos_s, const double4* img_tab,
               int img_bits, const uint32_t* list_c, const int* cnt_c,
               int cap_c, const ElemTab* tab, const double* c6ref,
               double rc2, double* cn, double* w, double* wd, double* P,
               float* Pf, float* cnf, hipStream_t s)
{
    if (n <= 0) return;
    const int waves = pass_waves(n);
    const dim3 grid(nblk(waves, WAVES_PER_BLOCK));
    if (mode == D3_MODE_PREC_F32)
        hipLaunchKernelGGL(k_cn<true>, grid, dim3(BLOCK), 0, s, n, pos_s, img_tab,
                           img_bits, list_c, cnt_c, cap_c, tab, c6ref, rc2, cn,
                           w, wd, P, Pf, cnf);
    else
        hipLaunchKernelGGL(k_cn<false>, grid, dim3(BLOCK), 0, s, n, pos_s, img_tab,
                           img_bits, list_c, cnt_c, cap_c, tab, c6ref, rc2, cn,
                           w, wd, P, Pf, cnf);
}

void launch_pair(int mode, int n, const double4* pos_s,
                 const double4* img_tab, int img_bits,
                 const uint32_t* list_p, const int* cnt_p, int cap_p,
                 const ElemTab* tab, const double4* pc, PairScal sc,
                 const double* w, const double* wd, const double* P,
                 const float* Pf, double* Fp, double* U, double* G,
                 double* vpart, hipStream_t s)
{
    if (n <= 0) return;
    const int waves = pass_waves(n);
    const dim3 grid(nblk(waves, WAVES_PER_BLOCK));
    if (mode == D3_MODE_PREC_F32)
        hipLaunchKernelGGL(k_pair<true>, grid, dim3(BLOCK), 0, s, n, pos_s, img_tab,
                           img_bits, list_p, cnt_p, cap_p, tab, pc, sc, w, wd, P,
                           Pf, Fp, U, G, vpart);
    else
        hipLaunchKernelGGL(k_pair<false>, grid, dim3(BLOCK), 0, s, n, pos_s, img_tab,
                           img_bits, list_p, cnt_p, cap_p, tab, pc, sc, w, wd, P,
                           Pf, Fp, U, G, vpart);
}

void launch_chain(int mode, int n, const double4* pos_s,
                  const double4* img_tab, int img_bits,
                  const uint32_t* list_c, const int* cnt_c, int cap_c,
                  const ElemTab* tab, double rc2, const double* G,
                  const double* Fp, const double* U, const int* perm,
                  double* forces, double* atom_energy, int accumulate,
                  double* vpart, hipStream_t s)
{
    if (n <= 0) return;
    const int waves = pass_waves(n);
    const dim3 grid(nblk(waves, WAVES_PER_BLOCK));
    if (mode == D3_MODE_PREC_F32)
        hipLaunchKernelGGL(k_chain<true>, grid, dim3(BLOCK), 0, s, n, pos_s, img_tab,
                           img_bits, list_c, cnt_c, cap_c, tab, rc2, G, Fp, U,
                           perm, forces, atom_energy, accumulate, vpart);
    else
        hipLaunchKernelGGL(k_chain<false>, grid, dim3(BLOCK), 0, s, n, pos_s, img_tab,
                           img_bits, list_c, cnt_c, cap_c, tab, rc2, G, Fp, U,
                           perm, forces, atom_energy, accumulate, vpart);
}

void launch_reduce(int n, const double* U, int nparts, const double* vpart,
                   const double* vpart2, double* energy, double* virial,
                   int accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(1024), 0, s, n, U, nparts, vpart,
                       vpart2, energy, virial, accumulate);
}

void launch_scatter_out(int n, const double* src, const int* perm,
                        double* dst, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scatter_out, dim3(nblk(n, BLOCK)), dim3(BLOCK), 0, s, n,
                       src, perm, dst);
}

}  // namespace d3
