// Learned C6 surrogate: a per-element-pair multilayer perceptron that maps
// the two coordination numbers to (C6, dC6/dn_i, dC6/dn_j) of Eq. 3.  It is
// not part of the paper; it approximates Eq. 3, is trained on samples that
// the exact interpolation labels, and exact Eq. 3 stays both the fallback
// (coordination numbers outside the trained box) and the reference its
// error is measured against.
//
// Network, per unordered element pair (e <= f), row-vector convention,
// inputs x = 2 n / cn_hi - 1:
//   h1 = silu(x W1 + b1)   2 -> 32
//   h2 = silu(h1 W2 + b2)  32 -> 32
//   y  = h2 W3 + b3        32 -> 3, y = standardised (C6, dC6/dn_e, dC6/dn_f)
// A query whose first atom has the larger element uses the pair's network
// with its inputs swapped and its two derivative outputs swapped back.
//
// Training (FP32): one workgroup per element pair, one sample per thread,
// 256 samples per step drawn with a counter-based hash, mean-squared error
// on standardised targets, gradients by backpropagation with the per-sample
// activations in LDS, Adam with a cosine step-size decay.
//
// Inference: layer 1 and the SiLUs on the vector ALU in FP32; the 32x32
// layer as v_mfma_f32_32x32x16_bf16 with FP32 accumulation (64 queries per
// wave as two 32-row tiles); layer 3 in FP32.  The BF16 operands are split
// into a high and a low BF16 part, and three products (hi*hi, hi*lo,
// lo*hi) recover close to FP32 accuracy for the layer.
#include <cmath>
#include <cstring>
#include <vector>

#include "d3_ctx.h"
#include "d3_device.h"

namespace d3 {

constexpr int H = D3_MLP_HIDDEN;
constexpr int NPAR = D3_MLP_PARAMS;
constexpr int OW1 = 0, OB1 = 2 * H, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H,
              OB3 = OW3 + 3 * H;
static_assert(OB3 + 3 == NPAR, "parameter layout");
constexpr int SM_W1 = 0, SM_B1 = 2 * H, SM_B2 = 3 * H, SM_W3 = 4 * H, SM_B3 = 7 * H;
constexpr int SMALL = 7 * H + 4;  // W1, b1, b2, W3, b3 (+pad) per pair, FP32
constexpr int TB = 256;           // training samples per pair per step
constexpr int SUR_CAP = 448;      // list entries per atom sorted in LDS at a time
constexpr int MAXPAIR = MAXELEM * (MAXELEM + 1) / 2;
constexpr int SUR_ELEM = 8;       // elements the surrogate dispersion pass supports
constexpr int SUR_PAIR = SUR_ELEM * (SUR_ELEM + 1) / 2;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__host__ __device__ inline int pair_index(int e, int f, int ne)
{
    return e * ne - e * (e - 1) / 2 + (f - e);
}

// splitmix64 finaliser (Steele, Lea & Flood 2014) as a counter-based hash
__host__ __device__ inline uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline double u01(uint64_t seed, uint64_t a, uint64_t b)
{
    return (double)(mix64(seed ^ mix64(a * 0x9E3779B97F4A7C15ull + b)) >> 11) *
           (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ float sigm(float z) { return __frcp_rn(1.0f + __expf(-z)); }

// ----------------------------------------------------------- exact Eq. 3 --

__device__ void gauss_weights(const ElemTab* tab, int z, double n, double* w, double* wd)
{
    const int K = tab->n_ref[z];
    double dl[MAXREF], m = 1e300;
#pragma unroll
    for (int a = 0; a < MAXREF; a++) {
        dl[a] = n - tab->cn_ref[z * MAXREF + a];
        if (a < K) m = fmin(m, dl[a] * dl[a]);
    }
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < MAXREF; a++) {
        w[a] = (a < K) ? exp(-4.0 * (dl[a] * dl[a] - m)) : 0.0;
        s += w[a];
    }
    const double is = 1.0 / s;
    double mean = 0.0;
#pragma unroll
    for (int a = 0; a < MAXREF; a++) {
        w[a] *= is;
        mean += w[a] * dl[a];
    }
#pragma unroll
    for (int a = 0; a < MAXREF; a++) wd[a] = (a < K) ? -8.0 * w[a] * (dl[a] - mean) : 0.0;
}

// C6 of Eq. 3 and its two CN derivatives from the factorised weights (FP64)
__device__ void exact_c6(const ElemTab* tab, const double* __restrict__ c6ref, int zi, int zj,
                         double ni, double nj, double* out)
{
    double wi[MAXREF], wdi[MAXREF], wj[MAXREF], wdj[MAXREF];
    gauss_weights(tab, zi, ni, wi, wdi);
    gauss_weights(tab, zj, nj, wj, wdj);
    const double* M = c6ref + (size_t)(zi * MAXELEM + zj) * MAXREF * MAXREF;
    double c = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
    for (int a = 0; a < MAXREF; a++) {
        double t = 0.0, td = 0.0;
#pragma unroll
        for (int b = 0; b < MAXREF; b++) {
            t = fma(M[a * MAXREF + b], wj[b], t);
            td = fma(M[a * MAXREF + b], wdj[b], td);
        }
        c = fma(wi[a], t, c);
        d1 = fma(wdi[a], t, d1);
        d2 = fma(wi[a], td, d2);
    }
    out[0] = c;
    out[1] = d1;
    out[2] = d2;
}

// exact_c6 behind a call, so that its registers do not count against the
// surrogate dispersion pass, which needs it only for CNs outside the box
__device__ __noinline__ double2 exact_c6_call(const ElemTab* tab, const double* __restrict__ c6ref,
                                             int zi, int zj, double ni, double nj)
{
    double ex[3];
    exact_c6(tab, c6ref, zi, zj, ni, nj, ex);
    return make_double2(ex[0], ex[1]);
}

__global__ void __launch_bounds__(BLOCK)
k_exact_eval(int m, const int32_t* __restrict__ ei, const int32_t* __restrict__ ej,
             const double* __restrict__ ni, const double* __restrict__ nj,
             const ElemTab* __restrict__ tab, const double* __restrict__ c6ref,
             double* __restrict__ out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= m) return;
    const int ne = tab->n_elem;
    int a = ei[q], b = ej[q];
    a = (a < 0 || a >= ne) ? 0 : a;
    b = (b < 0 || b >= ne) ? 0 : b;
    double r[3];
    exact_c6(tab, c6ref, a, b, ni[q], nj[q], r);
    out[3 * (size_t)q] = r[0];
    out[3 * (size_t)q + 1] = r[1];
    out[3 * (size_t)q + 2] = r[2];
}

// -------------------------------------------------------- training data --

__global__ void __launch_bounds__(BLOCK)
k_samples(int n_pairs, int n_per, uint64_t seed, double cn_hi, const int* __restrict__ pe,
          const int* __restrict__ pf, const ElemTab* __restrict__ tab,
          const double* __restrict__ c6ref, float* __restrict__ X, double* __restrict__ Yd)
{
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (long)n_pairs * n_per) return;
    const int p = (int)(g / n_per);
    const double u1 = u01(seed, (uint64_t)g, 0), u2 = u01(seed, (uint64_t)g, 1);
    double r[3];
    exact_c6(tab, c6ref, pe[p], pf[p], u1 * cn_hi, u2 * cn_hi, r);
    X[2 * g] = (float)(2.0 * u1 - 1.0);
    X[2 * g + 1] = (float)(2.0 * u2 - 1.0);
    Yd[3 * g] = r[0];
    Yd[3 * g + 1] = r[1];
    Yd[3 * g + 2] = r[2];
}

// per pair: mean and standard deviation of each output; targets
// standardised with them
__global__ void __launch_bounds__(BLOCK)
k_standardise(int n_per, const double* __restrict__ Yd, float* __restrict__ Y,
              float* __restrict__ stats)
{
    __shared__ double sh[6][BLOCK];
    const int p = blockIdx.x;
    const double* y = Yd + (size_t)p * n_per * 3;
    double s[3] = {0, 0, 0}, q[3] = {0, 0, 0};
    for (int i = threadIdx.x; i < n_per; i += BLOCK)
        for (int o = 0; o < 3; o++) {
            const double v = y[3 * (size_t)i + o];
            s[o] += v;
            q[o] += v * v;
        }
    for (int o = 0; o < 3; o++) {
        sh[o][threadIdx.x] = s[o];
        sh[3 + o][threadIdx.x] = q[o];
    }
    __syncthreads();
    for (int off = BLOCK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int c = 0; c < 6; c++) sh[c][threadIdx.x] += sh[c][threadIdx.x + off];
        __syncthreads();
    }
    double mean[3], scale[3];
    for (int o = 0; o < 3; o++) {
        mean[o] = sh[o][0] / n_per;
        const double var = sh[3 + o][0] / n_per - mean[o] * mean[o];
        scale[o] = var > 1e-20 ? sqrt(var) : 1.0;
    }
    if (threadIdx.x == 0)
        for (int o = 0; o < 3; o++) {
            stats[6 * p + o] = (float)mean[o];
            stats[6 * p + 3 + o] = (float)scale[o];
        }
    for (int i = threadIdx.x; i < n_per; i += BLOCK)
        for (int o = 0; o < 3; o++)
            Y[((size_t)p * n_per + i) * 3 + o] =
                (float)((y[3 * (size_t)i + o] - mean[o]) / scale[o]);
}

// ------------------------------------------------------------- training --

struct TrainLds {
    float w[NPAR + 1];
    float x[TB][2];
    float h1[TB][H + 1];
    float h2[TB][H + 1];
    float dz1[TB][H + 1];
    float dz2[TB][H + 1];
    float dy[TB][3];
    float red[TB / WAVE];
};

// forward and backward pass of one sample per thread; activations and
// output-side gradients go to LDS; returns the squared error of the sample
__device__ float fwd_bwd(TrainLds& L, float x0, float x1, const float* tg, bool active, float norm)
{
    const int t = threadIdx.x;
    float h1[H], d1[H];
#pragma unroll
    for (int k = 0; k < H; k++) {
        const float z = fmaf(x0, L.w[OW1 + k], fmaf(x1, L.w[OW1 + H + k], L.w[OB1 + k]));
        const float s = sigm(z);
        h1[k] = z * s;
        d1[k] = s * (1.0f + z * (1.0f - s));
        L.h1[t][k] = h1[k];
    }
    float h2[H], d2[H];
#pragma unroll 4
    for (int m = 0; m < H; m++) {
        float z = L.w[OB2 + m];
#pragma unroll
        for (int k = 0; k < H; k++) z = fmaf(h1[k], L.w[OW2 + k * H + m], z);
        const float s = sigm(z);
        h2[m] = z * s;
        d2[m] = s * (1.0f + z * (1.0f - s));
        L.h2[t][m] = h2[m];
    }
    float r[3], se = 0.0f;
#pragma unroll
    for (int o = 0; o < 3; o++) {
        float y = L.w[OB3 + o];
#pragma unroll
        for (int m = 0; m < H; m++) y = fmaf(h2[m], L.w[OW3 + m * 3 + o], y);
        r[o] = active ? y - tg[o] : 0.0f;
        se += r[o] * r[o];
        L.dy[t][o] = 2.0f * r[o] * norm;
    }
    float dz2[H];
#pragma unroll
    for (int m = 0; m < H; m++) {
        float g = 0.0f;
#pragma unroll
        for (int o = 0; o < 3; o++) g = fmaf(L.dy[t][o], L.w[OW3 + m * 3 + o], g);
        dz2[m] = g * d2[m];
        L.dz2[t][m] = dz2[m];
    }
#pragma unroll 4
    for (int k = 0; k < H; k++) {
        float g = 0.0f;
#pragma unroll
        for (int m = 0; m < H; m++) g = fmaf(dz2[m], L.w[OW2 + k * H + m], g);
        L.dz1[t][k] = g * d1[k];
    }
    L.x[t][0] = x0;
    L.x[t][1] = x1;
    return se;
}

// gradient of parameter q summed over the block's samples (after fwd_bwd
// and a barrier)
__device__ float grad_param(const TrainLds& L, int q)
{
    float g = 0.0f;
    if (q < OB1) {
        const int i = q / H, k = q - i * H;
        for (int s = 0; s < TB; s++) g = fmaf(L.x[s][i], L.dz1[s][k], g);
    } else if (q < OW2) {
        const int k = q - OB1;
        for (int s = 0; s < TB; s++) g += L.dz1[s][k];
    } else if (q < OB2) {
        const int k = (q - OW2) / H, m = (q - OW2) - k * H;
        for (int s = 0; s < TB; s++) g = fmaf(L.h1[s][k], L.dz2[s][m], g);
    } else if (q < OW3) {
        const int m = q - OB2;
        for (int s = 0; s < TB; s++) g += L.dz2[s][m];
    } else if (q < OB3) {
        const int m = (q - OW3) / 3, o = (q - OW3) - m * 3;
        for (int s = 0; s < TB; s++) g = fmaf(L.h2[s][m], L.dy[s][o], g);
    } else {
        const int o = q - OB3;
        for (int s = 0; s < TB; s++) g += L.dy[s][o];
    }
    return g;
}

__device__ float block_sum_f(TrainLds& L, float v)
{
    v = wave_sum(v);
    if ((threadIdx.x & (WAVE - 1)) == 0) L.red[threadIdx.x / WAVE] = v;
    __syncthreads();
    float s = 0.0f;
    for (int w = 0; w < TB / WAVE; w++) s += L.red[w];
    __syncthreads();
    return s;
}

constexpr int PPT = (NPAR + TB - 1) / TB;  // parameters owned per thread

// Step size of training step gs (0-based) of total: cosine decay from lr0
// at step 0 to lr1 at step total.
__device__ __forceinline__ float cosine_lr(int gs, int total, float lr0, float lr1)
{
    return lr1 + 0.5f * (lr0 - lr1) * (1.0f + cosf(3.14159265f * (float)gs / (float)total));
}

// Adam (Kingma & Ba) for the parameters this thread owns (q = t + r TB):
// first and second moments am, av updated with gradient g, then the bias-
// corrected step of size lr for training step gs (0-based, so the bias
// corrections use gs + 1).  Writes the new weights to wn (L.w is left for
// the caller to overwrite once every thread has read it).
__device__ __forceinline__ void adam_update(const TrainLds& L, const float* g, float* am,
                                            float* av, float* wn, int gs, float lr)
{
    const float bc1 = 1.0f - powf(0.9f, (float)(gs + 1));
    const float bc2 = 1.0f - powf(0.999f, (float)(gs + 1));
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < PPT; r++) {
        const int q = t + r * TB;
        wn[r] = 0.0f;
        if (q < NPAR) {
            am[r] = 0.9f * am[r] + 0.1f * g[r];
            av[r] = 0.999f * av[r] + 0.001f * g[r] * g[r];
            wn[r] = L.w[q] - lr * (am[r] / bc1) / (sqrtf(av[r] / bc2) + 1e-8f);
        }
    }
}

__global__ void __launch_bounds__(TB)
k_train(int n_per, const float* __restrict__ X, const float* __restrict__ Y,
        float* __restrict__ Wg, float* __restrict__ Mg, float* __restrict__ Vg, int step0,
        int n_steps, int total_steps, float lr0, float lr1, uint64_t seed,
        float* __restrict__ loss_out)
{
    __shared__ TrainLds L;
    const int p = blockIdx.x, t = threadIdx.x;
    float* W = Wg + (size_t)p * NPAR;
    for (int q = t; q < NPAR; q += TB) L.w[q] = W[q];
    float am[PPT], av[PPT];
#pragma unroll
    for (int r = 0; r < PPT; r++) {
        const int q = t + r * TB;
        am[r] = q < NPAR ? Mg[(size_t)p * NPAR + q] : 0.0f;
        av[r] = q < NPAR ? Vg[(size_t)p * NPAR + q] : 0.0f;
    }
    __syncthreads();
    const float norm = 1.0f / (3.0f * TB);
    for (int st = 0; st < n_steps; st++) {
        const int gs = step0 + st;
        const uint64_t key = ((uint64_t)p * (uint64_t)total_steps + (uint64_t)gs) * TB + t;
        const int idx = (int)(mix64(seed ^ mix64(key)) % (uint64_t)n_per);
        const size_t s = (size_t)p * n_per + idx;
        const float tg[3] = {Y[3 * s], Y[3 * s + 1], Y[3 * s + 2]};
        const float se = fwd_bwd(L, X[2 * s], X[2 * s + 1], tg, true, norm);
        __syncthreads();
        float gr[PPT], wn[PPT];
#pragma unroll
        for (int r = 0; r < PPT; r++) {
            const int q = t + r * TB;
            gr[r] = q < NPAR ? grad_param(L, q) : 0.0f;
        }
        adam_update(L, gr, am, av, wn, gs, cosine_lr(gs, total_steps, lr0, lr1));
        const float tot = block_sum_f(L, se);  // includes a barrier: all reads done
#pragma unroll
        for (int r = 0; r < PPT; r++) {
            const int q = t + r * TB;
            if (q < NPAR) L.w[q] = wn[r];
        }
        if (t == 0) loss_out[(size_t)p * n_steps + st] = tot * norm;
        __syncthreads();
    }
    for (int q = t; q < NPAR; q += TB) W[q] = L.w[q];
#pragma unroll
    for (int r = 0; r < PPT; r++) {
        const int q = t + r * TB;
        if (q < NPAR) {
            Mg[(size_t)p * NPAR + q] = am[r];
            Vg[(size_t)p * NPAR + q] = av[r];
        }
    }
}

// Mean-squared-error gradient of pair p's network (the block's) over the
// explicit samples whose pair index is p, summed into gacc (parameters
// q = t + r TB of this thread) and normalised by 1/(3 m_p); returns this
// thread's share of the squared error and sets *mp_out = m_p.
__device__ float pair_gradient(TrainLds& L, int* s_cnt, int m, const int32_t* __restrict__ pair,
                               const float* __restrict__ X, const float* __restrict__ Y,
                               float* gacc, int* mp_out)
{
    const int p = blockIdx.x, t = threadIdx.x;
    if (t == 0) *s_cnt = 0;
    __syncthreads();
    int c = 0;
    for (int s = t; s < m; s += TB) c += pair[s] == p ? 1 : 0;
    atomicAdd(s_cnt, c);
    __syncthreads();
    const int mp = *s_cnt;
#pragma unroll
    for (int r = 0; r < PPT; r++) gacc[r] = 0.0f;
    float sse = 0.0f;
    const float norm = mp > 0 ? 1.0f / (3.0f * mp) : 0.0f;
    for (int s0 = 0; s0 < m; s0 += TB) {
        const int s = s0 + t;
        const bool act = s < m && pair[s] == p;
        const int sc = s < m ? s : 0;
        const float tg[3] = {Y[3 * (size_t)sc], Y[3 * (size_t)sc + 1], Y[3 * (size_t)sc + 2]};
        sse += fwd_bwd(L, act ? X[2 * (size_t)sc] : 0.0f, act ? X[2 * (size_t)sc + 1] : 0.0f,
                       tg, act, norm);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < PPT; r++) {
            const int q = t + r * TB;
            if (q < NPAR) gacc[r] += grad_param(L, q);
        }
        __syncthreads();
    }
    *mp_out = mp;
    return sse;
}

// mean-squared-error gradient of every pair's network on explicit samples
// (no update); one workgroup per pair walks all samples
__global__ void __launch_bounds__(TB)
k_grad(int m, const int32_t* __restrict__ pair, const float* __restrict__ X,
       const float* __restrict__ Y, const float* __restrict__ Wg, float* __restrict__ grads,
       float* __restrict__ loss)
{
    __shared__ TrainLds L;
    __shared__ int s_cnt;
    const int p = blockIdx.x, t = threadIdx.x;
    for (int q = t; q < NPAR; q += TB) L.w[q] = Wg[(size_t)p * NPAR + q];
    float gacc[PPT];
    int mp = 0;
    const float sse = pair_gradient(L, &s_cnt, m, pair, X, Y, gacc, &mp);
#pragma unroll
    for (int r = 0; r < PPT; r++) {
        const int q = t + r * TB;
        if (q < NPAR) grads[(size_t)p * NPAR + q] = gacc[r];
    }
    const float tot = block_sum_f(L, sse);
    if (t == 0 && m > 0) atomicAdd(loss, tot / (3.0f * m));
}

// One training step on explicit samples: the gradient of k_grad, then the
// Adam update and cosine step size of k_train for step gs of total, on the
// weights and moments in global memory.  Pairs without samples keep their
// weights and moments.
__global__ void __launch_bounds__(TB)
k_adam_step(int m, const int32_t* __restrict__ pair, const float* __restrict__ X,
            const float* __restrict__ Y, float* __restrict__ Wg, float* __restrict__ Mg,
            float* __restrict__ Vg, int gs, int total, float lr0, float lr1)
{
    __shared__ TrainLds L;
    __shared__ int s_cnt;
    const int p = blockIdx.x, t = threadIdx.x;
    for (int q = t; q < NPAR; q += TB) L.w[q] = Wg[(size_t)p * NPAR + q];
    float gacc[PPT], am[PPT], av[PPT], wn[PPT];
    int mp = 0;
    (void)pair_gradient(L, &s_cnt, m, pair, X, Y, gacc, &mp);
    if (mp == 0) return;
#pragma unroll
    for (int r = 0; r < PPT; r++) {
        const int q = t + r * TB;
        am[r] = q < NPAR ? Mg[(size_t)p * NPAR + q] : 0.0f;
        av[r] = q < NPAR ? Vg[(size_t)p * NPAR + q] : 0.0f;
    }
    adam_update(L, gacc, am, av, wn, gs, cosine_lr(gs, total, lr0, lr1));
#pragma unroll
    for (int r = 0; r < PPT; r++) {
        const int q = t + r * TB;
        if (q < NPAR) {
            Wg[(size_t)p * NPAR + q] = wn[r];
            Mg[(size_t)p * NPAR + q] = am[r];
            Vg[(size_t)p * NPAR + q] = av[r];
        }
    }
}

// ------------------------------------------------------------ inference --

// FP32 reference forward of one query (weights from global memory)
__device__ void mlp_ref(const float* __restrict__ w, float x0, float x1, float* y)
{
    float h1[H];
#pragma unroll
    for (int k = 0; k < H; k++) {
        const float z = fmaf(x0, w[OW1 + k], fmaf(x1, w[OW1 + H + k], w[OB1 + k]));
        h1[k] = z * sigm(z);
    }
    float acc[3] = {w[OB3], w[OB3 + 1], w[OB3 + 2]};
    for (int m = 0; m < H; m++) {
        float z = w[OB2 + m];
#pragma unroll
        for (int k = 0; k < H; k++) z = fmaf(h1[k], w[OW2 + k * H + m], z);
        const float h = z * sigm(z);
#pragma unroll
        for (int o = 0; o < 3; o++) acc[o] = fmaf(h, w[OW3 + m * 3 + o], acc[o]);
    }
    y[0] = acc[0];
    y[1] = acc[1];
    y[2] = acc[2];
}

__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }

// One network on 64 queries of a wave (lane l = query l), all lanes
// active.  Tile 0 holds queries 0..31, tile 1 queries 32..63; lane l works
// on row l % 32 of both tiles and on hidden units 8h..8h+7, 16+8h..16+8h+7
// (h = l / 32), which is the B-operand layout of v_mfma_f32_32x32x16_bf16.
// sm: the pair's FP32 small weights (W1, b1, b2, W3, b3); a_hi/a_lo: this
// lane's A operands (W2 transposed, split into BF16 high and low parts) for
// the two 16-wide K blocks.
__device__ void mlp64(float x0, float x1, const float* sm, const bf16x8* a_hi, const bf16x8* a_lo,
                      float* y)
{
    const int l = threadIdx.x & (WAVE - 1), h = l >> 5;
    const float p0 = __shfl_xor(x0, 32, WAVE), p1 = __shfl_xor(x1, 32, WAVE);
    const float t0x0 = h ? p0 : x0, t0x1 = h ? p1 : x1;  // tile-0 row inputs
    const float t1x0 = h ? x0 : p0, t1x1 = h ? x1 : p1;  // tile-1 row inputs
    bf16x8 b_hi[2][2], b_lo[2][2];  // [tile][K block]
#pragma unroll
    for (int blk = 0; blk < 2; blk++)
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int k = 16 * blk + 8 * h + j;
            const float w0 = sm[SM_W1 + k], w1 = sm[SM_W1 + H + k], bb = sm[SM_B1 + k];
            const float z0 = fmaf(t0x0, w0, fmaf(t0x1, w1, bb));
            const float z1 = fmaf(t1x0, w0, fmaf(t1x1, w1, bb));
            const float a0 = z0 * sigm(z0), a1 = z1 * sigm(z1);
            const __bf16 h0 = to_bf16(a0), h1v = to_bf16(a1);
            b_hi[0][blk][j] = h0;
            b_hi[1][blk][j] = h1v;
            b_lo[0][blk][j] = to_bf16(a0 - (float)h0);
            b_lo[1][blk][j] = to_bf16(a1 - (float)h1v);
        }
    f32x16 d[2];
#pragma unroll
    for (int tt = 0; tt < 2; tt++) {
        f32x16 c = {};
#pragma unroll
        for (int blk = 0; blk < 2; blk++) {
            c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_hi[blk], b_hi[tt][blk], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_hi[blk], b_lo[tt][blk], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a_lo[blk], b_hi[tt][blk], c, 0, 0, 0);
        }
        d[tt] = c;
    }
    // row m of the 32x32 result held in register r of lane l
    float part[2][3] = {{0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const int m = 8 * (r >> 2) + 4 * h + (r & 3);
        const float b2 = sm[SM_B2 + m];
#pragma unroll
        for (int tt = 0; tt < 2; tt++) {
            const float z = d[tt][r] + b2;
            const float a = z * sigm(z);
#pragma unroll
            for (int o = 0; o < 3; o++) part[tt][o] = fmaf(a, sm[SM_W3 + m * 3 + o], part[tt][o]);
        }
    }
    // lane l < 32 owns query l (tile 0), lane l >= 32 owns query l (tile 1)
#pragma unroll
    for (int o = 0; o < 3; o++) {
        const float send = h ? part[0][o] : part[1][o];
        const float recv = __shfl_xor(send, 32, WAVE);
        y[o] = (h ? part[1][o] : part[0][o]) + recv + sm[SM_B3 + o];
    }
}

struct SurView {
    const float* w32;     // master weights [P][NPAR]
    const float* small;   // [P][SMALL]
    const bf16x8* a_hi;   // [P][2][64]
    const bf16x8* a_lo;   // [P][2][64]
    const float* stats;   // [P][6]
    float cn_hi;
    int ne;
};

__device__ __forceinline__ void order_query(int zi, int zj, int ne, int* p, bool* swapped)
{
    *swapped = zi > zj;
    *p = *swapped ? pair_index(zj, zi, ne) : pair_index(zi, zj, ne);
}

__global__ void __launch_bounds__(BLOCK)
k_sur_eval(int m, const int32_t* __restrict__ ei, const int32_t* __restrict__ ej,
           const float* __restrict__ ni, const float* __restrict__ nj, SurView sv, int precision,
           float* __restrict__ out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = q < m;
    const int qc = valid ? q : 0;
    int a = ei[qc], b = ej[qc];
    a = (a < 0 || a >= sv.ne) ? 0 : a;
    b = (b < 0 || b >= sv.ne) ? 0 : b;
    int p;
    bool sw;
    order_query(a, b, sv.ne, &p, &sw);
    const float xa = 2.0f * ni[qc] / sv.cn_hi - 1.0f, xb = 2.0f * nj[qc] / sv.cn_hi - 1.0f;
    const float x0 = sw ? xb : xa, x1 = sw ? xa : xb;
    float y[3] = {0, 0, 0};
    if (precision == 0) {
        mlp_ref(sv.w32 + (size_t)p * NPAR, x0, x1, y);
    } else {
        // one MFMA pass per distinct network among the wave's queries
        uint64_t todo = __ballot(valid);
        while (todo) {
            const int leader = __builtin_ctzll(todo);
            const int pp = __shfl(p, leader, WAVE);
            float yy[3];
            const int l = threadIdx.x & (WAVE - 1);
            bf16x8 ah[2], al[2];
            for (int blk = 0; blk < 2; blk++) {
                ah[blk] = sv.a_hi[((size_t)pp * 2 + blk) * WAVE + l];
                al[blk] = sv.a_lo[((size_t)pp * 2 + blk) * WAVE + l];
            }
            mlp64(x0, x1, sv.small + (size_t)pp * SMALL, ah, al, yy);
            if (p == pp) {
                y[0] = yy[0];
                y[1] = yy[1];
                y[2] = yy[2];
            }
            todo &= ~__ballot(p == pp);
        }
    }
    if (!valid) return;
    const float* st = sv.stats + 6 * p;
    const float c6 = y[0] * st[3] + st[0];
    const float da = y[1] * st[4] + st[1], db = y[2] * st[5] + st[2];
    out[3 * (size_t)q] = c6;
    out[3 * (size_t)q + 1] = sw ? db : da;
    out[3 * (size_t)q + 2] = sw ? da : db;
}

// ---------------------------------------- surrogate dispersion pass ------

// Same sums as the plain dispersion pass (FP32 pair arithmetic, FP64
// accumulation), with C6 and dC6/dn_i from the surrogate.  Each atom's
// list is first sorted by the neighbour's element in LDS, so every 64-entry
// step uses a single network.
// AV: also the direct part of each atom's virial (Eq. 7) to Vp, as in the
// exact dispersion pass.
template <bool IMG, bool AV>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(3)))
k_pair_sur(int n, const double4* __restrict__ pos_s, const double4* __restrict__ img_tab,
           int n_img, int img_bits, const uint32_t* __restrict__ list_p,
           const int* __restrict__ cnt_p, int cap_p, const ElemTab* __restrict__ tab,
           const double* __restrict__ c6ref, const double4* __restrict__ pc, PairScal sc,
           const double* __restrict__ cn, SurView sv, double* __restrict__ Fp,
           double* __restrict__ U, double* __restrict__ G, double* __restrict__ Vp,
           double* __restrict__ part)
{
    __shared__ double4 s_img[IMG ? IMG_LDS : 1];
    __shared__ double4 s_pc[SUR_ELEM * SUR_ELEM];
    __shared__ float s_small[SUR_PAIR * SMALL];
    __shared__ uint32_t s_raw[WAVES_PER_BLOCK][SUR_CAP];
    __shared__ uint32_t s_srt[WAVES_PER_BLOCK][SUR_CAP];
    __shared__ int s_tally[WAVES_PER_BLOCK][SUR_ELEM];
    const int ne = tab->n_elem;  // <= SUR_ELEM (checked on the host)
    const int npair = ne * (ne + 1) / 2;
    load_images<IMG>(s_img, img_tab, n_img);
    for (int k = threadIdx.x; k < SUR_ELEM * SUR_ELEM; k += blockDim.x)
        s_pc[k] = pc[(k / SUR_ELEM) * MAXELEM + (k % SUR_ELEM)];
    for (int k = threadIdx.x; k < npair * SMALL; k += blockDim.x) s_small[k] = sv.small[k];
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    const unsigned long long lanemask = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    const uint32_t img_mask = (1u << img_bits) - 1u;
    const float cn_hi = sv.cn_hi;
    double vir[6] = {0, 0, 0, 0, 0, 0};
    double esum = 0.0;
    const Walk wk = atom_walk(n);
    for (int i = wk.first; i < wk.end; i += wk.step) {
        const double4 pi = pos_s[i];
        const int zi = __builtin_amdgcn_readfirstlane(zbits(pi.w));
        const double ni = cn[i];
        const int cnt_all = min(cnt_p[i], cap_p);
        const uint32_t* row = list_p + (size_t)i * cap_p;
        double fx = 0.0, fy = 0.0, fz = 0.0, ue = 0.0, g = 0.0;
        double av[6] = {0, 0, 0, 0, 0, 0};  // this atom's virial (AV only)
        // the list is taken in chunks of at most SUR_CAP entries
        for (int c0 = 0; c0 < cnt_all; c0 += SUR_CAP) {
            const int cnt = min(cnt_all - c0, SUR_CAP);
            const uint32_t* lp = row + c0;
            const int capr = cap_p - c0;
            // pass 1: codes to LDS, element tallies
            int tally[SUR_ELEM];
#pragma unroll
            for (int f = 0; f < SUR_ELEM; f++) tally[f] = 0;
            for (int k0 = 0; k0 < cnt; k0 += WAVE) {
                const int k = k0 + lane;
                const uint32_t code = list_code(lp, k, cnt, capr);
                const int zj = zbits(pos_s[code >> img_bits].w);
                if (k < cnt) s_raw[wv][k] = code;
#pragma unroll
                for (int f = 0; f < SUR_ELEM; f++)
                    if (f < ne) tally[f] += __popcll(__ballot(k < cnt && zj == f));
            }
            // pass 2: stable partition by element
            int off[SUR_ELEM];
            {
                int o = 0;
#pragma unroll
                for (int f = 0; f < SUR_ELEM; f++) {
                    off[f] = o;
                    o += (f < ne) ? tally[f] : 0;
                    if (lane == 0) s_tally[wv][f] = tally[f];
                }
            }
            __builtin_amdgcn_wave_barrier();
            for (int k0 = 0; k0 < cnt; k0 += WAVE) {
                const int k = k0 + lane;
                const uint32_t code = k < cnt ? s_raw[wv][k] : 0u;
                const int zj = zbits(pos_s[code >> img_bits].w);
#pragma unroll
                for (int f = 0; f < SUR_ELEM; f++) {
                    if (f < ne) {
                        const unsigned long long b = __ballot(k < cnt && zj == f);
                        if (k < cnt && zj == f) s_srt[wv][off[f] + __popcll(b & lanemask)] = code;
                        off[f] += __popcll(b);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            int base = 0;
            for (int f = 0; f < ne; f++) {
                const int cf = __builtin_amdgcn_readfirstlane(s_tally[wv][f]);
                if (cf == 0) continue;
                int p;
                bool sw;
                order_query(zi, f, ne, &p, &sw);
                bf16x8 ah[2], al[2];
                for (int blk = 0; blk < 2; blk++) {
                    ah[blk] = sv.a_hi[((size_t)p * 2 + blk) * WAVE + lane];
                    al[blk] = sv.a_lo[((size_t)p * 2 + blk) * WAVE + lane];
                }
                const float* st = sv.stats + 6 * p;
                const float st0 = st[0], st1 = st[1], st2 = st[2], st3 = st[3], st4 = st[4],
                            st5 = st[5];
                const double4 c = s_pc[zi * SUR_ELEM + f];
                for (int it = 0; it < cf; it += WAVE) {
                    const bool valid = it + lane < cf;
                    const uint32_t code = valid ? s_srt[wv][base + it + lane] : 0u;
                    const uint32_t j = code >> img_bits;
                    const double4 pj = pos_s[j];
                    const double nj = cn[j];
                    const double4 T = image<IMG>(s_img, img_tab, code & img_mask);
                    const double dx = pj.x + T.x - pi.x;
                    const double dy = pj.y + T.y - pi.y;
                    const double dz = pj.z + T.z - pi.z;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    const bool in = valid && r2 < sc.rp2;
                    const float xa = (float)(2.0 * ni / cn_hi - 1.0);
                    const float xb = (float)(2.0 * nj / cn_hi - 1.0);
                    float y[3];
                    // the weights are re-read from LDS every step rather than held in
                    // registers across the loop (an opaque offset keeps them from being
                    // hoisted), which leaves room for three waves per SIMD
                    int smo = p * SMALL;
                    asm volatile("" : "+v"(smo));
                    mlp64(sw ? xb : xa, sw ? xa : xb, s_small + smo, ah, al, y);
                    float c6 = y[0] * st3 + st0;
                    const float da = y[1] * st4 + st1, db = y[2] * st5 + st2;
                    float dc6 = sw ? db : da;
                    if (ni > (double)cn_hi || nj > (double)cn_hi) {
                        // exact Eq. 3 outside the trained box (out of line: rare)
                        const double2 ex = exact_c6_call(tab, c6ref, zi, f, ni, nj);
                        c6 = (float)ex.x;
                        dc6 = (float)ex.y;
                    }
                    c6 = in ? c6 : 0.0f;
                    dc6 = in ? dc6 : 0.0f;
                    const float x = (float)dx, yv = (float)dy, zz = (float)dz;
                    const float q2 = (float)r2;
                    const float r4 = q2 * q2, r6 = r4 * q2, r8 = r4 * r4;
                    const float t6 = __frcp_rn(r6 + (float)c.x), t8 = __frcp_rn(r8 + (float)c.y);
                    const float a6 = (float)sc.s6 * t6, a8 = (float)c.w * t8;
                    const float gg = a6 + a8;
                    const float dphi_r = c6 * (6.0f * a6 * r4 * t6 + 8.0f * a8 * r6 * t8);
                    ue += (double)(-0.5f * c6 * gg);
                    g += (double)(-gg * dc6);
                    fx += (double)(dphi_r * x);
                    fy += (double)(dphi_r * yv);
                    fz += (double)(dphi_r * zz);
                    const float hh = -0.5f * dphi_r;
                    const float hx = hh * x, hy = hh * yv;
                    vir[0] += (double)(hx * x);
                    vir[1] += (double)(hx * yv);
                    vir[2] += (double)(hx * zz);
                    vir[3] += (double)(hy * yv);
                    vir[4] += (double)(hy * zz);
                    vir[5] += (double)(hh * zz * zz);
                    if constexpr (AV) {
                        av[0] += (double)(hx * x);
                        av[1] += (double)(hx * yv);
                        av[2] += (double)(hx * zz);
                        av[3] += (double)(hy * yv);
                        av[4] += (double)(hy * zz);
                        av[5] += (double)(hh * zz * zz);
                    }
                }
                base += cf;
            }
            __builtin_amdgcn_wave_barrier();  // LDS rows are reused by the next chunk
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
        __builtin_amdgcn_wave_barrier();
    }
    const double vals[7] = {lane == 0 ? esum : 0.0, vir[0], vir[1], vir[2], vir[3], vir[4], vir[5]};
    block_partials(vals, part);
}

// ------------------------------------------------------------ host side --

static uint16_t bf16_bits(float v)
{
    uint32_t u;
    std::memcpy(&u, &v, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);
    u = u + 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

static float bf16_value(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float v;
    std::memcpy(&v, &u, 4);
    return v;
}

static int n_pairs(const d3_ctx* c) { return c->n_elem * (c->n_elem + 1) / 2; }

void surrogate_free(d3_ctx* c)
{
    if (c && c->sur) {
        Surrogate* s = c->sur;
        for (Buf* b : {&s->w32, &s->stats, &s->adam_m, &s->adam_v, &s->grad, &s->packed,
                       &s->samples, &s->loss})
            release(*b);
        delete s;
        c->sur = nullptr;
    }
}

// upload the master weights and stats from s->h_w and build the inference pack
static int upload_weights(d3_ctx* c, hipStream_t st)
{
    Surrogate* s = c->sur;
    const int P = n_pairs(c);
    const size_t nw = (size_t)P * NPAR;
    // host pack: small weights, A operands (hi, lo)
    std::vector<float> small((size_t)P * SMALL, 0.0f);
    std::vector<uint16_t> apk((size_t)P * 2 * 2 * WAVE * 8);  // [hi/lo][P][2][64][8]
    for (int p = 0; p < P; p++) {
        const float* w = s->h_w.data() + (size_t)p * NPAR;
        float* sm = small.data() + (size_t)p * SMALL;
        for (int k = 0; k < 2 * H; k++) sm[SM_W1 + k] = w[OW1 + k];
        for (int k = 0; k < H; k++) sm[SM_B1 + k] = w[OB1 + k];
        for (int k = 0; k < H; k++) sm[SM_B2 + k] = w[OB2 + k];
        for (int k = 0; k < 3 * H; k++) sm[SM_W3 + k] = w[OW3 + k];
        for (int k = 0; k < 3; k++) sm[SM_B3 + k] = w[OB3 + k];
        for (int blk = 0; blk < 2; blk++)
            for (int l = 0; l < WAVE; l++)
                for (int j = 0; j < 8; j++) {
                    const int k = 16 * blk + 8 * (l / 32) + j;  // input unit
                    const int m = l % 32;                       // output unit
                    const float v = w[OW2 + k * H + m];
                    const uint16_t hi = bf16_bits(v);
                    const uint16_t lo = bf16_bits(v - bf16_value(hi));
                    const size_t o = (((size_t)p * 2 + blk) * WAVE + l) * 8 + j;
                    apk[o] = hi;
                    apk[(size_t)P * 2 * WAVE * 8 + o] = lo;
                }
    }
    const size_t small_bytes = small.size() * sizeof(float);
    const size_t apk_bytes = apk.size() * sizeof(uint16_t);
    int r = ensure(s->packed, small_bytes + apk_bytes + 256);
    if (r) return r;
    hipError_t e = hipMemcpyAsync(s->w32.p, s->h_w.data(), nw * sizeof(float),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->stats.p, s->h_w.data() + nw, (size_t)P * 6 * sizeof(float),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->packed.p, small.data(), small_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync((char*)s->packed.p + ((small_bytes + 255) & ~(size_t)255), apk.data(),
                           apk_bytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "surrogate upload");
    return D3_OK;
}

static SurView view(const d3_ctx* c)
{
    const Surrogate* s = c->sur;
    const int P = n_pairs(c);
    SurView v;
    v.w32 = s->w32.as<float>();
    v.small = s->packed.as<float>();
    const size_t small_bytes = ((size_t)P * SMALL * sizeof(float) + 255) & ~(size_t)255;
    v.a_hi = (const bf16x8*)((const char*)s->packed.p + small_bytes);
    v.a_lo = v.a_hi + (size_t)P * 2 * WAVE;
    v.stats = s->stats.as<float>();
    v.cn_hi = s->cn_hi;
    v.ne = c->n_elem;
    return v;
}

int surrogate_pair(d3_ctx* c, const PairScal& sc, double* Vp, hipStream_t st, int* nblk)
{
    *nblk = 0;
    if (!c->sur || !c->sur->trained)
        return fail(D3_ERR_NOT_TRAINED, "surrogate mode before training or loading weights");
    if (c->n_elem > SUR_ELEM)
        return fail(D3_ERR_INVALID_ARG, "surrogate pass supports at most %d elements", SUR_ELEM);
    const int n = (int)c->n;
    if (n <= 0) return D3_OK;
    const Geo& g = c->geo;
#define D3_SUR(I, A)                                                                           \
    hipLaunchKernelGGL((k_pair_sur<I, A>),                                                     \
                       dim3(*nblk = pass_blocks((const void*)&k_pair_sur<I, A>, n)),           \
                       dim3(BLOCK), 0, st, n, c->pos_s.as<double4>(), c->img_tab.as<double4>(), \
                       g.n_img, g.img_bits, c->list_p.as<uint32_t>(), c->cnt_p.as<int>(),      \
                       c->cap_p, c->d_tab.as<ElemTab>(), c->d_c6.as<double>(),                 \
                       c->d_pc.as<double4>(), sc, c->cn.as<double>(), view(c),                 \
                       c->Fp.as<double>(), c->U.as<double>(), c->G.as<double>(), Vp,           \
                       c->vpart.as<double>())
    const bool lds = g.n_img <= IMG_LDS;
    if (Vp) {
        if (lds) D3_SUR(true, true);
        else D3_SUR(false, true);
    } else {
        if (lds) D3_SUR(true, false);
        else D3_SUR(false, false);
    }
#undef D3_SUR
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_pair_sur");
    return D3_OK;
}

static int ensure_sur(d3_ctx* c)
{
    if (!c->sur) c->sur = new Surrogate();
    Surrogate* s = c->sur;
    const int P = n_pairs(c);
    s->n_pairs = P;
    int r;
    if ((r = ensure(s->w32, (size_t)P * NPAR * sizeof(float)))) return r;
    if ((r = ensure(s->adam_m, (size_t)P * NPAR * sizeof(float)))) return r;
    if ((r = ensure(s->adam_v, (size_t)P * NPAR * sizeof(float)))) return r;
    if ((r = ensure(s->stats, (size_t)P * 6 * sizeof(float)))) return r;
    return D3_OK;
}

}  // namespace d3

using namespace d3;

extern "C" {

int d3_c6_surrogate_init(d3_ctx* c, uint64_t seed)
{
    if (!c) return fail(D3_ERR_INVALID_ARG, "ctx is NULL");
    int r = ensure_sur(c);
    if (r) return r;
    Surrogate* s = c->sur;
    const int P = n_pairs(c);
    s->h_w.assign((size_t)P * NPAR + (size_t)P * 6, 0.0f);
    uint64_t state = seed;
    auto uni = [&](float lim) {
        state = mix64(state);
        const double u = (double)(state >> 11) * (1.0 / 9007199254740992.0);
        return (float)((2.0 * u - 1.0) * lim);
    };
    for (int p = 0; p < P; p++) {
        float* w = s->h_w.data() + (size_t)p * NPAR;
        const float g1 = sqrtf(6.0f / (2 + H)), g2 = sqrtf(6.0f / (H + H)), g3 = sqrtf(6.0f / (H + 3));
        for (int k = 0; k < 2 * H; k++) w[OW1 + k] = uni(g1);
        for (int k = 0; k < H * H; k++) w[OW2 + k] = uni(g2);
        for (int k = 0; k < 3 * H; k++) w[OW3 + k] = uni(g3);
        float* st = s->h_w.data() + (size_t)P * NPAR + 6 * p;
        st[3] = st[4] = st[5] = 1.0f;
    }
    if (s->cn_hi <= 0.0f) s->cn_hi = 6.0f;
    s->trained = false;
    hipError_t e = hipMemset(s->adam_m.p, 0, (size_t)P * NPAR * sizeof(float));
    if (e == hipSuccess) e = hipMemset(s->adam_v.p, 0, (size_t)P * NPAR * sizeof(float));
    if (e != hipSuccess) return hip_fail(e, "surrogate init");
    return upload_weights(c, c->last_stream);
}

int d3_c6_surrogate_train(d3_ctx* c, const d3_train_cfg* cfg, double* final_loss, void* stream)
{
    if (!c || !cfg) return fail(D3_ERR_INVALID_ARG, "NULL argument");
    if (!c->sur) return fail(D3_ERR_STATE, "d3_c6_surrogate_init first");
    const int P = n_pairs(c);
    if (cfg->n_samples < P || cfg->n_samples > (1LL << 30) || cfg->epochs < 1 ||
        cfg->epochs > 100000 || !(cfg->lr > 0.0) || !(cfg->lr_final >= 0.0) ||
        !(cfg->cn_hi > 0.0) || (cfg->batch != 0 && cfg->batch != TB))
        return fail(D3_ERR_INVALID_ARG, "bad training configuration (batch must be 0 or %d)", TB);
    hipStream_t st = (hipStream_t)stream;
    c->last_stream = st;
    Surrogate* s = c->sur;
    s->cn_hi = (float)cfg->cn_hi;
    const int n_per = (int)(cfg->n_samples / P);
    const size_t ns = (size_t)P * n_per;
    int r;
    // layout of the sample buffer: X float[ns*2] | Y float[ns*3] | Yd double[ns*3]
    const size_t offY = ((ns * 2 * sizeof(float)) + 255) & ~(size_t)255;
    const size_t offYd = offY + (((ns * 3 * sizeof(float)) + 255) & ~(size_t)255);
    if ((r = ensure(s->samples, offYd + ns * 3 * sizeof(double)))) return r;
    const int spe = (n_per + TB - 1) / TB;  // steps per epoch
    if ((r = ensure(s->loss, (size_t)P * spe * sizeof(float)))) return r;
    if ((r = ensure(s->grad, 2 * MAXPAIR * sizeof(int)))) return r;
    std::vector<int> pe(2 * MAXPAIR, 0);
    for (int e = 0; e < c->n_elem; e++)
        for (int f = e; f < c->n_elem; f++) {
            pe[pair_index(e, f, c->n_elem)] = e;
            pe[MAXPAIR + pair_index(e, f, c->n_elem)] = f;
        }
    hipError_t e = hipMemcpyAsync(s->grad.p, pe.data(), pe.size() * sizeof(int),
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "upload pair table");
    float* X = s->samples.as<float>();
    float* Y = (float*)((char*)s->samples.p + offY);
    double* Yd = (double*)((char*)s->samples.p + offYd);
    hipLaunchKernelGGL(k_samples, dim3((unsigned)((ns + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st,
                       P, n_per, (uint64_t)cfg->seed, cfg->cn_hi, s->grad.as<int>(),
                       s->grad.as<int>() + MAXPAIR, c->d_tab.as<ElemTab>(), c->d_c6.as<double>(),
                       X, Yd);
    hipLaunchKernelGGL(k_standardise, dim3(P), dim3(BLOCK), 0, st, n_per, Yd, Y,
                       s->stats.as<float>());
    const int total = spe * cfg->epochs;
    for (int ep = 0; ep < cfg->epochs; ep++)
        hipLaunchKernelGGL(k_train, dim3(P), dim3(TB), 0, st, n_per, X, Y, s->w32.as<float>(),
                           s->adam_m.as<float>(), s->adam_v.as<float>(), ep * spe, spe, total,
                           (float)cfg->lr, (float)cfg->lr_final, (uint64_t)cfg->seed * 7919u + 11u,
                           s->loss.as<float>());
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "surrogate training launch");
    std::vector<float> losses((size_t)P * spe);
    s->h_w.resize((size_t)P * NPAR + (size_t)P * 6);
    e = hipMemcpyAsync(losses.data(), s->loss.p, losses.size() * sizeof(float),
                       hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->h_w.data(), s->w32.p, (size_t)P * NPAR * sizeof(float),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->h_w.data() + (size_t)P * NPAR, s->stats.p,
                           (size_t)P * 6 * sizeof(float), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "surrogate training");
    double sum = 0.0;
    for (float v : losses) sum += v;
    if (final_loss) *final_loss = sum / (double)losses.size();
    r = upload_weights(c, st);
    if (r) return r;
    s->trained = true;
    return D3_OK;
}

int d3_c6_surrogate_eval(d3_ctx* c, int64_t m, const int32_t* ei, const int32_t* ej,
                         const float* ni, const float* nj, float* out, int32_t precision,
                         void* stream)
{
    if (!c) return fail(D3_ERR_INVALID_ARG, "ctx is NULL");
    if (!c->sur) return fail(D3_ERR_NOT_TRAINED, "surrogate not initialised");
    if (m < 0 || m > INT32_MAX) return fail(D3_ERR_INVALID_ARG, "bad query count");
    if (m == 0) return D3_OK;
    if (!ei || !ej || !ni || !nj || !out) return fail(D3_ERR_INVALID_ARG, "NULL buffer");
    if (precision != 0 && precision != 1) return fail(D3_ERR_INVALID_ARG, "precision must be 0 or 1");
    hipStream_t st = (hipStream_t)stream;
    c->last_stream = st;
    hipLaunchKernelGGL(k_sur_eval, dim3((unsigned)((m + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st,
                       (int)m, ei, ej, ni, nj, view(c), precision, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_sur_eval");
    return D3_OK;
}

int d3_c6_exact_eval(d3_ctx* c, int64_t m, const int32_t* ei, const int32_t* ej,
                     const double* ni, const double* nj, double* out, void* stream)
{
    if (!c) return fail(D3_ERR_INVALID_ARG, "ctx is NULL");
    if (m < 0 || m > INT32_MAX) return fail(D3_ERR_INVALID_ARG, "bad query count");
    if (m == 0) return D3_OK;
    if (!ei || !ej || !ni || !nj || !out) return fail(D3_ERR_INVALID_ARG, "NULL buffer");
    hipStream_t st = (hipStream_t)stream;
    c->last_stream = st;
    hipLaunchKernelGGL(k_exact_eval, dim3((unsigned)((m + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st,
                       (int)m, ei, ej, ni, nj, c->d_tab.as<ElemTab>(), c->d_c6.as<double>(), out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_exact_eval");
    return D3_OK;
}

int64_t d3_c6_surrogate_bytes(d3_ctx* c)
{
    if (!c) return 0;
    const int P = n_pairs(c);
    return ((int64_t)P * NPAR + (int64_t)P * 6 + 1) * (int64_t)sizeof(float);
}

int d3_c6_surrogate_get_weights(d3_ctx* c, float* buf, int64_t bytes)
{
    if (!c || !buf) return fail(D3_ERR_INVALID_ARG, "NULL argument");
    if (!c->sur) return fail(D3_ERR_NOT_TRAINED, "surrogate not initialised");
    if (bytes != d3_c6_surrogate_bytes(c)) return fail(D3_ERR_INVALID_ARG, "wrong buffer size");
    const size_t nv = c->sur->h_w.size();
    std::memcpy(buf, c->sur->h_w.data(), nv * sizeof(float));
    buf[nv] = c->sur->cn_hi;
    return D3_OK;
}

int d3_c6_surrogate_set_weights(d3_ctx* c, const float* buf, int64_t bytes)
{
    if (!c || !buf) return fail(D3_ERR_INVALID_ARG, "NULL argument");
    if (bytes != d3_c6_surrogate_bytes(c)) return fail(D3_ERR_INVALID_ARG, "wrong buffer size");
    const size_t nv = (size_t)(bytes / sizeof(float)) - 1;
    for (size_t k = 0; k <= nv; k++)
        if (!std::isfinite(buf[k])) return fail(D3_ERR_INVALID_ARG, "non-finite weight");
    if (!(buf[nv] > 0.0f)) return fail(D3_ERR_INVALID_ARG, "cn_hi must be positive");
    int r = ensure_sur(c);
    if (r) return r;
    Surrogate* s = c->sur;
    s->h_w.assign(buf, buf + nv);
    s->cn_hi = buf[nv];
    r = upload_weights(c, c->last_stream);
    if (r) return r;
    s->trained = true;
    return D3_OK;
}

int d3_c6_surrogate_grad(d3_ctx* c, int64_t m, const int32_t* pair, const float* x,
                         const float* y, float* grads, float* loss, void* stream)
{
    if (!c) return fail(D3_ERR_INVALID_ARG, "ctx is NULL");
    if (!c->sur) return fail(D3_ERR_NOT_TRAINED, "surrogate not initialised");
    if (m < 1 || m > INT32_MAX || !pair || !x || !y || !grads || !loss)
        return fail(D3_ERR_INVALID_ARG, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    c->last_stream = st;
    hipError_t e = hipMemsetAsync(loss, 0, sizeof(float), st);
    if (e != hipSuccess) return hip_fail(e, "memset");
    hipLaunchKernelGGL(k_grad, dim3(n_pairs(c)), dim3(TB), 0, st, (int)m, pair, x, y,
                       c->sur->w32.as<float>(), grads, loss);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_grad");
    return D3_OK;
}

int d3_c6_surrogate_adam_step(d3_ctx* c, int64_t m, const int32_t* pair, const float* x,
                              const float* y, int64_t step, int64_t total_steps, double lr,
                              double lr_final, void* stream)
{
    if (!c) return fail(D3_ERR_INVALID_ARG, "ctx is NULL");
    if (!c->sur) return fail(D3_ERR_NOT_TRAINED, "surrogate not initialised");
    if (m < 1 || m > INT32_MAX || !pair || !x || !y)
        return fail(D3_ERR_INVALID_ARG, "bad arguments");
    if (step < 0 || total_steps < 1 || step > total_steps || total_steps > INT32_MAX ||
        !(lr > 0.0) || !(lr_final >= 0.0))
        return fail(D3_ERR_INVALID_ARG, "bad step, step count or step size");
    hipStream_t st = (hipStream_t)stream;
    c->last_stream = st;
    Surrogate* s = c->sur;
    const int P = n_pairs(c);
    hipLaunchKernelGGL(k_adam_step, dim3(P), dim3(TB), 0, st, (int)m, pair, x, y,
                       s->w32.as<float>(), s->adam_m.as<float>(), s->adam_v.as<float>(),
                       (int)step, (int)total_steps, (float)lr, (float)lr_final);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->h_w.data(), s->w32.p, (size_t)P * NPAR * sizeof(float),
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "k_adam_step");
    return upload_weights(c, st);
}

}  // extern "C"
