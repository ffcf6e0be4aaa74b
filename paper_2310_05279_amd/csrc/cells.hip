// Cell binning and neighbour-list construction for the two neighbour sets
// the D3 energy needs: pairs within R_pot (Eq. 2) and within R_cn (Eq. 4),
// each widened by the skin.
//
// Atoms are binned along the three lattice vectors (fractional
// coordinates, wrapped on periodic axes), sorted by bin with a counting
// sort, and stored cell-sorted as double4 (x, y, z, species bits).  A bin
// index runs fastest along the first lattice vector, so one stencil row of
// bins is one contiguous range of sorted atoms.  One wavefront builds the
// lists of one atom: it walks the stencil rows, tests 64 candidates per
// step, and compacts the hits with a ballot.
#include "d3_internal.h"

namespace d3 {

__device__ __forceinline__ int floordiv(int a, int b)
{
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

__global__ void __launch_bounds__(BLOCK)
k_bin(int n, const double* __restrict__ pos, const int32_t* __restrict__ type,
      int n_elem, Geo g, int* __restrict__ bin_of, double4* __restrict__ shift,
      int* __restrict__ count, int* __restrict__ status)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    int t = type[i];
    if (t < 0 || t >= n_elem) atomicOr(status, ST_SPECIES);
    double sh[3] = {0.0, 0.0, 0.0};
    int b[3];
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        double s = r[0] * g.Hinv[k] + r[1] * g.Hinv[3 + k] + r[2] * g.Hinv[6 + k];
        if (!isfinite(s)) { finite = false; s = 0.0; }
        double q;
        if (g.pbc[k]) {
            double f = floor(s);
            sh[0] -= f * g.H[3 * k];
            sh[1] -= f * g.H[3 * k + 1];
            sh[2] -= f * g.H[3 * k + 2];
            q = floor((s - f) * g.nb[k]);
        } else {
            q = floor(s * g.nb[k]);
        }
        // clamp: atoms outside the cell along an open axis (or at the
        // rounding edge of a periodic one) join the edge bins
        b[k] = !(q >= 0.0) ? 0 : (q >= (double)(g.nb[k] - 1) ? g.nb[k] - 1 : (int)q);
    }
    if (!finite) atomicOr(status, ST_NONFINITE);
    int bin = (b[2] * g.nb[1] + b[1]) * g.nb[0] + b[0];
    bin_of[i] = bin;
    shift[i] = make_double4(sh[0], sh[1], sh[2], 0.0);
    atomicAdd(&count[bin], 1);
}

// three-phase exclusive scan, 1024 elements per block
constexpr int SCAN_PER_BLOCK = 1024;

__global__ void __launch_bounds__(BLOCK)
k_scan_local(int m, const int* __restrict__ in, int* __restrict__ out,
             int* __restrict__ blocksum)
{
    __shared__ int sh[BLOCK];
    int base = blockIdx.x * SCAN_PER_BLOCK + threadIdx.x * 4;
    int v[4], s = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        v[q] = (base + q < m) ? in[base + q] : 0;
        s += v[q];
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < BLOCK; off <<= 1) {
        int t = (threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int excl = sh[threadIdx.x] - s;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        if (base + q < m) out[base + q] = excl;
        excl += v[q];
    }
    if (threadIdx.x == BLOCK - 1) blocksum[blockIdx.x] = sh[BLOCK - 1];
}

__global__ void __launch_bounds__(1024)
k_scan_top(int nblocks, int* __restrict__ blocksum, int* __restrict__ total)
{
    __shared__ int sh[1024];
    int carry = 0;
    for (int c = 0; c < nblocks; c += 1024) {
        int i = c + threadIdx.x;
        int v = (i < nblocks) ? blocksum[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int t = (threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nblocks) blocksum[i] = carry + sh[threadIdx.x] - v;
        int last = sh[1023];
        __syncthreads();
        carry += last;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(BLOCK)
k_scan_add(int m, int* __restrict__ out, const int* __restrict__ blocksum,
           const int* __restrict__ total)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] += blocksum[i / SCAN_PER_BLOCK];
    if (i == 0) out[m] = *total;
}

__global__ void __launch_bounds__(BLOCK)
k_scatter(int n, const int* __restrict__ bin_of, const int* __restrict__ bin_start,
          int* __restrict__ fill, int* __restrict__ perm)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = bin_of[i];
    int slot = bin_start[b] + atomicAdd(&fill[b], 1);
    perm[slot] = i;
}

// Atomics leave the order inside a bin arbitrary; sorting each (short)
// bin by atom index makes the layout, and every sum over it, deterministic.
__global__ void __launch_bounds__(BLOCK)
k_binsort(int nbins, const int* __restrict__ bin_start, int* __restrict__ perm,
          int* __restrict__ bin_s)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    int s = bin_start[b], e = bin_start[b + 1];
    for (int k = s + 1; k < e; k++) {
        int v = perm[k];
        int q = k - 1;
        while (q >= s && perm[q] > v) {
            perm[q + 1] = perm[q];
            q--;
        }
        perm[q + 1] = v;
    }
    for (int k = s; k < e; k++) bin_s[k] = b;
}

__global__ void __launch_bounds__(BLOCK)
k_gather_build(int n, const double* __restrict__ pos, const int32_t* __restrict__ type,
               int n_elem, const int* __restrict__ perm, const double4* __restrict__ shift,
               double4* __restrict__ pos_s, double4* __restrict__ shift_s,
               double4* __restrict__ ref_s)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int i = perm[k];
    double4 sh = shift[i];
    double x = pos[3 * i] + sh.x, y = pos[3 * i + 1] + sh.y, z = pos[3 * i + 2] + sh.z;
    // an out-of-range species was flagged by k_bin; clamp it so that no
    // later table lookup leaves its table
    int t = type[i];
    t = (t < 0 || t >= n_elem) ? 0 : t;
    double tb = __hiloint2double(0, t);
    pos_s[k] = make_double4(x, y, z, tb);
    shift_s[k] = sh;
    ref_s[k] = make_double4(x, y, z, 0.0);
}

// Per-evaluation copy of the caller's positions into the cell-sorted
// layout, using the wrap shifts of the last build so that list images
// stay valid; flags atoms that moved more than half the skin.
__global__ void __launch_bounds__(BLOCK)
k_update(int n, const double* __restrict__ pos, const int* __restrict__ perm,
         const double4* __restrict__ shift_s, const double4* __restrict__ ref_s,
         double4* __restrict__ pos_s, double half_skin2, int* __restrict__ status)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int i = perm[k];
    double4 sh = shift_s[k];
    double x = pos[3 * i] + sh.x, y = pos[3 * i + 1] + sh.y, z = pos[3 * i + 2] + sh.z;
    double4 r = ref_s[k];
    double dx = x - r.x, dy = y - r.y, dz = z - r.z;
    double d2 = dx * dx + dy * dy + dz * dz;
    if (!(d2 <= half_skin2)) atomicOr(status, ST_STALE);
    double4 p = pos_s[k];
    pos_s[k] = make_double4(x, y, z, p.w);
}

__global__ void __launch_bounds__(BLOCK)
k_list(int n, const double4* __restrict__ pos_s, const int* __restrict__ bin_s,
       const int* __restrict__ bin_start, Geo g, const double4* __restrict__ img_tab,
       double rp2, double rc2, uint32_t* __restrict__ list_p, int* __restrict__ cnt_p,
       int cap_p, uint32_t* __restrict__ list_c, int* __restrict__ cnt_c, int cap_c,
       int count_only, int* __restrict__ maxcnt, int* __restrict__ status)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
    const int nwaves = (gridDim.x * blockDim.x) / WAVE;
    const double rmax2 = rp2 > rc2 ? rp2 : rc2;
    const int nim1 = 2 * g.timg[1] + 1, nim2 = 2 * g.timg[2] + 1;
    const unsigned long long lanemask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int i = wave; i < n; i += nwaves) {
        const double4 pi = pos_s[i];
        const int bin = bin_s[i];
        const int b0 = bin % g.nb[0];
        const int b1 = (bin / g.nb[0]) % g.nb[1];
        const int b2 = bin / (g.nb[0] * g.nb[1]);
        int np = 0, nc = 0;
        uint32_t* lp = list_p + (size_t)i * cap_p;
        uint32_t* lc = list_c + (size_t)i * cap_c;
        for (int d2 = -g.reach[2]; d2 <= g.reach[2]; d2++) {
            int u2 = b2 + d2, t2, w2;
            if (g.pbc[2]) { t2 = floordiv(u2, g.nb[2]); w2 = u2 - t2 * g.nb[2]; }
            else { if (u2 < 0 || u2 >= g.nb[2]) continue; t2 = 0; w2 = u2; }
            for (int d1 = -g.reach[1]; d1 <= g.reach[1]; d1++) {
                int u1 = b1 + d1, t1, w1;
                if (g.pbc[1]) { t1 = floordiv(u1, g.nb[1]); w1 = u1 - t1 * g.nb[1]; }
                else { if (u1 < 0 || u1 >= g.nb[1]) continue; t1 = 0; w1 = u1; }
                const int row = (w2 * g.nb[1] + w1) * g.nb[0];
                int ua = b0 - g.reach[0], ub = b0 + g.reach[0];
                int ta0, ta1;
                if (g.pbc[0]) { ta0 = floordiv(ua, g.nb[0]); ta1 = floordiv(ub, g.nb[0]); }
                else { ua = ua < 0 ? 0 : ua; ub = ub >= g.nb[0] ? g.nb[0] - 1 : ub; ta0 = ta1 = 0; }
                for (int t0 = ta0; t0 <= ta1; t0++) {
                    int lo = (ua > t0 * g.nb[0] ? ua : t0 * g.nb[0]) - t0 * g.nb[0];
                    int hi = (ub < t0 * g.nb[0] + g.nb[0] - 1 ? ub : t0 * g.nb[0] + g.nb[0] - 1) - t0 * g.nb[0];
                    if (lo > hi) continue;
                    const int jb = bin_start[row + lo], je = bin_start[row + hi + 1];
                    const int img = ((t0 + g.timg[0]) * nim1 + (t1 + g.timg[1])) * nim2 + (t2 + g.timg[2]);
                    const double4 T = img_tab[img];
                    const bool self_img = (t0 == 0 && t1 == 0 && t2 == 0);
                    for (int j0 = jb; j0 < je; j0 += WAVE) {
                        const int j = j0 + lane;
                        bool inp = false, inc = false;
                        if (j < je) {
                            const double4 pj = pos_s[j];
                            const double dx = pj.x + T.x - pi.x;
                            const double dy = pj.y + T.y - pi.y;
                            const double dz = pj.z + T.z - pi.z;
                            const double r2 = dx * dx + dy * dy + dz * dz;
                            const bool ok = !(self_img && j == i) && r2 < rmax2;
                            inp = ok && r2 < rp2;
                            inc = ok && r2 < rc2;
                        }
                        const unsigned long long bp = __ballot(inp);
                        const unsigned long long bc = __ballot(inc);
                        if (!count_only) {
                            const uint32_t code = ((uint32_t)j << g.img_bits) | (uint32_t)img;
                            if (inp) {
                                int slot = np + __popcll(bp & lanemask);
                                if (slot < cap_p) lp[slot] = code;
                            }
                            if (inc) {
                                int slot = nc + __popcll(bc & lanemask);
                                if (slot < cap_c) lc[slot] = code;
                            }
                        }
                        np += __popcll(bp);
                        nc += __popcll(bc);
                    }
                }
            }
        }
        if (lane == 0) {
            cnt_p[i] = np < cap_p ? np : cap_p;
            cnt_c[i] = nc < cap_c ? nc : cap_c;
            if (!count_only && (np > cap_p || nc > cap_c)) atomicOr(status, ST_CAPACITY);
            atomicMax(&maxcnt[0], np);
            atomicMax(&maxcnt[1], nc);
            atomicAdd((unsigned long long*)&maxcnt[2], (unsigned long long)np);
            atomicAdd((unsigned long long*)&maxcnt[4], (unsigned long long)nc);
        }
    }
}

static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

void launch_bin(int n, const double* pos, const int32_t* type, int n_elem,
                const Geo& g, int* bin_of, double4* shift, int* count,
                int* status, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bin, dim3(nblk(n, BLOCK)), dim3(BLOCK), 0, s, n, pos,
                       type, n_elem, g, bin_of, shift, count, status);
}

void launch_scan(int nbins, const int* count, int* bin_start, int* tmp,
                 hipStream_t s)
{
    int nb = nblk(nbins, SCAN_PER_BLOCK);
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(BLOCK), 0, s, nbins, count,
                       bin_start, tmp);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, nb, tmp, tmp + nb);
    hipLaunchKernelGGL(k_scan_add, dim3(nblk(nbins, BLOCK)), dim3(BLOCK), 0, s,
                       nbins, bin_start, tmp, tmp + nb);
}

void launch_scatter(int n, const int* bin_of, const int* bin_start, int* fill,
                    int* perm, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scatter, dim3(nblk(n, BLOCK)), dim3(BLOCK), 0, s, n,
                       bin_of, bin_start, fill, perm);
}

void launch_binsort(int nbins, const int* bin_start, int* perm, int* bin_s,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_binsort, dim3(nblk(nbins, BLOCK)), dim3(BLOCK), 0, s,
                       nbins, bin_start, perm, bin_s);
}

void launch_gather_build(int n, const double* pos, const int32_t* type, int n_elem,
                         const int* perm, const double4* shift,
                         double4* pos_s, double4* shift_s, double4* ref_s,
                         hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_build, dim3(nblk(n, BLOCK)), dim3(BLOCK), 0, s,
                       n, pos, type, n_elem, perm, shift, pos_s, shift_s, ref_s);
}

void launch_update(int n, const double* pos, const int* perm,
                   const double4* shift_s, const double4* ref_s,
                   double4* pos_s, double half_skin2, int* status,
                   hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_update, dim3(nblk(n, BLOCK)), dim3(BLOCK), 0, s, n,
                       pos, perm, shift_s, ref_s, pos_s, half_skin2, status);
}

void launch_list(int n, const double4* pos_s, const int* bin_s,
                 const int* bin_start, const Geo& g, const double4* img_tab,
                 double rp2, double rc2, uint32_t* list_p, int* cnt_p,
                 int cap_p, uint32_t* list_c, int* cnt_c, int cap_c,
                 int count_only, int* maxcnt, int* status, hipStream_t s)
{
    if (n <= 0) return;
    int waves = pass_waves(n);
    hipLaunchKernelGGL(k_list, dim3(nblk(waves, WAVES_PER_BLOCK)), dim3(BLOCK), 0,
                       s, n, pos_s, bin_s, bin_start, g, img_tab, rp2, rc2,
                       list_p, cnt_p, cap_p, list_c, cnt_c, cap_c, count_only,
                       maxcnt, status);
}

}  // namespace d3
