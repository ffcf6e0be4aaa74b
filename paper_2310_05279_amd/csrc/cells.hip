// Cell binning and neighbour-list construction for the two neighbour sets
// the D3 energy needs: pairs within R_pot (Eq. 2) and within R_cn (Eq. 4),
// each widened by the skin.
//
// Atoms are binned along the three lattice vectors (fractional
// coordinates, wrapped on periodic axes) and stored cell-sorted as double4
// (x, y, z, species bits) by a counting sort whose order inside a bin is
// the atom index (so every later sum has a fixed order).  A bin index runs
// fastest along the first lattice vector, so one stencil row of bins is one
// contiguous range of sorted atoms.
//
// Bins are a third of the list cutoff wide (a 7-bin stencil along each
// axis) or, for long cutoffs, narrow enough to hold a few atoms at the mean
// density (a deeper stencil).  One wave builds the lists of all atoms of
// one bin, or of a unit of two neighbouring bins along the first lattice
// vector in large periodic cells (see k_list); the bins are split between
// the XCDs in slabs that hold equal shares of the atoms.
#include "d3_device.h"

namespace d3 {

__device__ __forceinline__ int floordiv(int a, int b)
{
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

static inline int nblk(long n, int b) { return (int)((n + b - 1) / b); }

__global__ void __launch_bounds__(BLOCK)
k_bin(int n, const double* __restrict__ pos, const int32_t* __restrict__ type,
      int n_elem, Geo g, int* __restrict__ bin_of, double4* __restrict__ shift,
      int* __restrict__ count, int32_t* __restrict__ type_copy, int* __restrict__ status,
      const int* __restrict__ need)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (need && *need == 0)) return;
    double r[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    int t = type[i];
    if (t < 0 || t >= n_elem) {
        atomicOr(status, ST_SPECIES);
        t = 0;  // contained: no later table lookup leaves its table
    }
    type_copy[i] = t;
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
        // rounding edge of a periodic one) join the edge bins; bin
        // distances only shrink, so the stencil still covers every pair
        b[k] = !(q >= 0.0) ? 0 : (q >= (double)(g.nb[k] - 1) ? g.nb[k] - 1 : (int)q);
    }
    // an atom with a non-finite position goes to the extra bin nbins, which
    // no stencil visits and no list wave takes: it is left out of every list
    int bin = (b[2] * g.nb[1] + b[1]) * g.nb[0] + b[0];
    if (!finite) {
        atomicOr(status, ST_NONFINITE);
        bin = g.nbins;
    }
    bin_of[i] = bin;
    shift[i] = make_double4(sh[0], sh[1], sh[2], 0.0);
    atomicAdd(&count[bin], 1);
}

// Block-wide exclusive scan of one int per thread (LDS Hillis-Steele).
__device__ int block_excl_scan(int v, int* sh, int* total)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        int t = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    const int incl = sh[threadIdx.x];
    *total = sh[blockDim.x - 1];
    __syncthreads();
    return incl - v;
}

// Exclusive scan of up to SCAN_ONE_MAX bin counts by one workgroup of 1024
// threads, in tiles of 4096 bins: each thread takes 4 consecutive bins (the
// next tile's are loaded while this one is scanned), the thread sums are
// scanned across the wave with shuffles and across the 16 waves through LDS.
constexpr int SCAN_ONE_MAX = 65536;

__global__ void __launch_bounds__(1024)
k_scan_one(int m, const int* __restrict__ count, int* __restrict__ out,
           const int* __restrict__ need)
{
    if (need && *need == 0) return;
    __shared__ int wsum[2][1024 / WAVE];
    const int lane = threadIdx.x & (WAVE - 1), wv = threadIdx.x / WAVE;
    int carry = 0;
    int4 vn;
    {
        const int k0 = 4 * threadIdx.x;
        vn = (k0 + 3 < m) ? *(const int4*)(count + k0)
                          : make_int4(k0 < m ? count[k0] : 0, k0 + 1 < m ? count[k0 + 1] : 0,
                                      k0 + 2 < m ? count[k0 + 2] : 0, 0);
    }
    for (int base = 0, t = 0; base < m; base += 4096, t ^= 1) {
        const int k0 = base + 4 * threadIdx.x;
        const int4 v = vn;
        const int kn = k0 + 4096;
        if (base + 4096 < m)
            vn = (kn + 3 < m) ? *(const int4*)(count + kn)
                              : make_int4(kn < m ? count[kn] : 0, kn + 1 < m ? count[kn + 1] : 0,
                                          kn + 2 < m ? count[kn + 2] : 0, 0);
        const int tsum = v.x + v.y + v.z + v.w;
        int incl = tsum;
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
            const int u = __shfl_up(incl, d, WAVE);
            if (lane >= d) incl += u;
        }
        if (lane == WAVE - 1) wsum[t][wv] = incl;
        __syncthreads();
        int ex = carry + incl - tsum, tile = 0;
        for (int w = 0; w < 1024 / WAVE; w++) {
            const int ws = wsum[t][w];
            ex += (w < wv) ? ws : 0;
            tile += ws;
        }
        const int4 o = make_int4(ex, ex + v.x, ex + v.x + v.y, ex + v.x + v.y + v.z);
        if (k0 + 3 < m) {
            *(int4*)(out + k0) = o;
        } else {
            if (k0 < m) out[k0] = o.x;
            if (k0 + 1 < m) out[k0 + 1] = o.y;
            if (k0 + 2 < m) out[k0 + 2] = o.z;
        }
        carry += tile;
    }
    if (threadIdx.x == 0) out[m] = carry;
}

// three-phase exclusive scan for large bin tables, 1024 bins per block
constexpr int SCAN_PER_BLOCK = 1024;

__global__ void __launch_bounds__(BLOCK)
k_scan_local(int m, const int* __restrict__ in, int* __restrict__ out, int* __restrict__ blocksum,
             const int* __restrict__ need)
{
    if (need && *need == 0) return;
    __shared__ int sh[BLOCK];
    int base = blockIdx.x * SCAN_PER_BLOCK + threadIdx.x * 4;
    int v[4], s = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        v[q] = (base + q < m) ? in[base + q] : 0;
        s += v[q];
    }
    int total;
    int excl = block_excl_scan(s, sh, &total);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        if (base + q < m) out[base + q] = excl;
        excl += v[q];
    }
    if (threadIdx.x == 0) blocksum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(1024)
k_scan_top(int nblocks, int* __restrict__ blocksum, int* __restrict__ total,
           const int* __restrict__ need)
{
    if (need && *need == 0) return;
    __shared__ int sh[1024];
    int carry = 0;
    for (int c = 0; c < nblocks; c += 1024) {
        int i = c + threadIdx.x;
        int v = (i < nblocks) ? blocksum[i] : 0;
        int tot;
        int ex = block_excl_scan(v, sh, &tot);
        if (i < nblocks) blocksum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(BLOCK)
k_scan_add(int m, int* __restrict__ out, const int* __restrict__ blocksum,
           const int* __restrict__ total, const int* __restrict__ need)
{
    if (need && *need == 0) return;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] += blocksum[i / SCAN_PER_BLOCK];
    if (i == 0) out[m] = *total;
}

__global__ void __launch_bounds__(BLOCK)
k_scatter(int n, const int* __restrict__ bin_of, const int* __restrict__ bin_start,
          int* __restrict__ fill, int* __restrict__ perm_tmp, const int* __restrict__ need)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || (need && *need == 0)) return;
    int b = bin_of[i];
    int slot = bin_start[b] + atomicAdd(&fill[b], 1);
    perm_tmp[slot] = i;
}

// The scatter leaves the order inside a bin arbitrary.  Each slot computes
// the rank of its atom index among the bin's atoms and writes the atom to
// the sorted position, gathering its wrapped position and species.
__global__ void __launch_bounds__(BLOCK)
k_rank(int n, const int* __restrict__ perm_tmp, const int* __restrict__ bin_of,
       const int* __restrict__ bin_start, const double* __restrict__ pos,
       const int32_t* __restrict__ type_copy, const double4* __restrict__ shift,
       int* __restrict__ perm, double4* __restrict__ pos_s, double4* __restrict__ shift_s,
       double4* __restrict__ ref_s, int nbins, int* __restrict__ slab, int* __restrict__ count,
       int* __restrict__ cnt_p, int* __restrict__ cnt_c, const int* __restrict__ need)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || (need && *need == 0)) return;
    const int v = perm_tmp[k];
    const int b = bin_of[v];
    const int s = bin_start[b], e = bin_start[b + 1];
    int rank = 0;
    for (int q = s; q < e; q++) rank += (perm_tmp[q] < v) ? 1 : 0;
    const int o = s + rank;
    // the bin's count and scatter cursor are spent: leave them at zero for
    // the next build (every atom of the bin writes the same zeros); the
    // counts are nbins + 1 long, the last for atoms left out of the lists
    count[b] = 0;
    count[nbins + 1 + b] = 0;
    // XCD slabs of bins holding equal shares of the sorted atoms: slab x
    // starts at the bin of sorted atom floor(n x / 8)
#pragma unroll
    for (int x = 0; x < 8; x++)
        if (o == (int)((long long)n * x / 8)) slab[x] = b;
    if (o == 0) slab[8] = nbins;
    const double4 sh = shift[v];
    const double x = pos[3 * v] + sh.x, y = pos[3 * v + 1] + sh.y, z = pos[3 * v + 2] + sh.z;
    perm[o] = v;
    // an atom whose position is not finite (binned into the extra bin, after
    // every other atom) gets empty lists, a finite stand-in position (so that
    // no pass ever reads a non-finite coordinate) and a mark in the high word
    // of w, which the per-evaluation position copy reads
    // ref_s keeps the caller's positions of this build, unwrapped and
    // exact: the stale test measures displacements from them, and a
    // checkpoint reads them back to rebuild the same lists
    ref_s[o] = make_double4(pos[3 * v], pos[3 * v + 1], pos[3 * v + 2], 0.0);
    if (b < nbins) {
        pos_s[o] = make_double4(x, y, z, __hiloint2double(0, type_copy[v]));
    } else {
        pos_s[o] = make_double4(0.0, 0.0, 0.0, __hiloint2double(1, type_copy[v]));
        cnt_p[o] = 0;
        cnt_c[o] = 0;
    }
    shift_s[o] = sh;
}

// atom left out of the lists (non-finite position at the build)
__device__ __forceinline__ bool dead_atom(const double4& p) { return __double2hiint(p.w) != 0; }

// Per-evaluation copy of the caller's positions into the cell-sorted
// layout, using the wrap shifts of the last build so that list images
// stay valid; flags atoms that moved more than half the skin.
__global__ void __launch_bounds__(BLOCK)
k_update(int n, const double* __restrict__ pos, const int* __restrict__ perm,
         const double4* __restrict__ shift_s, const double4* __restrict__ ref_s,
         double4* __restrict__ pos_s, double half_skin2, int* __restrict__ status,
         int* __restrict__ stale_out, int stale_bit)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int i = perm[k];
    double4 sh = shift_s[k];
    double x = pos[3 * i] + sh.x, y = pos[3 * i + 1] + sh.y, z = pos[3 * i + 2] + sh.z;
    double4 p = pos_s[k];
    // a non-finite position is reported and not copied: the atom keeps its
    // last finite position (or its stand-in, if the build left it out)
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
        atomicOr(status, ST_NONFINITE);
        return;
    }
    if (dead_atom(p)) return;
    const double4 r = ref_s[k];
    const double dx = pos[3 * i] - r.x, dy = pos[3 * i + 1] - r.y, dz = pos[3 * i + 2] - r.z;
    double d2 = dx * dx + dy * dy + dz * dz;
    if (!(d2 <= half_skin2)) atomicOr(stale_out, stale_bit);
    pos_s[k] = make_double4(x, y, z, p.w);
}

constexpr int LIST_AHEAD = 4;  // candidate steps whose loads are in flight together
constexpr int UB_UNITE = 5;             // most atoms per bin of a unit built together
constexpr int UNIT2_MIN_BINS = 100000;  // units of several bins from this many bins on
constexpr int LIST_UB = 2;  // bins per unit then (three were no faster at 10^6 atoms)
constexpr int ROW_LDS = 1024;  // stencil rows of the row table held in LDS

// number of set bits of m below this lane
__device__ __forceinline__ int lanes_below(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const int t = __shfl_up(v, d, WAVE);
        if (lane >= d) v += t;
    }
    return v;
}

// One wave builds the lists of all atoms of one unit: a bin, or (UB > 1)
// UB neighbouring bins of a row, whose stencils then share one candidate
// set.  The unit's stencil is cut into segments, one per stencil row and
// periodic image; each segment is one contiguous range of sorted atoms.  TABLE (deep stencils of long
// cutoffs): the rows come from a host-made table that drops the bins lying
// wholly beyond the cutoff and puts the rows within R_cn reach first, so
// the later candidates skip the R_cn test.  Lanes take the segments' candidates
// densely packed, 64 per step (a lane finds its segment by a binary search
// over the segment offsets held by the lanes), load each candidate once, and
// test it in FP64 against every atom of the bin in turn; hits are compacted
// with a ballot into the atom's row.  The test is the same FP64 arithmetic
// as the passes, with a 1e-12 relative widening so that no pair a pass would
// accept is missed; the passes make the exact decision.  COUNT: count only.
template <bool IMG, bool COUNT, bool TABLE, int UB>
__global__ void __launch_bounds__(BLOCK)
k_list(const double4* __restrict__ pos_s, const int* __restrict__ bin_start,
       const int* __restrict__ slab, Geo g, const RowSpan* __restrict__ row_tab,
       const double4* __restrict__ img_tab, double rp2, double rc2,
       uint32_t* __restrict__ list_p, int* __restrict__ cnt_p, int cap_p,
       uint32_t* __restrict__ list_c, int* __restrict__ cnt_c, int cap_c,
       int* __restrict__ status, const int* __restrict__ need)
{
    if (need && *need == 0) return;  // the same for every thread of the grid
    __shared__ double4 s_img[IMG ? IMG_LDS : 1];
    __shared__ RowSpan s_rows[TABLE ? ROW_LDS : 1];
    load_images<IMG>(s_img, img_tab, g.n_img);
    if constexpr (TABLE)
        for (int i = threadIdx.x; i < g.nrows && i < ROW_LDS; i += BLOCK) s_rows[i] = row_tab[i];
    __syncthreads();
    const double rp2w = rp2 * (1.0 + 1e-12), rc2w = rc2 * (1.0 + 1e-12);
    const int lane = threadIdx.x & (WAVE - 1);
    const int nb0 = g.nb[0], nb1 = g.nb[1], nb2 = g.nb[2];
    const int n1 = 2 * g.timg[1] + 1, n2 = 2 * g.timg[2] + 1;
    const int n1r = 2 * g.reach[1] + 1, n2r = 2 * g.reach[2] + 1;
    const int nrows = TABLE ? g.nrows : n1r * n2r;
    const uint32_t img_self = (uint32_t)((g.timg[0] * n1 + g.timg[1]) * n2 + g.timg[2]);
    // the waves of XCD x take the units of slab x round-robin.  A unit is UB
    // neighbouring bins along the first lattice vector, bins UB k .. UB k +
    // UB - 1 of a row: their stencils differ by one bin per row and bin, so
    // the candidate set-up of the union serves the atoms of all of them.  A
    // unit holding more than UB_UNITE atoms per bin takes its bins one at a
    // time
    const int per = gridDim.x >> 3;
    const int lb = xcd_block();
    const int x = lb / per;
    const int wave0 = (lb - x * per) * WAVES_PER_BLOCK + (int)(threadIdx.x / WAVE);
    const int hu = (nb0 + UB - 1) / UB;  // units per row
    // the first unit whose first bin is at or after bin b
    auto unit_of = [&](int b) -> int {
        if constexpr (UB == 1) return b;
        const int r = b / nb0, c0 = b - r * nb0;
        return r * hu + (c0 + UB - 1) / UB;
    };
    const int u_lo = unit_of(__builtin_amdgcn_readfirstlane(slab[x]));
    const int u_hi = unit_of(__builtin_amdgcn_readfirstlane(slab[x + 1]));
    for (int un = __builtin_amdgcn_readfirstlane(u_lo + wave0); un < u_hi;
         un += per * WAVES_PER_BLOCK) {
        int bin0 = un, nbh = 1;
        if constexpr (UB > 1) {
            const int r = un / hu, k0 = UB * (un - r * hu);
            bin0 = r * nb0 + k0;
            nbh = min(UB, nb0 - k0);
        }
        const int s_all = __builtin_amdgcn_readfirstlane(bin_start[bin0]);
        const int e_all = __builtin_amdgcn_readfirstlane(bin_start[bin0 + nbh]);
        if (s_all == e_all) continue;
        const bool unite = e_all - s_all <= UB_UNITE * nbh;
        const int nsub = unite ? 1 : nbh;
      for (int sub = 0; sub < nsub; sub++) {
        const int bin = bin0 + sub, span = unite ? nbh : 1;
        const int s = __builtin_amdgcn_readfirstlane(bin_start[bin]);
        const int e = __builtin_amdgcn_readfirstlane(bin_start[bin + span]);
        if (s == e) continue;
        const int b0 = bin % nb0, b1 = (bin / nb0) % nb1, b2 = bin / (nb0 * nb1);
        int ua = b0 - g.reach[0], ub = b0 + (span - 1) + g.reach[0], ta0, ta1;
        if (g.pbc[0]) {
            ta0 = floordiv(ua, nb0);
            ta1 = floordiv(ub, nb0);
        } else {
            ua = ua < 0 ? 0 : ua;
            ub = ub >= nb0 ? nb0 - 1 : ub;
            ta0 = ta1 = 0;
        }
        const int spr = ta1 - ta0 + 1;  // segments per stencil row
        const int nseg = nrows * spr;
        const int ncnseg = g.ncnrows * spr;  // TABLE: segments of the rows within R_cn reach
        for (int a0 = s; a0 < e; a0 += WAVE) {
            const int na = (e - a0) < WAVE ? (e - a0) : WAVE;
            int np = 0, nc = 0;  // lane t counts the entries of atom a0 + t
            for (int sb = 0; sb < nseg; sb += WAVE) {
                // lane -> segment sb + lane: first sorted atom, length, image
                int len = 0, jb = 0, img = 0;
                const int sg = sb + lane;
                if (sg < nseg) {
                    const int r = sg / spr, q = sg - r * spr;
                    int u1, u2;
                    if constexpr (TABLE) {
                        // the row's own span of first-axis bins
                        const RowSpan rs = r < ROW_LDS ? s_rows[r] : row_tab[r];
                        u1 = b1 + rs.d1;
                        u2 = b2 + rs.d2;
                        ua = b0 + rs.lo;
                        ub = b0 + rs.hi;
                        if (!g.pbc[0]) {
                            ua = ua < 0 ? 0 : ua;
                            ub = ub >= nb0 ? nb0 - 1 : ub;
                        }
                    } else {
                        u1 = b1 + (r % n1r - g.reach[1]);
                        u2 = b2 + (r / n1r - g.reach[2]);
                    }
                    int t1 = 0, w1 = u1, t2 = 0, w2 = u2;
                    bool ok = true;
                    if (g.pbc[1]) { t1 = floordiv(u1, nb1); w1 = u1 - t1 * nb1; }
                    else if (u1 < 0 || u1 >= nb1) ok = false;
                    if (g.pbc[2]) { t2 = floordiv(u2, nb2); w2 = u2 - t2 * nb2; }
                    else if (u2 < 0 || u2 >= nb2) ok = false;
                    const int t0 = ta0 + q;
                    const int lo = (ua > t0 * nb0 ? ua : t0 * nb0) - t0 * nb0;
                    const int hi = (ub < t0 * nb0 + nb0 - 1 ? ub : t0 * nb0 + nb0 - 1) - t0 * nb0;
                    if (ok && lo <= hi) {
                        const int row = (w2 * nb1 + w1) * nb0;
                        jb = bin_start[row + lo];
                        len = bin_start[row + hi + 1] - jb;
                        img = ((t0 + g.timg[0]) * n1 + (t1 + g.timg[1])) * n2 + (t2 + g.timg[2]);
                    }
                }
                const int incl = wave_incl_scan(len);
                const int excl = incl - len;  // non-decreasing over the lanes
                const int total = __builtin_amdgcn_readlane(incl, WAVE - 1);
                // TABLE: candidates [0, cn_total) come from the rows within R_cn
                // reach (they come first), the rest skip the R_cn test
                int cn_total = total;
                if constexpr (TABLE) {
                    const int last_cn = min(ncnseg - sb, WAVE) - 1;
                    const int at_last = __shfl(incl, last_cn < 0 ? 0 : last_cn, WAVE);
                    cn_total = last_cn < 0 ? 0 : __builtin_amdgcn_readfirstlane(at_last);
                }
                for (int kb = 0; kb < total; kb += LIST_AHEAD * WAVE) {
                    // candidates kb + u*64 + lane: sorted atom, image, position; each
                    // lies in the last segment whose offset is <= its index
                    int jj[LIST_AHEAD], ii[LIST_AHEAD];
                    double4 pp[LIST_AHEAD];
#pragma unroll
                    for (int u = 0; u < LIST_AHEAD; u++) {
                        const int k = kb + u * WAVE + lane;
                        int sl = 0;
#pragma unroll
                        for (int step = WAVE / 2; step >= 1; step >>= 1) {
                            const int o = __shfl(excl, sl + step, WAVE);
                            sl = (o <= k) ? sl + step : sl;
                        }
                        // all lanes take part in the shuffles (a lane cannot read an
                        // inactive lane), then the lanes past the end are cleared
                        const int o = __shfl(excl, sl, WAVE);
                        const int jv = __shfl(jb, sl, WAVE) + (k - o);
                        const int iv = __shfl(img, sl, WAVE);
                        const bool in = k < total;
                        jj[u] = in ? jv : 0;
                        ii[u] = in ? iv : 0;
                        pp[u] = pos_s[jj[u]];
                    }
                    const int nch = min(LIST_AHEAD, (total - kb + WAVE - 1) / WAVE);
                    double qx[LIST_AHEAD], qy[LIST_AHEAD], qz[LIST_AHEAD];
                    uint32_t code[LIST_AHEAD];
                    bool valid[LIST_AHEAD];
#pragma unroll
                    for (int u = 0; u < LIST_AHEAD; u++) {
                        valid[u] = kb + u * WAVE + lane < total;
                        const double4 T = image<IMG>(s_img, img_tab, (uint32_t)ii[u]);
                        qx[u] = pp[u].x + T.x;
                        qy[u] = pp[u].y + T.y;
                        qz[u] = pp[u].z + T.z;
                        code[u] = ((uint32_t)jj[u] << g.img_bits) | (uint32_t)ii[u];
                    }
                    // the bin's atoms in turn, each against the block's candidates;
                    // atom positions and entry counts are wave-uniform
                    for (int t = 0; t < na; t++) {
                        const int a = a0 + t;
                        const double4 pa = pos_s[a];
                        const uint32_t self = ((uint32_t)a << g.img_bits) | img_self;
                        int np_t = __builtin_amdgcn_readlane(np, t);
                        int nc_t = __builtin_amdgcn_readlane(nc, t);
                        uint32_t* rowp = list_p + (size_t)a * cap_p;
                        uint32_t* rowc = list_c + (size_t)a * cap_c;
#pragma unroll
                        for (int u = 0; u < LIST_AHEAD; u++) {
                            if (u >= nch) break;
                            const double dx = qx[u] - pa.x, dy = qy[u] - pa.y, dz = qz[u] - pa.z;
                            const double r2 = dx * dx + dy * dy + dz * dz;
                            const bool other = valid[u] & (code[u] != self);
                            const bool inp = other & (r2 < rp2w);
                            const bool inc =
                                (!TABLE || kb + u * WAVE < cn_total) & other & (r2 < rc2w);
                            unsigned long long bp, bc;
                            if constexpr (TABLE) {
                                bp = __ballot(inp);
                                bc = __ballot(inc);
                            } else {
                                // a ballot of a combined predicate goes through a VGPR;
                                // ballots of the single compares are the compares' own
                                // lane masks, combined on the scalar unit (the valid
                                // lanes are a prefix of the wave)
                                const int nv = total - (kb + u * WAVE);
                                const unsigned long long m_valid =
                                    nv >= WAVE ? ~0ull : (1ull << (nv > 0 ? nv : 0)) - 1ull;
                                const unsigned long long m_other =
                                    m_valid & __builtin_amdgcn_ballot_w64(code[u] != self);
                                bp = m_other & __builtin_amdgcn_ballot_w64(r2 < rp2w);
                                bc = m_other & __builtin_amdgcn_ballot_w64(r2 < rc2w);
                            }
                            if constexpr (!COUNT) {
                                if (inp) {
                                    const int sp = np_t + lanes_below(bp);
                                    if (sp < cap_p) rowp[(uint32_t)sp] = code[u];
                                }
                                if (inc) {
                                    const int sc = nc_t + lanes_below(bc);
                                    if (sc < cap_c) rowc[(uint32_t)sc] = code[u];
                                }
                            }
                            np_t += (int)__popcll(bp);
                            nc_t += (int)__popcll(bc);
                        }
                        const bool mine = lane == t;
                        np = mine ? np_t : np;
                        nc = mine ? nc_t : nc;
                    }
                }
            }
            if (lane < na) {
                cnt_p[a0 + lane] = np;  // true count; readers clamp to the capacity
                cnt_c[a0 + lane] = nc;
                if (!COUNT && (np > cap_p || nc > cap_c)) atomicOr(status, ST_CAPACITY);
            }
        }
      }
    }
}

// max and sum of the list lengths (sizing and statistics)
__global__ void __launch_bounds__(BLOCK)
k_cnt_stats(int n, const int* __restrict__ cnt_p, const int* __restrict__ cnt_c,
            int* __restrict__ out)
{
    __shared__ unsigned long long sh[4][BLOCK];
    unsigned long long mp = 0, mc = 0, sp = 0, sc = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const unsigned long long a = (unsigned)cnt_p[i], b = (unsigned)cnt_c[i];
        mp = a > mp ? a : mp;
        mc = b > mc ? b : mc;
        sp += a;
        sc += b;
    }
    sh[0][threadIdx.x] = mp;
    sh[1][threadIdx.x] = mc;
    sh[2][threadIdx.x] = sp;
    sh[3][threadIdx.x] = sc;
    __syncthreads();
    for (int off = BLOCK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            const int o = threadIdx.x + off;
            sh[0][threadIdx.x] = sh[0][o] > sh[0][threadIdx.x] ? sh[0][o] : sh[0][threadIdx.x];
            sh[1][threadIdx.x] = sh[1][o] > sh[1][threadIdx.x] ? sh[1][o] : sh[1][threadIdx.x];
            sh[2][threadIdx.x] += sh[2][o];
            sh[3][threadIdx.x] += sh[3][o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&out[0], (int)sh[0][0]);
        atomicMax(&out[1], (int)sh[1][0]);
        atomicAdd((unsigned long long*)&out[2], sh[2][0]);
        atomicAdd((unsigned long long*)&out[4], sh[3][0]);
    }
}

void launch_bin(int n, const double* pos, const int32_t* type, int n_elem,
                const Geo& g, int* bin_of, double4* shift, int* count,
                int32_t* type_copy, int* status, hipStream_t s, const int* need)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bin, dim3(nblk(n, BLOCK)), dim3(BLOCK), 0, s, n, pos,
                       type, n_elem, g, bin_of, shift, count, type_copy, status, need);
}

void launch_scan(int nbins, const int* count, int* bin_start, int* tmp, hipStream_t s,
                 const int* need)
{
    if (nbins <= SCAN_ONE_MAX) {
        hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(1024), 0, s, nbins, count, bin_start, need);
        return;
    }
    int nb = nblk(nbins, SCAN_PER_BLOCK);
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(BLOCK), 0, s, nbins, count,
                       bin_start, tmp, need);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, nb, tmp, tmp + nb, need);
    hipLaunchKernelGGL(k_scan_add, dim3(nblk(nbins, BLOCK)), dim3(BLOCK), 0, s,
                       nbins, bin_start, tmp, tmp + nb, need);
}

void launch_scatter(int n, const int* bin_of, const int* bin_start, int* fill,
                    int* perm_tmp, hipStream_t s, const int* need)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scatter, dim3(nblk(n, BLOCK)), dim3(BLOCK), 0, s, n,
                       bin_of, bin_start, fill, perm_tmp, need);
}

void launch_rank(int n, const int* perm_tmp, const int* bin_of, const int* bin_start,
                 const double* pos, const int32_t* type_copy, const double4* shift,
                 int* perm, double4* pos_s, double4* shift_s, double4* ref_s, int nbins,
                 int* slab, int* count, int* cnt_p, int* cnt_c, hipStream_t s, const int* need)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rank, dim3(nblk(n, BLOCK)), dim3(BLOCK), 0, s, n, perm_tmp,
                       bin_of, bin_start, pos, type_copy, shift, perm, pos_s, shift_s,
                       ref_s, nbins, slab, count, cnt_p, cnt_c, need);
}

void launch_update(int n, const double* pos, const int* perm,
                   const double4* shift_s, const double4* ref_s,
                   double4* pos_s, double half_skin2, int* status,
                   int* stale_out, int stale_bit, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_update, dim3(nblk(n, BLOCK)), dim3(BLOCK), 0, s, n,
                       pos, perm, shift_s, ref_s, pos_s, half_skin2, status, stale_out, stale_bit);
}

// The caller's positions of the last build, back in the caller's order.
__global__ void __launch_bounds__(BLOCK)
k_build_pos(int n, const int* __restrict__ perm, const double4* __restrict__ ref_s,
            double* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int i = perm[k];
    const double4 r = ref_s[k];
    out[3 * i] = r.x;
    out[3 * i + 1] = r.y;
    out[3 * i + 2] = r.z;
}

void launch_build_pos(int n, const int* perm, const double4* ref_s, double* out, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_build_pos, dim3(nblk(n, BLOCK)), dim3(BLOCK), 0, s, n, perm, ref_s, out);
}

void launch_list(int n, const double4* pos_s, const int* bin_start, const int* slab, const Geo& g,
                 const RowSpan* row_tab, const double4* img_tab, double rp2, double rc2,
                 uint32_t* list_p, int* cnt_p, int cap_p, uint32_t* list_c, int* cnt_c,
                 int cap_c, int count_only, int* status, hipStream_t s, const int* need)
{
    if (n <= 0) return;
#define D3_LIST(I, C, T, U)                                                                \
    hipLaunchKernelGGL((k_list<I, C, T, U>),                                               \
                       dim3(pass_blocks((const void*)&k_list<I, C, T, U>, units)), dim3(BLOCK), \
                       0, s, pos_s, bin_start, slab, g, row_tab, img_tab, rp2, rc2, list_p, \
                       cnt_p, cap_p, list_c, cnt_c, cap_c, status, need)
    const bool lds = g.n_img <= IMG_LDS;
    // the row table (trimmed, R_cn rows first) only for deep stencils.  Units
    // of two bins for large periodic bulk cells without a table: there the
    // build is bound by its VALU work, which the shared set-up cuts (about
    // 12 % from 110 000 bins on), while smaller builds, bound by each wave's
    // chain of dependent steps, and slabs with vacuum, whose bins hold many
    // atoms, were measured slower with them
    const bool unit2 = g.nrows == 0 && g.nbins >= UNIT2_MIN_BINS && g.pbc[0] && g.pbc[1] &&
                       g.pbc[2];
    const int units = unit2 ? g.nbins / g.nb[0] * ((g.nb[0] + LIST_UB - 1) / LIST_UB) : g.nbins;
    if (g.nrows > 0) {
        if (count_only) {
            if (lds) D3_LIST(true, true, true, 1);
            else D3_LIST(false, true, true, 1);
        } else {
            if (lds) D3_LIST(true, false, true, 1);
            else D3_LIST(false, false, true, 1);
        }
    } else if (unit2) {
        if (count_only) {
            if (lds) D3_LIST(true, true, false, LIST_UB);
            else D3_LIST(false, true, false, LIST_UB);
        } else {
            if (lds) D3_LIST(true, false, false, LIST_UB);
            else D3_LIST(false, false, false, LIST_UB);
        }
    } else {
        if (count_only) {
            if (lds) D3_LIST(true, true, false, 1);
            else D3_LIST(false, true, false, 1);
        } else {
            if (lds) D3_LIST(true, false, false, 1);
            else D3_LIST(false, false, false, 1);
        }
    }
#undef D3_LIST
}

void launch_cnt_stats(int n, const int* cnt_p, const int* cnt_c, int* out, hipStream_t s)
{
    if (n <= 0) return;
    int blocks = nblk(n, BLOCK);
    blocks = blocks > 1024 ? 1024 : blocks;
    hipLaunchKernelGGL(k_cnt_stats, dim3(blocks), dim3(BLOCK), 0, s, n, cnt_p, cnt_c, out);
}

}  // namespace d3
