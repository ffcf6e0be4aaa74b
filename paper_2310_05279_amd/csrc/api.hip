// Host side of the C ABI declared in include/d3.h: argument validation,
// table conversion, bin geometry, device scratch and launch sequencing.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <mutex>
#include <atomic>

#include "d3_ctx.h"

#define HIPCHK_T(call)                                    \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

namespace d3 {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(D3_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// set while an allocation-free entry point runs on this thread: a buffer
// that would have to grow is an error instead of an allocation
thread_local bool g_no_alloc = false;

int ensure_bytes(void** p, size_t* have, size_t need)
{
    if (need == 0) need = 256;
    if (*p && *have >= need) return D3_OK;
    if (g_no_alloc)
        return fail(D3_ERR_CAPACITY,
                    "static scratch too small: a buffer of %zu bytes needs %zu", *have, need);
    if (*p) {
        hipError_t e = hipFree(*p);
        *p = nullptr;
        *have = 0;
        if (e != hipSuccess) return hip_fail(e, "hipFree");
    }
    hipError_t e = hipMalloc(p, need);
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(e, "hipMalloc");
    }
    *have = need;
    return D3_OK;
}

void release(Buf& b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

static const double HARTREE_EV = 27.211386245988;
static const double BOHR_ANG = 0.529177210903;

static void inv3(const double* m, double* o)
{
    const double det = m[0] * (m[4] * m[8] - m[5] * m[7]) -
                       m[1] * (m[3] * m[8] - m[5] * m[6]) +
                       m[2] * (m[3] * m[7] - m[4] * m[6]);
    o[0] = (m[4] * m[8] - m[5] * m[7]) / det;
    o[1] = (m[2] * m[7] - m[1] * m[8]) / det;
    o[2] = (m[1] * m[5] - m[2] * m[4]) / det;
    o[3] = (m[5] * m[6] - m[3] * m[8]) / det;
    o[4] = (m[0] * m[8] - m[2] * m[6]) / det;
    o[5] = (m[2] * m[3] - m[0] * m[5]) / det;
    o[6] = (m[3] * m[7] - m[4] * m[6]) / det;
    o[7] = (m[1] * m[6] - m[0] * m[7]) / det;
    o[8] = (m[0] * m[4] - m[1] * m[3]) / det;
}

// Squared smallest distance between the points of two bins whose indices
// differ by d: the minimum of |sum_k t_k e_k|^2 over t_k in [d_k - 1,
// d_k + 1], with e_k the bin edge vectors (lattice vector k / nb_k).  Along
// an open axis t_k is free, because atoms outside the cell join the edge
// bins.  The function is convex in t, so its minimum is one of the
// stationary points of the 27 choices (free, lower bound, upper bound) per
// axis; a free coordinate is clamped into its interval, which only gives a
// feasible point (never a value below the minimum).
static double bin_gap2(const double G[3][3], const int d[3], const int* pbc)
{
    double best = INFINITY;
    for (int code = 0; code < 27; code++) {
        const int mode[3] = {code % 3, (code / 3) % 3, code / 9};  // 0 free, 1 low, 2 high
        double t[3] = {0.0, 0.0, 0.0};
        int fr[3], nf = 0;
        bool ok = true;
        for (int k = 0; k < 3; k++) {
            if (mode[k] == 0) fr[nf++] = k;
            else if (!pbc[k]) ok = false;
            else t[k] = d[k] + (mode[k] == 1 ? -1.0 : 1.0);
        }
        if (!ok) continue;
        // G_FF t_F = -G_F,fixed t_fixed
        double b[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < nf; a++)
            for (int k = 0; k < 3; k++)
                if (mode[k] != 0) b[a] -= G[fr[a]][k] * t[k];
        if (nf == 1) {
            t[fr[0]] = b[0] / G[fr[0]][fr[0]];
        } else if (nf == 2) {
            const double a00 = G[fr[0]][fr[0]], a01 = G[fr[0]][fr[1]], a11 = G[fr[1]][fr[1]];
            const double det = a00 * a11 - a01 * a01;
            t[fr[0]] = (b[0] * a11 - a01 * b[1]) / det;
            t[fr[1]] = (a00 * b[1] - a01 * b[0]) / det;
        }  // nf == 3: the unconstrained minimum t = 0
        for (int a = 0; a < nf; a++) {
            const int k = fr[a];
            if (pbc[k]) t[k] = std::min(std::max(t[k], d[k] - 1.0), d[k] + 1.0);
        }
        double q = 0.0;
        for (int k = 0; k < 3; k++)
            for (int l = 0; l < 3; l++) q += t[k] * G[k][l] * t[l];
        best = std::min(best, q);
    }
    return std::max(best, 0.0);
}

// Stencil row table of deep stencils (reach >= ROW_TABLE_REACH): for every
// row offset (d1, d2) the range of d0 whose bins can hold a pair within
// rlist (an interval, the gap being convex in d), the rows that can hold a
// pair within rcn first.  Left empty (every row of the full stencil, as
// computed in the kernel) for shallow stencils and for stencils too large
// for a table.
static void make_rows(const double* cell, Geo& g, double rlist, double rcn, RowSpan* rows)
{
    g.nrows = g.ncnrows = 0;
    const int rmax = std::max(g.reach[0], std::max(g.reach[1], g.reach[2]));
    const long n0 = 2L * g.reach[0] + 1, n1 = 2L * g.reach[1] + 1, n2 = 2L * g.reach[2] + 1;
    if (rmax < ROW_TABLE_REACH || n1 * n2 > MAX_ROW_TAB || n0 * n1 * n2 > (1L << 18)) return;
    double e[3][3], G[3][3];
    for (int k = 0; k < 3; k++)
        for (int m = 0; m < 3; m++) e[k][m] = cell[3 * k + m] / g.nb[k];
    for (int k = 0; k < 3; k++)
        for (int l = 0; l < 3; l++) G[k][l] = e[k][0] * e[l][0] + e[k][1] * e[l][1] + e[k][2] * e[l][2];
    // keep a bin when its gap is within the cutoff, with a relative margin
    // far above the rounding of binning and wrapping
    const double lim = rlist * rlist * (1.0 + 1e-9) + 1e-12;
    const double limc = rcn * rcn * (1.0 + 1e-9) + 1e-12;
    // two sweeps: the rows that can hold R_cn pairs, then the others
    int nr = 0, ncn = 0;
    for (int sweep = 0; sweep < 2; sweep++)
        for (int d2 = -g.reach[2]; d2 <= g.reach[2]; d2++)
            for (int d1 = -g.reach[1]; d1 <= g.reach[1]; d1++) {
                int lo = INT32_MAX, hi = INT32_MIN;
                bool cn = false;
                for (int d0 = -g.reach[0]; d0 <= g.reach[0]; d0++) {
                    const int d[3] = {d0, d1, d2};
                    const double q = bin_gap2(G, d, g.pbc);
                    if (q <= lim) {
                        lo = std::min(lo, d0);
                        hi = std::max(hi, d0);
                    }
                    if (q <= limc) cn = true;
                }
                if (lo > hi || cn != (sweep == 0)) continue;
                if (rows) rows[nr] = RowSpan{d1, d2, lo, hi};
                nr++;
                ncn += cn ? 1 : 0;
            }
    g.nrows = nr;
    g.ncnrows = ncn;
}

// Bin layout for list cutoff rlist: nb_k bins along lattice vector k,
// each about rlist / BIN_DIV wide or, for long cutoffs, the width that
// holds BIN_ATOMS atoms (measured between lattice planes),
// stencil reach ceil(rlist / width) bins, the image translations the
// stencil can reach on periodic axes, and the row table of a deep stencil
// (rcn: the shorter list cutoff).
int make_geo(const double* cell, const int32_t* pbc, double rlist, double rcn, int64_t n,
             Geo& g, double4* imgs, RowSpan* rows)
{
    double la[3];
    for (int k = 0; k < 3; k++)
        la[k] = std::sqrt(cell[3 * k] * cell[3 * k] + cell[3 * k + 1] * cell[3 * k + 1] +
                          cell[3 * k + 2] * cell[3 * k + 2]);
    const double det = cell[0] * (cell[4] * cell[8] - cell[5] * cell[7]) -
                       cell[1] * (cell[3] * cell[8] - cell[5] * cell[6]) +
                       cell[2] * (cell[3] * cell[7] - cell[4] * cell[6]);
    if (!std::isfinite(det) || la[0] == 0.0 || la[1] == 0.0 || la[2] == 0.0 ||
        std::fabs(det) <= 1e-10 * la[0] * la[1] * la[2])
        return fail(D3_ERR_CELL, "singular or non-finite cell (det=%g)", det);
    std::memcpy(g.H, cell, sizeof(g.H));
    inv3(cell, g.Hinv);
    const double vol = std::fabs(det);
    // bins at least rlist / BIN_DIV wide; for a long cutoff, narrower bins
    // that hold about BIN_ATOMS atoms at the cell's mean density (a deeper
    // stencil of small bins keeps one bin per wave, with enough bins to
    // fill the chip), but never narrower than rlist / MAX_REACH
    double target = rlist / BIN_DIV;
    if (n > 0)
        target = std::min(target, std::max(std::cbrt(BIN_ATOMS * vol / (double)n),
                                           rlist / MAX_REACH));
    double h[3];
    long nb[3];
    for (int k = 0; k < 3; k++) {
        g.pbc[k] = pbc[k] ? 1 : 0;
        const double* u = cell + 3 * ((k + 1) % 3);
        const double* v = cell + 3 * ((k + 2) % 3);
        const double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2],
                     cz = u[0] * v[1] - u[1] * v[0];
        h[k] = vol / std::sqrt(cx * cx + cy * cy + cz * cz);
        nb[k] = (long)std::floor(h[k] / target);
        nb[k] = std::max(1L, std::min(nb[k], 2048L));
    }
    while (nb[0] * nb[1] * nb[2] > (1L << 24)) {  // keep the bin table modest
        int k = 0;
        for (int q = 1; q < 3; q++)
            if (nb[q] > nb[k]) k = q;
        nb[k] = (nb[k] + 1) / 2;
    }
    for (int k = 0; k < 3; k++) {
        const double width = h[k] / (double)nb[k];
        long reach = (long)std::ceil(rlist / width * (1.0 + 1e-12));
        if (!g.pbc[k] && reach > nb[k] - 1) reach = nb[k] - 1;
        if (reach > 4096)
            return fail(D3_ERR_CELL, "cutoff spans %ld cells along lattice vector %d", reach, k);
        g.nb[k] = (int)nb[k];
        g.reach[k] = (int)reach;
        g.timg[k] = g.pbc[k] ? (int)((reach + nb[k] - 1) / nb[k]) : 0;
    }
    g.nbins = (int)(nb[0] * nb[1] * nb[2]);
    const long nimg = (long)(2 * g.timg[0] + 1) * (2 * g.timg[1] + 1) * (2 * g.timg[2] + 1);
    int bits = 0;
    while ((1L << bits) < nimg) bits++;
    if (n > 0 && ((uint64_t)(n - 1) << bits) >= (1ull << 32))
        return fail(D3_ERR_CELL,
                    "%lld atoms x %ld periodic images exceed the 32-bit list encoding",
                    (long long)n, nimg);
    g.n_img = (int)nimg;
    g.img_bits = bits;
    int c = 0;
    if (imgs)
        for (int t0 = -g.timg[0]; t0 <= g.timg[0]; t0++)
            for (int t1 = -g.timg[1]; t1 <= g.timg[1]; t1++)
                for (int t2 = -g.timg[2]; t2 <= g.timg[2]; t2++) {
                    double T[3];
                    for (int m = 0; m < 3; m++)
                        T[m] = t0 * cell[m] + t1 * cell[3 + m] + t2 * cell[6 + m];
                    imgs[c++] = make_double4(T[0], T[1], T[2], 0.0);
                }
    make_rows(cell, g, rlist, rcn, rows);
    return D3_OK;
}

// make_geo into the context's host staging arrays: sized first, then
// filled; a context without growable staging (the allocation-free entry
// point) must already hold enough
int make_geo_staged(d3_ctx* c, const double* cell, const int32_t* pbc, double rlist, double rcn,
                    int64_t n, Geo& g)
{
    D3CHK(make_geo(cell, pbc, rlist, rcn, n, g, nullptr, nullptr));
    const size_t ni = (size_t)g.n_img, nr = (size_t)std::max(g.nrows, 1);
    if (c->stage_fixed) {
        if (ni > c->h_img_cap || nr > c->h_rows_cap)
            return fail(D3_ERR_CAPACITY, "%zu images or %zu stencil rows exceed the static limits "
                        "(%zu, %zu)", ni, nr, c->h_img_cap, c->h_rows_cap);
    } else {
        c->img_store.resize(ni);
        c->rows_store.resize(nr);
        c->h_img = c->img_store.data();
        c->h_rows = c->rows_store.data();
        c->h_img_cap = ni;
        c->h_rows_cap = nr;
    }
    return make_geo(cell, pbc, rlist, rcn, n, g, c->h_img, c->h_rows);
}

static int device_cus()
{
    static std::atomic<int> ncu{0};
    int v = ncu.load();
    if (v > 0) return v;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v < 1)
        v = 256;
    ncu.store(v);
    return v;
}

int max_pass_blocks()
{
    const int waves = MAX_WAVES_PER_SIMD * 4 * device_cus();
    return ((waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK + 7) / 8 * 8;
}

int pass_blocks(const void* kernel, int units, size_t dyn_lds)
{
    // resident workgroups per CU of each kernel, from the runtime's occupancy
    // (a fixed table: no heap use, so the allocation-free path may call it)
    constexpr int CACHE = 128;
    static std::mutex mu;
    static const void* keys[CACHE];
    static int vals[CACHE];
    static int used = 0;
    int per_cu = 0;
    {
        std::lock_guard<std::mutex> lock(mu);
        for (int k = 0; k < used; k++)
            if (keys[k] == kernel) per_cu = vals[k];
        if (per_cu == 0) {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, BLOCK, dyn_lds) !=
                    hipSuccess || nb < 1)
                nb = 1;
            (void)hipGetLastError();
            if (used < CACHE) {
                keys[used] = kernel;
                vals[used] = nb;
                used++;
            }
            per_cu = nb;
        }
    }
    const long cus = device_cus();
    const long resident = (long)per_cu * WAVES_PER_BLOCK * cus;
    long waves = units < 1 ? 1 : units;
    if (waves <= 8 * resident) waves = waves < resident ? waves : resident;
    else waves = std::min(waves, (long)MAX_WAVES_PER_SIMD * 4 * cus);
    return (int)(((waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK + 7) / 8 * 8);
}

void phase_mark(d3_ctx* c, int phase, hipStream_t s)
{
    if (!c->timing) return;
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        c->ev_pool.push_back(e);
        c->ev_phase.push_back(0);
    }
    c->ev_phase[c->ev_used] = phase;
    (void)hipEventRecord(c->ev_pool[c->ev_used], s);
    c->ev_used++;
}

int timing_flush(d3_ctx* c)
{
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        HIPCHK_T(hipEventSynchronize(c->ev_pool[k + 1]));
        float ms = 0.0f;
        HIPCHK_T(hipEventElapsedTime(&ms, c->ev_pool[k], c->ev_pool[k + 1]));
        c->t_ms[c->ev_phase[k]] += ms;
        c->t_calls[c->ev_phase[k]] += 1;
    }
    c->ev_used = 0;
    return D3_OK;
}

static bool same_geometry(const d3_ctx* c, int64_t n, const double* cell, const int32_t* pbc)
{
    if (!c->built || c->n != n) return false;
    for (int k = 0; k < 9; k++)
        if (c->cell[k] != cell[k]) return false;
    for (int k = 0; k < 3; k++)
        if ((c->geo.pbc[k] != 0) != (pbc[k] != 0)) return false;
    return true;
}


int alloc_atoms(d3_ctx* c, int64_t n)
{
    const size_t N = (size_t)(n > 0 ? n : 1);
    D3CHK(ensure(c->bin_of, N * sizeof(int)));
    D3CHK(ensure(c->shift, N * sizeof(double4)));
    D3CHK(ensure(c->perm, N * sizeof(int)));
    D3CHK(ensure(c->perm_tmp, N * sizeof(int)));
    D3CHK(ensure(c->pos_s, N * sizeof(double4)));
    D3CHK(ensure(c->shift_s, N * sizeof(double4)));
    D3CHK(ensure(c->ref_s, N * sizeof(double4)));
    D3CHK(ensure(c->type_copy, N * sizeof(int32_t)));
    D3CHK(ensure(c->cn, N * sizeof(double)));
    D3CHK(ensure(c->cnf, N * sizeof(float)));
    D3CHK(ensure(c->w, N * MAXREF * sizeof(double)));
    D3CHK(ensure(c->wd, N * MAXREF * sizeof(double)));
    D3CHK(ensure(c->G, N * sizeof(double)));
    D3CHK(ensure(c->Fp, N * 3 * sizeof(double)));
    D3CHK(ensure(c->U, N * sizeof(double)));
    D3CHK(ensure(c->cnt_p, N * sizeof(int)));
    D3CHK(ensure(c->cnt_c, N * sizeof(int)));
    const size_t nb = (size_t)max_pass_blocks();
    D3CHK(ensure(c->vpart, nb * 8 * sizeof(double)));
    D3CHK(ensure(c->vpart2, nb * 8 * sizeof(double)));
    D3CHK(ensure(c->vpart3, nb * 8 * sizeof(double)));
    return D3_OK;
}

int alloc_proj(d3_ctx* c, int mode)
{
    const size_t N = (size_t)(c->n > 0 ? c->n : 1);
    // per-atom neighbour data of the dispersion pass, 16-byte pieces in
    // whole blocks of PBLK atoms
    if (mode == D3_MODE_PREC_F32)
        return ensure(c->Pf, (N + PBLKF - 1) / PBLKF * PBLKF * NPIECEF * 4 * sizeof(float));
    return ensure(c->P, (N + PBLK - 1) / PBLK * PBLK * NPIECE * 4 * sizeof(double));
}

// Binning, counting sort and list construction on stream s.
int list_stats(d3_ctx* c, hipStream_t s, int* mc)
{
    HIPCHK(hipMemsetAsync(c->maxcnt.p, 0, 8 * sizeof(int), s));
    launch_cnt_stats((int)c->n, c->cnt_p.as<int>(), c->cnt_c.as<int>(), c->maxcnt.as<int>(), s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(mc, c->maxcnt.p, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return D3_OK;
}

// Binning, counting sort and list construction on stream s.  With
// size_lists the list lengths are counted first and the capacities set
// (one synchronisation).
int run_build(d3_ctx* c, const double* pos, const int32_t* type, bool size_lists,
              hipStream_t s, const int* need)
{
    const int n = (int)c->n;
    const Geo& g = c->geo;
    // counts and scatter cursors of nbins + 1 bins (the last: atoms left out)
    int* count = c->count.as<int>();
    int* fill = count + g.nbins + 1;
    // a build decided on the device (need) reuses the sizes and relies on
    // the counts that every completed build leaves at zero
    if (need && (size_lists || !c->counts_clean))
        return fail(D3_ERR_STATE, "a device-decided rebuild needs a completed sized build");
    // the bin counts and scatter cursors are left at zero by the ranking
    // kernel of the previous build; they are cleared here only after an
    // allocation or a build that did not complete
    phase_mark(c, PH_BUILD, s);
    if (!c->counts_clean)
        HIPCHK(hipMemsetAsync(count, 0, 2 * ((size_t)g.nbins + 1) * sizeof(int), s));
    c->counts_clean = false;
    launch_bin(n, pos, type, c->n_elem, g, c->bin_of.as<int>(), c->shift.as<double4>(), count,
               c->type_copy.as<int32_t>(), c->status.as<int>(), s, need);
    launch_scan(g.nbins + 1, count, c->bin_start.as<int>(), c->scan_tmp.as<int>(), s, need);
    launch_scatter(n, c->bin_of.as<int>(), c->bin_start.as<int>(), fill, c->perm_tmp.as<int>(), s,
                   need);
    launch_rank(n, c->perm_tmp.as<int>(), c->bin_of.as<int>(), c->bin_start.as<int>(), pos,
                c->type_copy.as<int32_t>(), c->shift.as<double4>(), c->perm.as<int>(),
                c->pos_s.as<double4>(), c->shift_s.as<double4>(), c->ref_s.as<double4>(),
                g.nbins, c->slab.as<int>(), count, c->cnt_p.as<int>(), c->cnt_c.as<int>(), s,
                need);
    HIPCHK(hipGetLastError());
    const double rp = c->prm.r_pot + c->prm.skin, rcn = c->prm.r_cn + c->prm.skin;
    if (size_lists) {
        launch_list(n, c->pos_s.as<double4>(), c->bin_start.as<int>(), c->slab.as<int>(), g,
                    c->row_tab.as<RowSpan>(), c->img_tab.as<double4>(),
                    rp * rp, rcn * rcn, nullptr, c->cnt_p.as<int>(), 0, nullptr,
                    c->cnt_c.as<int>(), 0, 1, c->status.as<int>(), s);
        HIPCHK(hipGetLastError());
        int mc[8];
        D3CHK(list_stats(c, s, mc));
        // headroom for later rebuilds of the same geometry (MD)
        c->cap_p = std::max(std::max(1, mc[0] + std::max(16, mc[0] / 8)), c->min_cap_p);
        c->cap_c = std::max(std::max(1, mc[1] + std::max(16, mc[1] / 8)), c->min_cap_c);
        c->cap_p = (c->cap_p + 3) & ~3;
        c->cap_c = (c->cap_c + 3) & ~3;
        const size_t N = (size_t)(n > 0 ? n : 1);
        D3CHK(ensure(c->list_p, N * c->cap_p * sizeof(uint32_t)));
        D3CHK(ensure(c->list_c, N * c->cap_c * sizeof(uint32_t)));
    }
    phase_mark(c, PH_BUILD, s);
    phase_mark(c, PH_LIST, s);
    launch_list(n, c->pos_s.as<double4>(), c->bin_start.as<int>(), c->slab.as<int>(), g,
                c->row_tab.as<RowSpan>(), c->img_tab.as<double4>(),
                rp * rp, rcn * rcn, c->list_p.as<uint32_t>(), c->cnt_p.as<int>(), c->cap_p,
                c->list_c.as<uint32_t>(), c->cnt_c.as<int>(), c->cap_c, 0, c->status.as<int>(), s,
                need);
    phase_mark(c, PH_LIST, s);
    HIPCHK(hipGetLastError());
    c->counts_clean = true;
    return D3_OK;
}

int read_status(d3_ctx* c, hipStream_t s, int* out)
{
    HIPCHK(hipMemcpyAsync(c->h_status, c->status.p, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *out = *c->h_status;
    if (*out & ST_CAPACITY) c->lists_bad = true;
    return D3_OK;
}

int status_code(int bits)
{
    if (bits & ST_SPECIES) return fail(D3_ERR_SPECIES, "a species index is outside [0, n_elem)");
    if (bits & ST_NONFINITE) return fail(D3_ERR_INVALID_ARG, "non-finite atomic position");
    if (bits & ST_CAPACITY) return fail(D3_ERR_CAPACITY, "neighbour list capacity exceeded");
    if (bits & ST_STALE) return fail(D3_ERR_STALE, "an atom moved more than skin/2 since the last build");
    return D3_OK;
}

// geometry-aware build used by d3_build_neighbors and by auto-rebuilds
int build(d3_ctx* c, int64_t n, const double* pos, const int32_t* type, const double* cell,
          const int32_t* pbc, hipStream_t s)
{
    // lists known to have overflowed are sized again, as for a new geometry
    const bool same = same_geometry(c, n, cell, pbc) && !c->lists_bad;
    if (!same) {
        Geo g;
        const double rlist = std::max(c->prm.r_pot, c->prm.r_cn) + c->prm.skin;
        D3CHK(make_geo_staged(c, cell, pbc, rlist, c->prm.r_cn + c->prm.skin, n, g));
        c->n = n;
        c->geo = g;
        std::memcpy(c->cell, cell, sizeof(c->cell));
        D3CHK(alloc_atoms(c, n));
        D3CHK(ensure(c->count, 2 * ((size_t)g.nbins + 1) * sizeof(int)));
        c->counts_clean = false;
        D3CHK(ensure(c->bin_start, ((size_t)g.nbins + 2) * sizeof(int)));
        D3CHK(ensure(c->slab, 16 * sizeof(int)));
        D3CHK(ensure(c->scan_tmp, ((size_t)g.nbins / 1024 + 5) * sizeof(int)));
        D3CHK(ensure(c->img_tab, (size_t)g.n_img * sizeof(double4)));
        HIPCHK(hipMemcpyAsync(c->img_tab.p, c->h_img, (size_t)g.n_img * sizeof(double4),
                              hipMemcpyHostToDevice, s));
        D3CHK(ensure(c->row_tab, (size_t)std::max(g.nrows, 1) * sizeof(RowSpan)));
        if (g.nrows > 0)
            HIPCHK(hipMemcpyAsync(c->row_tab.p, c->h_rows, (size_t)g.nrows * sizeof(RowSpan),
                                  hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
        c->built = false;
    }
    D3CHK(run_build(c, pos, type, !same, s));
    if (!same) c->lists_bad = false;  // capacities counted from these positions
    c->built = true;
    c->last_stream = s;
    return D3_OK;
}

int update_positions(d3_ctx* c, const double* pos, hipStream_t s)
{
    const double hs = 0.5 * c->prm.skin;
    phase_mark(c, PH_UPDATE, s);
    launch_update((int)c->n, pos, c->perm.as<int>(), c->shift_s.as<double4>(),
                  c->ref_s.as<double4>(), c->pos_s.as<double4>(), hs * hs,
                  c->status.as<int>(), c->status.as<int>(), ST_STALE, s);
    phase_mark(c, PH_UPDATE, s);
    HIPCHK(hipGetLastError());
    return D3_OK;
}

int coordination(d3_ctx* c, int mode, hipStream_t s)
{
    D3CHK(alloc_proj(c, mode));
    const Geo& g = c->geo;
    phase_mark(c, PH_CN, s);
    launch_cn(mode, (int)c->n, c->pos_s.as<double4>(), c->img_tab.as<double4>(), g.n_img,
              g.img_bits, c->list_c.as<uint32_t>(), c->cnt_c.as<int>(), c->cap_c,
              c->d_tab.as<ElemTab>(), c->prm.r_cn * c->prm.r_cn, c->cn.as<double>(),
              c->w.as<double>(), c->wd.as<double>(), c->P.as<double>(), c->Pf.as<float>(), s);
    phase_mark(c, PH_CN, s);
    HIPCHK(hipGetLastError());
    return D3_OK;
}

// Validation of d3_build_neighbors' arguments (also used by the
// allocation-free entry point).
int check_build_args(int64_t n, const double* pos, const int32_t* type, const double* cell,
                     const int32_t* pbc)
{
    if (n < 0 || n > (int64_t)INT32_MAX / 2) return fail(D3_ERR_INVALID_ARG, "n=%lld out of range", (long long)n);
    if (n > 0 && (!pos || !type)) return fail(D3_ERR_INVALID_ARG, "pos or type is NULL");
    if (!cell || !pbc) return fail(D3_ERR_INVALID_ARG, "cell or pbc is NULL");
    for (int k = 0; k < 9; k++)
        if (!std::isfinite(cell[k])) return fail(D3_ERR_CELL, "non-finite cell");
    for (int k = 0; k < 3; k++)
        if (pbc[k] != 0 && pbc[k] != 1) return fail(D3_ERR_INVALID_ARG, "pbc[%d]=%d not 0/1", k, pbc[k]);
    if (((uintptr_t)pos & 7) || ((uintptr_t)type & 3))
        return fail(D3_ERR_INVALID_ARG, "misaligned pos or type pointer");
    return D3_OK;
}

// Validation of d3_create's arguments (also used by the allocation-free
// entry point).
int check_params_table(const d3_params* prm, const d3_table* tab)
{
    if (!prm || !tab) return fail(D3_ERR_INVALID_ARG, "params or table is NULL");
    if (!(prm->r_pot > 0.0) || !(prm->r_cn > 0.0) || !(prm->skin >= 0.0) ||
        !std::isfinite(prm->r_pot) || !std::isfinite(prm->r_cn) || !std::isfinite(prm->skin))
        return fail(D3_ERR_INVALID_ARG, "cutoffs must be positive and finite, skin >= 0");
    if (!std::isfinite(prm->s6) || !std::isfinite(prm->s8) || !std::isfinite(prm->a1) ||
        !std::isfinite(prm->a2))
        return fail(D3_ERR_INVALID_ARG, "non-finite damping parameter");
    if (prm->mode < D3_MODE_PLAIN_F64 || prm->mode > D3_MODE_LITERAL)
        return fail(D3_ERR_INVALID_ARG, "unknown mode %d", prm->mode);
    if (prm->damping != D3_DAMP_BJ && prm->damping != D3_DAMP_ZERO)
        return fail(D3_ERR_INVALID_ARG, "unknown damping %d", prm->damping);
    if (prm->damping == D3_DAMP_ZERO &&
        !(prm->rs6 > 0.0 && prm->rs8 > 0.0 && std::isfinite(prm->rs6) && std::isfinite(prm->rs8)))
        return fail(D3_ERR_INVALID_ARG, "zero damping needs finite rs6 > 0 and rs8 > 0");
    if (!std::isfinite(prm->s9)) return fail(D3_ERR_INVALID_ARG, "non-finite s9");
    if (prm->s9 != 0.0 && !(prm->r_atm > 0.0 && prm->r_atm <= prm->r_cn))
        return fail(D3_ERR_INVALID_ARG, "the three-body cutoff must satisfy 0 < r_atm <= r_cn");
    const int ne = tab->n_elem;
    if (ne < 1 || ne > MAXELEM) return fail(D3_ERR_INVALID_ARG, "n_elem=%d outside 1..%d", ne, MAXELEM);
    if (!tab->n_ref || !tab->cn_ref || !tab->c6_ref || !tab->rcov || !tab->r2r4)
        return fail(D3_ERR_INVALID_ARG, "table array is NULL");
    for (int e = 0; e < ne; e++) {
        if (tab->n_ref[e] < 1 || tab->n_ref[e] > MAXREF)
            return fail(D3_ERR_INVALID_ARG, "n_ref[%d]=%d outside 1..%d", e, tab->n_ref[e], MAXREF);
        if (!(tab->rcov[e] >= 0.0) || !(tab->r2r4[e] >= 0.0) || !std::isfinite(tab->rcov[e]) ||
            !std::isfinite(tab->r2r4[e]))
            return fail(D3_ERR_INVALID_ARG, "rcov/r2r4 of element %d invalid", e);
        for (int a = 0; a < tab->n_ref[e]; a++)
            if (!std::isfinite(tab->cn_ref[e * MAXREF + a]))
                return fail(D3_ERR_INVALID_ARG, "cn_ref of element %d not finite", e);
    }
    for (int e = 0; e < ne; e++)
        for (int f = 0; f < ne; f++)
            for (int a = 0; a < tab->n_ref[e]; a++)
                for (int b = 0; b < tab->n_ref[f]; b++) {
                    const double x = tab->c6_ref[((e * ne + f) * MAXREF + a) * MAXREF + b];
                    const double y = tab->c6_ref[((f * ne + e) * MAXREF + b) * MAXREF + a];
                    if (!std::isfinite(x) || x != y)
                        return fail(D3_ERR_INVALID_ARG,
                                    "c6_ref not symmetric or not finite at (%d,%d,%d,%d)", e, f, a, b);
                }
    return D3_OK;
}

// The table in eV and Angstrom (FP64, on the host): per-element data, the
// C6 reference grid [MAXELEM][MAXELEM][MAXREF][MAXREF] and per element
// pair the damping constants: (Rd^6, Rd^8, R0^2, s8 R0^2), Rd = a1 R0 + a2
// (Eq. 2), or with zero damping (6 (rs6 R0)^14, 6 (rs8 R0)^16, R0^2,
// s8 R0^2).
void convert_table(const d3_params* prm, const d3_table* tab, ElemTab& et, double* c6,
                   double4* pc)
{
    const int ne = tab->n_elem;
    std::memset(&et, 0, sizeof(et));
    et.n_elem = ne;
    for (size_t q = 0; q < (size_t)MAXELEM * MAXELEM * MAXREF * MAXREF; q++) c6[q] = 0.0;
    for (int q = 0; q < MAXELEM * MAXELEM; q++) pc[q] = make_double4(0, 0, 0, 0);
    const double conv = HARTREE_EV * std::pow(BOHR_ANG, 6);
    for (int e = 0; e < ne; e++) {
        et.n_ref[e] = tab->n_ref[e];
        for (int a = 0; a < MAXREF; a++)
            et.cn_ref[e * MAXREF + a] = a < tab->n_ref[e] ? tab->cn_ref[e * MAXREF + a] : 0.0;
        et.rcov[e] = tab->rcov[e];
        for (int f = 0; f < ne; f++) {
            for (int a = 0; a < tab->n_ref[e]; a++)
                for (int b = 0; b < tab->n_ref[f]; b++)
                    c6[((size_t)(e * MAXELEM + f) * MAXREF + a) * MAXREF + b] =
                        tab->c6_ref[((e * ne + f) * MAXREF + a) * MAXREF + b] * conv;
            const double r0sq = 3.0 * tab->r2r4[e] * tab->r2r4[f] * BOHR_ANG * BOHR_ANG;
            if (prm->damping == D3_DAMP_ZERO) {
                // f_6 / r^6 = x^4 / (x^7 + K6) and f_8 / r^8 = x^4 / (x^8 + K8)
                // with x = r^2, K6 = 6 (rs6 R0)^14, K8 = 6 (rs8 R0)^16
                const double a6 = prm->rs6 * prm->rs6 * r0sq, a8 = prm->rs8 * prm->rs8 * r0sq;
                pc[e * MAXELEM + f] = make_double4(6.0 * std::pow(a6, 7), 6.0 * std::pow(a8, 8),
                                                   r0sq, prm->s8 * r0sq);
            } else {
                const double rd = prm->a1 * std::sqrt(r0sq) + prm->a2;
                const double rd2 = rd * rd, rd6 = rd2 * rd2 * rd2;
                pc[e * MAXELEM + f] = make_double4(rd6, rd6 * rd2, r0sq, prm->s8 * r0sq);
            }
        }
    }
}

}  // namespace d3

using namespace d3;

extern "C" {

const char* d3_last_error(void) { return g_err.c_str(); }

int d3_create(const d3_params* prm, const d3_table* tab, d3_ctx** out)
{
    if (!out) return fail(D3_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    D3CHK(check_params_table(prm, tab));
    const int ne = tab->n_elem;
    int device = 0;
    HIPCHK(hipGetDevice(&device));
    d3_ctx* c = new d3_ctx();
    c->prm = *prm;
    c->n_elem = ne;
    c->device = device;
    ElemTab et;
    std::vector<double> c6((size_t)MAXELEM * MAXELEM * MAXREF * MAXREF, 0.0);
    std::vector<double4> pc((size_t)MAXELEM * MAXELEM, make_double4(0, 0, 0, 0));
    convert_table(prm, tab, et, c6.data(), pc.data());
    c->h_c6 = c6;
    c->h_tab = et;
    for (int e = 0; e < ne; e++) c->h_r2r4[e] = tab->r2r4[e];
    int r;
    if ((r = ensure(c->d_tab, sizeof(ElemTab))) ||
        (r = ensure(c->d_c6, c6.size() * sizeof(double))) ||
        (r = ensure(c->d_pc, pc.size() * sizeof(double4))) ||
        (r = ensure(c->status, 256)) || (r = ensure(c->maxcnt, 256))) {
        d3_destroy(c);
        return r;
    }
    hipError_t e1 = hipMemcpy(c->d_tab.p, &et, sizeof(et), hipMemcpyHostToDevice);
    hipError_t e2 = hipMemcpy(c->d_c6.p, c6.data(), c6.size() * sizeof(double), hipMemcpyHostToDevice);
    hipError_t e3 = hipMemcpy(c->d_pc.p, pc.data(), pc.size() * sizeof(double4), hipMemcpyHostToDevice);
    hipError_t e4 = hipMemset(c->status.p, 0, 256);
    hipError_t e5 = hipHostMalloc((void**)&c->h_status, 64, hipHostMallocDefault);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess ||
        e5 != hipSuccess) {
        hipError_t e = e1 != hipSuccess ? e1 : e2 != hipSuccess ? e2 : e3 != hipSuccess ? e3
                     : e4 != hipSuccess ? e4 : e5;
        d3_destroy(c);
        return hip_fail(e, "d3_create upload");
    }
    *out = c;
    return D3_OK;
}

void d3_destroy(d3_ctx* c)
{
    if (!c) return;
    (void)hipDeviceSynchronize();
    for (Buf* b : c->all_buffers()) release(*b);
    if (c->h_status) (void)hipHostFree(c->h_status);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    surrogate_free(c);
    delete c;
}

int d3_set_mode(d3_ctx* c, int32_t mode)
{
    if (!c) return fail(D3_ERR_INVALID_ARG, "ctx is NULL");
    if (mode < D3_MODE_PLAIN_F64 || mode > D3_MODE_LITERAL)
        return fail(D3_ERR_INVALID_ARG, "unknown mode %d", mode);
    c->prm.mode = mode;
    return D3_OK;
}

int d3_build_neighbors(d3_ctx* c, int64_t n, const double* pos, const int32_t* type,
                       const double* cell, const int32_t* pbc, void* stream)
{
    if (!c) return fail(D3_ERR_INVALID_ARG, "ctx is NULL");
    D3CHK(check_build_args(n, pos, type, cell, pbc));
    hipStream_t s = (hipStream_t)stream;
    return build(c, n, pos, type, cell, pbc, s);
}

int d3_coordination(d3_ctx* c, const double* pos, double* cn_out, void* stream)
{
    if (!c) return fail(D3_ERR_INVALID_ARG, "ctx is NULL");
    if (!c->built) return fail(D3_ERR_STATE, "d3_coordination before d3_build_neighbors");
    if (c->n > 0 && !pos) return fail(D3_ERR_INVALID_ARG, "pos is NULL");
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    if (c->n == 0) return D3_OK;
    D3CHK(update_positions(c, pos, s));
    const int mode = c->prm.mode == D3_MODE_PREC_F32 ? D3_MODE_PREC_F32 : D3_MODE_PLAIN_F64;
    D3CHK(coordination(c, mode, s));
    if (cn_out) {
        launch_scatter_out((int)c->n, c->cn.as<double>(), c->perm.as<int>(), cn_out, s);
        HIPCHK(hipGetLastError());
    }
    return D3_OK;
}

int d3_build_positions(d3_ctx* c, double* pos_out, void* stream)
{
    if (!c) return fail(D3_ERR_INVALID_ARG, "ctx is NULL");
    if (!c->built) return fail(D3_ERR_STATE, "d3_build_positions before d3_build_neighbors");
    if (c->n > 0 && !pos_out) return fail(D3_ERR_INVALID_ARG, "pos_out is NULL");
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    launch_build_pos((int)c->n, c->perm.as<int>(), c->ref_s.as<double4>(), pos_out, s);
    HIPCHK(hipGetLastError());
    return D3_OK;
}

static int run_evaluate(d3_ctx* c, const double* pos, const d3_outputs& o, uint32_t flags,
                        void* stream, const char* who)
{
    double* energy = o.energy;
    double* virial = o.virial;
    if (!c) return fail(D3_ERR_INVALID_ARG, "ctx is NULL");
    if (!c->built) return fail(D3_ERR_STATE, "%s before d3_build_neighbors", who);
    if (!energy) return fail(D3_ERR_INVALID_ARG, "energy is NULL");
    if (o.heat_current && !o.velocities)
        return fail(D3_ERR_INVALID_ARG, "heat_current needs velocities");
    if (c->n > 0 && !pos) return fail(D3_ERR_INVALID_ARG, "pos is NULL");
    if (flags & ~(D3_ACCUMULATE | D3_AUTO_REBUILD | D3_REBUILD))
        return fail(D3_ERR_INVALID_ARG, "unknown flags");
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    const int acc = (flags & D3_ACCUMULATE) ? 1 : 0;
    const int n = (int)c->n;
    if (n == 0) {
        if (!acc) {
            HIPCHK(hipMemsetAsync(energy, 0, sizeof(double), s));
            if (virial) HIPCHK(hipMemsetAsync(virial, 0, 9 * sizeof(double), s));
        }
        return D3_OK;
    }
    if (c->lists_bad && !(flags & (D3_REBUILD | D3_AUTO_REBUILD)))
        return fail(D3_ERR_CAPACITY,
                    "the last build overflowed the neighbour lists: rebuild first "
                    "(d3_build_neighbors, D3_REBUILD or D3_AUTO_REBUILD)");
    if (flags & D3_REBUILD) {
        // a build from pos writes the sorted positions itself, so the
        // per-evaluation position update is not needed
        int32_t pbc[3];
        for (int k = 0; k < 3; k++) pbc[k] = c->geo.pbc[k];
        D3CHK(build(c, c->n, pos, c->type_copy.as<int32_t>(), c->cell, pbc, s));
    } else {
        D3CHK(update_positions(c, pos, s));
    }
    if ((flags & D3_AUTO_REBUILD) && !(flags & D3_REBUILD)) {
        int st = 0;
        D3CHK(read_status(c, s, &st));
        if (c->lists_bad) st |= ST_CAPACITY;
        if (st & (ST_STALE | ST_CAPACITY)) {
            const int keep = st & ~(ST_STALE | ST_CAPACITY);
            HIPCHK(hipMemsetAsync(c->status.p, 0, sizeof(int), s));
            if (keep) {
                *c->h_status = keep;
                HIPCHK(hipMemcpyAsync(c->status.p, c->h_status, sizeof(int), hipMemcpyHostToDevice, s));
            }
            D3CHK(rebuild_grow(c, pos, s));
        }
    }
    const int mode = c->prm.mode;
    D3CHK(evaluate(c, mode, energy, o.forces, virial, o.atom_energy, o.atom_virial, o.velocities,
                   o.heat_current, acc, s));
    return D3_OK;
}

int d3_energy_forces_virial(d3_ctx* c, const double* pos, double* energy, double* forces,
                            double* virial, double* atom_energy, uint32_t flags, void* stream)
{
    d3_outputs o{};
    o.energy = energy;
    o.forces = forces;
    o.virial = virial;
    o.atom_energy = atom_energy;
    return run_evaluate(c, pos, o, flags, stream, "d3_energy_forces_virial");
}

int d3_evaluate(d3_ctx* c, const double* pos, const d3_outputs* out, uint32_t flags, void* stream)
{
    if (!out) return fail(D3_ERR_INVALID_ARG, "out is NULL");
    return run_evaluate(c, pos, *out, flags, stream, "d3_evaluate");
}

int d3_status(d3_ctx* c)
{
    if (!c) return fail(D3_ERR_INVALID_ARG, "ctx is NULL");
    int st = 0;
    D3CHK(read_status(c, c->last_stream, &st));
    HIPCHK(hipMemsetAsync(c->status.p, 0, sizeof(int), c->last_stream));
    HIPCHK(hipStreamSynchronize(c->last_stream));
    return status_code(st);
}

int d3_set_timing(d3_ctx* c, int32_t enable)
{
    if (!c) return fail(D3_ERR_INVALID_ARG, "ctx is NULL");
    if (c->timing) D3CHK(timing_flush(c));
    c->timing = enable != 0;
    for (int k = 0; k < D3_N_PHASES; k++) {
        c->t_ms[k] = 0.0;
        c->t_calls[k] = 0;
    }
    return D3_OK;
}

int d3_get_timing(d3_ctx* c, double* ms, int64_t* calls)
{
    if (!c || !ms || !calls) return fail(D3_ERR_INVALID_ARG, "NULL argument");
    D3CHK(timing_flush(c));
    for (int k = 0; k < D3_N_PHASES; k++) {
        ms[k] = c->t_ms[k];
        calls[k] = c->t_calls[k];
    }
    return D3_OK;
}

int d3_list_stats(d3_ctx* c, double* out)
{
    if (!c || !out) return fail(D3_ERR_INVALID_ARG, "NULL argument");
    if (!c->built) return fail(D3_ERR_STATE, "no build yet");
    int mc[8];
    D3CHK(list_stats(c, c->last_stream, mc));
    unsigned long long sp, sc;
    std::memcpy(&sp, &mc[2], 8);
    std::memcpy(&sc, &mc[4], 8);
    const double n = c->n > 0 ? (double)c->n : 1.0;
    out[0] = mc[0];
    out[1] = (double)sp / n;
    out[2] = mc[1];
    out[3] = (double)sc / n;
    out[4] = c->geo.nbins;
    out[5] = c->geo.n_img;
    return D3_OK;
}

int d3_bin_plan(const double* cell, const int32_t* pbc, double rlist, double rcn, int64_t n,
                int32_t* nb, int32_t* reach, int32_t* nrows, int32_t* ncnrows, int32_t* rows,
                int32_t max_rows)
{
    if (!cell || !pbc || !nb || !reach || !nrows || !ncnrows)
        return fail(D3_ERR_INVALID_ARG, "NULL argument");
    if (!(rlist > 0.0) || !(rcn > 0.0) || rcn > rlist || n < 0 || max_rows < 0)
        return fail(D3_ERR_INVALID_ARG, "bad cutoffs, atom count or row capacity");
    Geo g{};
    D3CHK(make_geo(cell, pbc, rlist, rcn, n, g, nullptr, nullptr));
    std::vector<RowSpan> table((size_t)std::max(g.nrows, 1));
    D3CHK(make_geo(cell, pbc, rlist, rcn, n, g, nullptr, table.data()));
    for (int k = 0; k < 3; k++) {
        nb[k] = g.nb[k];
        reach[k] = g.reach[k];
    }
    *nrows = g.nrows;
    *ncnrows = g.ncnrows;
    if (rows)
        for (int r = 0; r < g.nrows && r < max_rows; r++) {
            rows[4 * r] = table[r].d1;
            rows[4 * r + 1] = table[r].d2;
            rows[4 * r + 2] = table[r].lo;
            rows[4 * r + 3] = table[r].hi;
        }
    return D3_OK;
}

}  // extern "C"

namespace d3 {

// rebuild from the current positions (auto-rebuild path); grows the lists
// if the previous build overflowed
int rebuild_grow(d3_ctx* c, const double* pos, hipStream_t s)
{
    double cell[9];
    int32_t pbc[3];
    std::memcpy(cell, c->cell, sizeof(cell));
    for (int k = 0; k < 3; k++) pbc[k] = c->geo.pbc[k];
    D3CHK(build(c, c->n, pos, c->type_copy.as<int32_t>(), cell, pbc, s));
    c->n_rebuilds++;
    int st = 0;
    D3CHK(read_status(c, s, &st));
    if (st & ST_CAPACITY) {
        int mc[8];
        D3CHK(list_stats(c, s, mc));
        c->cap_p = std::max(c->cap_p, mc[0] + std::max(16, mc[0] / 4));
        c->cap_c = std::max(c->cap_c, mc[1] + std::max(16, mc[1] / 4));
        c->cap_p = (c->cap_p + 3) & ~3;
        c->cap_c = (c->cap_c + 3) & ~3;
        const size_t N = (size_t)c->n;
        D3CHK(ensure(c->list_p, N * c->cap_p * sizeof(uint32_t)));
        D3CHK(ensure(c->list_c, N * c->cap_c * sizeof(uint32_t)));
        HIPCHK(hipMemsetAsync(c->status.p, 0, sizeof(int), s));
        D3CHK(run_build(c, pos, c->type_copy.as<int32_t>(), false, s));
        D3CHK(read_status(c, s, &st));
        if (st & ST_CAPACITY) return fail(D3_ERR_CAPACITY, "neighbour list capacity exceeded after regrow");
    }
    return D3_OK;
}

int evaluate(d3_ctx* c, int mode, double* energy, double* forces, double* virial,
             double* atom_energy, double* atom_virial, const double* vel, double* heat_current,
             int acc, hipStream_t s)
{
    const int n = (int)c->n;
    const Geo& g = c->geo;
    // per-atom virials: the direct part goes through Vp to the chain pass
    double* Vp = nullptr;
    if (atom_virial || heat_current) {
        D3CHK(ensure(c->Vp, (size_t)(n > 0 ? n : 1) * 6 * sizeof(double)));
        Vp = c->Vp.as<double>();
    }
    int cn_mode = mode == D3_MODE_PREC_F32 ? D3_MODE_PREC_F32 : D3_MODE_PLAIN_F64;
    if (mode == D3_MODE_SURROGATE) {
        if (!c->sur || !c->sur->trained)
            return fail(D3_ERR_NOT_TRAINED, "surrogate mode before training or loading weights");
        if (c->prm.damping != D3_DAMP_BJ)
            return fail(D3_ERR_INVALID_ARG, "the surrogate pass implements Becke-Johnson damping only");
        D3CHK(alloc_proj(c, D3_MODE_PREC_F32));
        cn_mode = D3_MODE_PREC_F32;  // surrogate needs float CNs; exact fallback uses Pf
    }
    D3CHK(coordination(c, cn_mode, s));
    PairScal sc;
    sc.s6 = c->prm.s6;
    sc.s8 = c->prm.s8;
    sc.rp2 = c->prm.r_pot * c->prm.r_pot;
    sc.rc2 = c->prm.r_cn * c->prm.r_cn;
    sc.zero = c->prm.damping == D3_DAMP_ZERO ? 1 : 0;
    sc.rs6sq = c->prm.rs6 * c->prm.rs6;
    sc.rs8sq = c->prm.rs8 * c->prm.rs8;
    phase_mark(c, PH_PAIR, s);
    int na = 0;
    if (mode == D3_MODE_SURROGATE) {
        D3CHK(surrogate_pair(c, sc, Vp, s, &na));
    } else if (mode == D3_MODE_LITERAL) {
        na = launch_pair_lit(n, c->pos_s.as<double4>(), c->img_tab.as<double4>(), g.n_img,
                             g.img_bits, c->list_p.as<uint32_t>(), c->cnt_p.as<int>(), c->cap_p,
                             c->d_tab.as<ElemTab>(), c->d_c6.as<double>(), c->d_pc.as<double4>(),
                             sc, c->cn.as<double>(), c->Fp.as<double>(), c->U.as<double>(),
                             c->G.as<double>(), Vp, c->vpart.as<double>(), s);
        HIPCHK(hipGetLastError());
    } else {
        na = launch_pair(mode, n, c->pos_s.as<double4>(), c->img_tab.as<double4>(), g.n_img,
                    g.img_bits, c->list_p.as<uint32_t>(), c->cnt_p.as<int>(), c->cap_p,
                    c->d_tab.as<ElemTab>(), c->d_c6.as<double>(), c->d_pc.as<double4>(), sc,
                    c->w.as<double>(), c->wd.as<double>(), c->P.as<double>(), c->Pf.as<float>(),
                    c->Fp.as<double>(), c->U.as<double>(),
                    c->G.as<double>(), Vp, c->vpart.as<double>(), s);
        HIPCHK(hipGetLastError());
    }
    phase_mark(c, PH_PAIR, s);
    // the three-body term adds to U, G, the direct forces and (per atom) Vp
    int n3 = 0;
    if (c->prm.s9 != 0.0) {
        phase_mark(c, PH_ATM, s);
        n3 = launch_atm(n, c->pos_s.as<double4>(), c->img_tab.as<double4>(), g.n_img, g.img_bits,
                        c->list_c.as<uint32_t>(), c->cnt_c.as<int>(), c->cap_c,
                        c->d_tab.as<ElemTab>(), c->n_elem, c->d_c6.as<double>(),
                        c->d_pc.as<double4>(), c->prm.s9, c->prm.r_atm * c->prm.r_atm,
                        c->w.as<double>(),
                        c->wd.as<double>(), c->Fp.as<double>(), c->U.as<double>(),
                        c->G.as<double>(), Vp, c->vpart3.as<double>(), s);
        phase_mark(c, PH_ATM, s);
        HIPCHK(hipGetLastError());
    }
    phase_mark(c, PH_CHAIN, s);
    const bool f64 = mode == D3_MODE_PLAIN_F64 || mode == D3_MODE_LITERAL;
    const int nb = launch_chain(f64 ? D3_MODE_PLAIN_F64 : D3_MODE_PREC_F32, n,
                 c->pos_s.as<double4>(), c->img_tab.as<double4>(), g.n_img, g.img_bits,
                 c->list_c.as<uint32_t>(), c->cnt_c.as<int>(), c->cap_c, c->d_tab.as<ElemTab>(),
                 sc.rc2, c->G.as<double>(), c->Fp.as<double>(), c->U.as<double>(),
                 c->perm.as<int>(), forces, atom_energy, Vp, vel, atom_virial, heat_current,
                 acc, c->vpart2.as<double>(), s);
    HIPCHK(hipGetLastError());
    launch_final(na, c->vpart.as<double>(), nb, c->vpart2.as<double>(), n3,
                 c->vpart3.as<double>(), energy, virial, acc, s);
    phase_mark(c, PH_CHAIN, s);
    HIPCHK(hipGetLastError());
    return D3_OK;
}

}  // namespace d3
