// Allocation-free evaluation of one small configuration, for callers that
// cannot allocate device memory.  Every device buffer the library would
// otherwise allocate in a context (the converted table, bins, sorted
// positions, neighbour lists, per-atom intermediates, partial sums and the
// status word) is carved out of one file-scope static device array,
// `scratch`, of D3_NOALLOC_SCRATCH_BYTES per GPU, which the library holds
// until the process ends.  The host side keeps to the stack: the context,
// the converted table and the staging of images and stencil rows are
// local arrays, and the shared build and evaluation code runs with
// allocation switched off (a buffer that would have to grow is an error).
//
// The array's name is a host-side stand-in in host code: its device
// address is looked up once per device with hipGetSymbolAddress and only
// that address is handed to kernels, copies and memsets.  Calls on one GPU
// share its array; calls that overlap on one GPU (two host threads, or two
// streams without ordering) race.
#include <mutex>

#include "d3_ctx.h"

namespace d3 {

constexpr size_t NA_BYTES = D3_NOALLOC_SCRATCH_BYTES;
constexpr int NA_MAX_ATOMS = D3_NOALLOC_MAX_ATOMS;
constexpr int NA_MAX_BINS = 65536;  // bins of one build
constexpr int NA_MAX_IMG = 1024;    // periodic images the stencil reaches
constexpr int NA_MAX_ROWS = (int)MAX_ROW_TAB;
constexpr int NA_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[NA_MAX_DEVICES];

// Device address of the current device's scratch array (looked up with that
// device current, once per device).
static int scratch_address(int dev, void** out)
{
    if (dev < 0 || dev >= NA_MAX_DEVICES)
        return fail(D3_ERR_INVALID_ARG, "device %d beyond the %d devices supported", dev,
                    NA_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(D3_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return D3_OK;
}

// Consecutive 256-byte aligned pieces of the scratch array.
struct Carver {
    char* base;
    size_t off, cap;
    bool take(Buf& b, size_t bytes)
    {
        off = (off + 255) & ~(size_t)255;
        if (bytes > cap || off > cap - bytes) return false;
        b.p = base + off;
        b.bytes = bytes;
        off += bytes;
        return true;
    }
};

// allocation stays switched off for the whole call on this thread
struct NoAllocScope {
    bool prev;
    NoAllocScope() : prev(g_no_alloc) { g_no_alloc = true; }
    ~NoAllocScope() { g_no_alloc = prev; }
};

}  // namespace d3

using namespace d3;

extern "C" int d3_energy_forces_virial_noalloc(const d3_params* prm, const d3_table* tab,
                                               int64_t n, const double* pos,
                                               const int32_t* type, const double* cell,
                                               const int32_t* pbc, double* energy,
                                               double* forces, double* virial,
                                               double* atom_energy, uint32_t flags,
                                               void* stream)
{
    D3CHK(check_params_table(prm, tab));
    if (prm->mode == D3_MODE_SURROGATE)
        return fail(D3_ERR_INVALID_ARG, "the surrogate mode needs a context (trained weights)");
    if (n > NA_MAX_ATOMS)
        return fail(D3_ERR_INVALID_ARG, "n=%lld atoms exceeds the allocation-free limit of %d",
                    (long long)n, NA_MAX_ATOMS);
    D3CHK(check_build_args(n, pos, type, cell, pbc));
    if (!energy) return fail(D3_ERR_INVALID_ARG, "energy is NULL");
    if (flags & ~D3_ACCUMULATE) return fail(D3_ERR_INVALID_ARG, "only D3_ACCUMULATE is accepted");
    const int acc = (flags & D3_ACCUMULATE) ? 1 : 0;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    void* base = nullptr;
    D3CHK(scratch_address(dev, &base));
    if (n == 0) {
        if (!acc) {
            HIPCHK(hipMemsetAsync(energy, 0, sizeof(double), s));
            if (virial) HIPCHK(hipMemsetAsync(virial, 0, 9 * sizeof(double), s));
        }
        HIPCHK(hipStreamSynchronize(s));
        return D3_OK;
    }

    // host side: the table in eV / Angstrom and the geometry staging
    // (about 150 KB of stack)
    ElemTab et;
    double c6[MAXELEM * MAXELEM * MAXREF * MAXREF];
    double4 pc[MAXELEM * MAXELEM];
    double4 imgs[NA_MAX_IMG];
    RowSpan rows[NA_MAX_ROWS];
    convert_table(prm, tab, et, c6, pc);

    d3_ctx c;
    c.prm = *prm;
    c.n_elem = tab->n_elem;
    c.device = dev;
    c.h_tab = et;
    c.stage_fixed = true;
    c.h_img = imgs;
    c.h_rows = rows;
    c.h_img_cap = NA_MAX_IMG;
    c.h_rows_cap = NA_MAX_ROWS;
    int h_status = 0;
    c.h_status = &h_status;
    c.last_stream = s;

    // carve every device buffer out of the scratch array
    const size_t N = (size_t)NA_MAX_ATOMS;
    const size_t nparts = (size_t)max_pass_blocks() * 8 * sizeof(double);
    Carver cv{(char*)base, 0, NA_BYTES};
    bool ok = cv.take(c.d_tab, sizeof(ElemTab)) &&
              cv.take(c.d_c6, sizeof(double) * MAXELEM * MAXELEM * MAXREF * MAXREF) &&
              cv.take(c.d_pc, sizeof(double4) * MAXELEM * MAXELEM) && cv.take(c.status, 256) &&
              cv.take(c.maxcnt, 256) && cv.take(c.bin_of, N * sizeof(int)) &&
              cv.take(c.shift, N * sizeof(double4)) && cv.take(c.perm, N * sizeof(int)) &&
              cv.take(c.perm_tmp, N * sizeof(int)) && cv.take(c.pos_s, N * sizeof(double4)) &&
              cv.take(c.shift_s, N * sizeof(double4)) && cv.take(c.ref_s, N * sizeof(double4)) &&
              cv.take(c.type_copy, N * sizeof(int32_t)) && cv.take(c.cn, N * sizeof(double)) &&
              cv.take(c.cnf, N * sizeof(float)) && cv.take(c.w, N * MAXREF * sizeof(double)) &&
              cv.take(c.wd, N * MAXREF * sizeof(double)) && cv.take(c.G, N * sizeof(double)) &&
              cv.take(c.Fp, N * 3 * sizeof(double)) && cv.take(c.U, N * sizeof(double)) &&
              cv.take(c.cnt_p, N * sizeof(int)) && cv.take(c.cnt_c, N * sizeof(int)) &&
              cv.take(c.P, N * NPIECE * 4 * sizeof(double)) &&
              cv.take(c.Pf, N * NPIECEF * 4 * sizeof(float)) &&
              cv.take(c.vpart, nparts) && cv.take(c.vpart2, nparts) &&
              cv.take(c.vpart3, nparts) &&
              cv.take(c.count, 2 * ((size_t)NA_MAX_BINS + 1) * sizeof(int)) &&
              cv.take(c.bin_start, ((size_t)NA_MAX_BINS + 2) * sizeof(int)) &&
              cv.take(c.scan_tmp, ((size_t)NA_MAX_BINS / 1024 + 5) * sizeof(int)) &&
              cv.take(c.slab, 16 * sizeof(int)) &&
              cv.take(c.img_tab, (size_t)NA_MAX_IMG * sizeof(double4)) &&
              cv.take(c.row_tab, (size_t)NA_MAX_ROWS * sizeof(RowSpan));
    // the rest holds the two lists, shared in the ratio of the cutoff spheres
    const double rp = prm->r_pot + prm->skin, rc = prm->r_cn + prm->skin;
    const size_t left = ok ? (NA_BYTES - ((cv.off + 255) & ~(size_t)255)) / 1024 * 1024 : 0;
    const double fp = rp * rp * rp / (rp * rp * rp + rc * rc * rc);
    const size_t lp = (size_t)((double)left * fp) / 1024 * 1024;
    ok = ok && left > 2048 && cv.take(c.list_p, lp) && cv.take(c.list_c, left - lp - 256);
    if (!ok) return fail(D3_ERR_CAPACITY, "static scratch layout does not fit %zu bytes", NA_BYTES);

    HIPCHK(hipMemcpyAsync(c.d_tab.p, &et, sizeof(et), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c.d_c6.p, c6, sizeof(c6), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(c.d_pc.p, pc, sizeof(pc), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(c.status.p, 0, sizeof(int), s));

    NoAllocScope scope;
    D3CHK(build(&c, n, pos, type, cell, pbc, s));
    D3CHK(evaluate(&c, prm->mode, energy, forces, virial, atom_energy, nullptr, nullptr, nullptr,
                   acc, s));
    int st = 0;
    D3CHK(read_status(&c, s, &st));
    return status_code(st);
}
