// Host-side context of the library (opaque d3_ctx of the C ABI).
#pragma once

#include <cstdarg>
#include <string>
#include <vector>

#include "d3_internal.h"

// return from the calling function on a failed HIP call or library call
#define HIPCHK(call)                                      \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

#define D3CHK(call)                 \
    do {                            \
        int r_ = (call);            \
        if (r_ != D3_OK) return r_; \
    } while (0)

namespace d3 {

constexpr double BIN_DIV = 3.0;     // bins per list cutoff along each axis (at most)
constexpr double BIN_ATOMS = 2.6;   // mean atoms per bin for long cutoffs
constexpr double MAX_REACH = 16.0;  // deepest stencil reach that narrower bins may give

struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
    template <class T>
    T* as() const { return (T*)p; }
};

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
int ensure_bytes(void** p, size_t* have, size_t need);
inline int ensure(Buf& b, size_t need) { return ensure_bytes(&b.p, &b.bytes, need); }
void release(Buf& b);

// learned C6 surrogate state (mlp.hip)
struct Surrogate {
    int n_pairs = 0;
    bool trained = false;
    float cn_hi = 0.0f;
    Buf w32;       // FP32 master weights, n_pairs * D3_MLP_PARAMS
    Buf stats;     // per pair: mean[3], scale[3] (FP32)
    Buf adam_m, adam_v, grad;
    Buf packed;    // inference pack (bf16 layer-2 weights + fp32 rest)
    Buf samples;   // training inputs/targets
    Buf loss;      // per-step losses
    std::vector<float> h_w;  // host copy (get/set)
};

struct d3_ctx_impl;

}  // namespace d3

struct d3_ctx {
    d3_params prm{};
    int n_elem = 0;
    int device = 0;
    d3::ElemTab h_tab{};
    std::vector<double> h_c6;
    double h_r2r4[D3_MAX_ELEM] = {};
    d3::Buf d_tab, d_c6, d_pc;
    // geometry of the last build
    int64_t n = 0;
    double cell[9] = {};
    d3::Geo geo{};
    bool built = false;
    bool counts_clean = false;  // bin counts and scatter cursors are zero
    // a build overflowed its lists (seen in the status word): the lists are
    // truncated until a build sizes them again
    bool lists_bad = false;
    // smallest list capacities a sizing build may choose (raised after an
    // overflow seen during MD, from the counts that overflowed)
    int min_cap_p = 0, min_cap_c = 0;
    // host staging of the image translations and stencil row table of a
    // build: growable vectors, or fixed arrays (stage_fixed) given by the
    // allocation-free entry point
    std::vector<double4> img_store;
    std::vector<d3::RowSpan> rows_store;
    double4* h_img = nullptr;
    d3::RowSpan* h_rows = nullptr;
    size_t h_img_cap = 0, h_rows_cap = 0;
    bool stage_fixed = false;
    // cell-sorted data
    d3::Buf bin_of, shift, count, bin_start, scan_tmp, perm_tmp, perm, slab;
    d3::Buf pos_s, shift_s, ref_s, type_copy, img_tab, row_tab;
    // lists
    d3::Buf list_p, cnt_p, list_c, cnt_c;
    int cap_p = 0, cap_c = 0;
    // per-atom results
    d3::Buf cn, cnf, w, wd, P, Pf, G, Fp, U, Vp, vpart, vpart2, vpart3;
    // status
    d3::Buf status, maxcnt;
    int* h_status = nullptr;
    hipStream_t last_stream = nullptr;
    d3::Surrogate* sur = nullptr;
    // MD scratch and the number of list rebuilds made by D3_AUTO_REBUILD
    d3::Buf md_scratch;
    int64_t n_rebuilds = 0;
    // phase timing (events recorded around launch groups)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_phase;  // phase of each begin/end pair
    size_t ev_used = 0;
    double t_ms[D3_N_PHASES] = {};
    int64_t t_calls[D3_N_PHASES] = {};

    std::vector<d3::Buf*> all_buffers()
    {
        return {&d_tab, &d_c6, &d_pc, &bin_of, &shift, &count, &bin_start,
                &scan_tmp, &perm_tmp, &perm, &slab, &pos_s, &shift_s, &ref_s, &type_copy,
                &img_tab, &row_tab, &list_p, &cnt_p, &list_c, &cnt_c, &cn, &cnf, &w, &wd, &P,
                &Pf, &G, &Fp, &U, &Vp, &vpart, &vpart2, &vpart3, &status, &maxcnt, &md_scratch};
    }
};

namespace d3 {

extern thread_local bool g_no_alloc;
int check_params_table(const d3_params* prm, const d3_table* tab);
void convert_table(const d3_params* prm, const d3_table* tab, ElemTab& et, double* c6,
                   double4* pc);
int check_build_args(int64_t n, const double* pos, const int32_t* type, const double* cell,
                     const int32_t* pbc);
int build(d3_ctx* c, int64_t n, const double* pos, const int32_t* type, const double* cell,
          const int32_t* pbc, hipStream_t s);
int rebuild_grow(d3_ctx* c, const double* pos, hipStream_t s);
// binning, sort and lists on stream s (size_lists: count first and size the
// lists, one synchronisation); need: a device flag gating the whole build
int run_build(d3_ctx* c, const double* pos, const int32_t* type, bool size_lists, hipStream_t s,
              const int* need = nullptr);
int update_positions(d3_ctx* c, const double* pos, hipStream_t s);
int coordination(d3_ctx* c, int mode, hipStream_t s);
int evaluate(d3_ctx* c, int mode, double* energy, double* forces, double* virial,
             double* atom_energy, double* atom_virial, const double* vel, double* heat_current,
             int acc, hipStream_t s);
int read_status(d3_ctx* c, hipStream_t s, int* out);
int list_stats(d3_ctx* c, hipStream_t s, int* mc);  // max/sum of the last build's list lengths
int status_code(int bits);
int alloc_proj(d3_ctx* c, int mode);

// phase timing
enum Phase { PH_BUILD = 0, PH_UPDATE = 1, PH_CN = 2, PH_PAIR = 3, PH_CHAIN = 4, PH_LIST = 5,
             PH_ATM = 6 };
void phase_mark(d3_ctx* c, int phase, hipStream_t s);  // call twice: begin, end
int timing_flush(d3_ctx* c);

// surrogate (mlp.hip)
void surrogate_free(d3_ctx* c);
int surrogate_pair(d3_ctx* c, const PairScal& sc, double* Vp, hipStream_t s, int* nblk);

}  // namespace d3
