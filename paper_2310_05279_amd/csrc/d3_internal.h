// Internal declarations shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/d3.h"

namespace d3 {

constexpr int WAVE = 64;
constexpr int MAXREF = D3_MAX_REF;
constexpr int MAXELEM = D3_MAX_ELEM;
constexpr int BLOCK = 256;          // 4 waves per workgroup
constexpr int WAVES_PER_BLOCK = BLOCK / WAVE;
// Per-atom neighbour data of the dispersion pass (position and Gaussian
// weights), in pieces stored in blocks of a few atoms, piece-major inside a
// block (piece q of atom j at piece_at(np, blk, q, j)): the lanes of a wave
// that read one piece of neighbours lying close together in the sorted
// order share cache lines, and all the pieces of an atom lie in one block.
//  FP64 form, 2 pieces of 32 bytes, 4 atoms per block: (x, y, z, w0),
//    (w1, w2, w3, w4); the species is carried by the sign bits of w0..w3
//    (bit k of the species in the sign of w_k): every weight is >= 0, so
//    the reader takes |w| and loses nothing;
//  FP32 form, 3 pieces of 16 bytes, 8 atoms per block: (x, y), (z, (w0,
//    w1)), (w2, w3, w4, species), the position in FP64, the weights in FP32
//    and the species as an int.
constexpr int NPIECE = 2;   // FP64 form: 32-byte pieces
constexpr int PBLK = 4;     // FP64 form: atoms per block
constexpr int NPIECEF = 3;  // FP32 form: 16-byte pieces
constexpr int PBLKF = 8;    // FP32 form: atoms per block
// index, in pieces, of piece q of atom j (np pieces per atom, blk atoms per block)
__host__ __device__ inline size_t piece_at(int np, int blk, int q, size_t j)
{
    return ((j / blk) * np + q) * blk + (j % blk);
}
static_assert(MAXELEM <= 16, "four sign bits carry the species in the FP64 form");

// device status bits (OR-ed by kernels, read by d3_status)
constexpr int ST_SPECIES = 1;
constexpr int ST_CAPACITY = 2;
constexpr int ST_STALE = 4;
constexpr int ST_NONFINITE = 8;

// Bin layout and periodic images of one build.
struct Geo {
    double H[9];     // lattice vectors as rows
    double Hinv[9];  // s_k = sum_m r_m Hinv[m*3+k]
    int pbc[3];
    int nb[3];       // bins along each lattice vector
    int reach[3];    // stencil reach in bins
    int timg[3];     // max |t_k| of image translations
    int img_bits;    // list entry = (j << img_bits) | image
    int n_img;
    int nbins;
    int nrows;       // rows of the stencil row table (0: no table, every row)
    int ncnrows;     // the first ncnrows rows can hold pairs within the R_cn list cutoff
};

// One stencil row of the list build with a row table: bins (b0 + lo ..
// b0 + hi, b1 + d1, b2 + d2) of the home bin (b0, b1, b2), the bins of the
// row whose nearest points lie within the list cutoff.
struct RowSpan {
    int d1, d2, lo, hi;
};
constexpr long MAX_ROW_TAB = 4096;  // largest stencil (rows) given a row table
constexpr int ROW_TABLE_REACH = 4;  // a row table from this stencil reach on

// Per-element data used inside kernels (kept in global memory).
struct ElemTab {
    int n_elem;
    int n_ref[MAXELEM];
    double cn_ref[MAXELEM * MAXREF];
    double rcov[MAXELEM];
};

// Scalars of the dispersion pass.
struct PairScal {
    double s6, s8;
    double rp2, rc2;  // evaluation cutoffs squared (no skin)
    int zero;           // zero damping (pair constants 6 (rs6 R0)^14, 6 (rs8 R0)^16, R0^2, s8 R0^2)
    double rs6sq, rs8sq;  // zero damping: rs6^2, rs8^2
};

// ---- launchers (cells.hip) --------------------------------------------
// The build kernels take `need`: NULL, or a device flag read first by every
// thread, the whole kernel doing nothing while it is 0 (a rebuild decided
// on the device, with no host synchronisation).
void launch_bin(int n, const double* pos, const int32_t* type, int n_elem,
                const Geo& g, int* bin_of, double4* shift, int* count,
                int32_t* type_copy, int* status, hipStream_t s, const int* need = nullptr);
void launch_scan(int nbins, const int* count, int* bin_start, int* tmp, hipStream_t s,
                 const int* need = nullptr);
void launch_scatter(int n, const int* bin_of, const int* bin_start, int* fill,
                    int* perm_tmp, hipStream_t s, const int* need = nullptr);
// nbins: the bins of the geometry; bin nbins holds the atoms left out of the
// lists (non-finite positions), whose list counts k_rank sets to zero
void launch_rank(int n, const int* perm_tmp, const int* bin_of, const int* bin_start,
                 const double* pos, const int32_t* type_copy, const double4* shift,
                 int* perm, double4* pos_s, double4* shift_s, double4* ref_s, int nbins,
                 int* slab, int* count, int* cnt_p, int* cnt_c, hipStream_t s,
                 const int* need = nullptr);
void launch_list(int n, const double4* pos_s, const int* bin_start, const int* slab, const Geo& g,
                 const RowSpan* row_tab,
                 const double4* img_tab, double rp2, double rc2, uint32_t* list_p,
                 int* cnt_p, int cap_p, uint32_t* list_c, int* cnt_c, int cap_c,
                 int count_only, int* status, hipStream_t s, const int* need = nullptr);
void launch_cnt_stats(int n, const int* cnt_p, const int* cnt_c, int* out, hipStream_t s);
// copies the caller's positions into the sorted layout; an atom that moved
// more than half the skin ORs stale_bit into *stale_out
void launch_update(int n, const double* pos, const int* perm,
                   const double4* shift_s, const double4* ref_s,
                   double4* pos_s, double half_skin2, int* status,
                   int* stale_out, int stale_bit, hipStream_t s);

// ---- launchers (cn.hip, disp.hip, chain.hip) --------------------------
// Workgroups of BLOCK threads for a pass whose waves take `units` work
// items one at a time (atoms, groups of atoms, bins), a whole number of
// 8-workgroup groups (one per XCD in turn).  When the resident waves of the
// kernel (from its occupancy) would get at most 8 units each, the grid is
// exactly the resident waves, so no tail round follows; otherwise it holds
// up to MAX_WAVES_PER_SIMD waves per SIMD, so that waves finishing early
// are replaced and the XCDs end together.
constexpr int MAX_WAVES_PER_SIMD = 24;
int pass_blocks(const void* kernel, int units, size_t dyn_lds = 0);
// upper bound of pass_blocks on this device (sizing of per-block partials)
int max_pass_blocks();
void launch_cn(int mode, int n, const double4* pos_s, const double4* img_tab, int n_img,
               int img_bits, const uint32_t* list_c, const int* cnt_c, int cap_c,
               const ElemTab* tab, double rc2, double* cn, double* w, double* wd, double* W,
               float* Wf, hipStream_t s);
int launch_pair(int mode, int n, const double4* pos_s, const double4* img_tab, int n_img,
                 int img_bits, const uint32_t* list_p, const int* cnt_p, int cap_p,
                 const ElemTab* tab, const double* c6ref, const double4* pc, PairScal sc,
                 const double* w, const double* wd, const double* W, const float* Wf, double* Fp,
                 double* U, double* G, double* Vp, double* part, hipStream_t s);
int launch_pair_lit(int n, const double4* pos_s, const double4* img_tab, int n_img, int img_bits,
                    const uint32_t* list_p, const int* cnt_p, int cap_p, const ElemTab* tab,
                    const double* c6ref, const double4* pc, PairScal sc, const double* cn,
                    double* Fp, double* U, double* G, double* Vp, double* part, hipStream_t s);
int launch_chain(int mode, int n, const double4* pos_s, const double4* img_tab, int n_img,
                  int img_bits, const uint32_t* list_c, const int* cnt_c, int cap_c,
                  const ElemTab* tab, double rc2, const double* G, const double* Fp,
                  const double* U, const int* perm, double* forces, double* atom_energy,
                  const double* Vp, const double* vel, double* atom_virial,
                  double* heat_current, int accumulate, double* part, hipStream_t s);
void launch_final(int na, const double* part_a, int nb, const double* part_b, int nc,
                  const double* part_c, double* energy, double* virial, int accumulate,
                  hipStream_t s);
int launch_atm(int n, const double4* pos_s, const double4* img_tab, int n_img, int img_bits,
               const uint32_t* list_c, const int* cnt_c, int cap_c, const ElemTab* tab,
               int n_elem, const double* c6ref, const double4* pc, double s9, double ra2,
               const double* w, const double* wd, double* Fp, double* U, double* G, double* Vp,
               double* part, hipStream_t s);
void launch_scatter_out(int n, const double* src, const int* perm, double* dst, hipStream_t s);
void launch_build_pos(int n, const int* perm, const double4* ref_s, double* out, hipStream_t s);

}  // namespace d3
