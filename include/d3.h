/*
 * d3.h -- C ABI of the MI355X (gfx950) D3(BJ) dispersion library.
 *
 * The library evaluates the D3 dispersion correction with Becke-Johnson
 * damping as stated by Ying & Fan, "Combining the D3 dispersion correction
 * with the neuroevolution machine-learned potential" (Sec. II A):
 *   Eq. 1   U = sum_i U_i
 *   Eq. 2   U_i = -1/2 sum_j [s6 C6_ij/(r^6 + (a1 R0 + a2)^6)
 *                           + s8 C8_ij/(r^8 + (a1 R0 + a2)^8)],  r < R_pot,
 *           C8 = C6 R0^2, R0 the geometric mean of per-species parameters
 *   Eq. 3   C6_ij(n_i, n_j): Gaussian-weighted (exponent -4) average of the
 *           reference C6 values over reference-CN pairs
 *   Eq. 4   n_i = sum_j 1/(1 + exp(-16 ((Rcov_i + Rcov_j)/r - 1))), r < R_cn
 *   Eqs. 5-7 forces and virial of this many-body energy.
 * The user supplies the damping parameters (the functional), R_pot and R_cn
 * (the three inputs the paper names), positions, species and the cell, and
 * receives energy, forces and virial; Eq. 9 (adding a short-range
 * potential) is served by the D3_ACCUMULATE flag.
 *
 * Conventions shared by every entry point:
 *  - Units: Angstrom, eV.  Reference C6 values are given in Hartree*bohr^6
 *    and r2r4 in bohr (the units D3 tables are published in); the library
 *    converts them once, on the host, in FP64.
 *  - Pointers documented "device" must point to memory of the current HIP
 *    device (e.g. a torch tensor's data_ptr()).  Pointers documented "host"
 *    are read before the call returns.  The caller owns all memory it
 *    passes; the library never frees it.
 *  - Positions are (n, 3) row-major FP64, atom order as the caller's.
 *    Cells are 3x3 row-major with the lattice vectors as rows (r = s @ cell).
 *  - "stream" is a hipStream_t (NULL = the default stream).  Work is
 *    enqueued asynchronously on it; outputs are valid once the stream has
 *    completed.  Conditions detected on the device (a species index out of
 *    range, neighbour-list overflow, an atom that moved more than half the
 *    skin) are recorded in the context and reported by d3_status().
 *  - Return value: 0 on success, a negative d3_status_code otherwise;
 *    d3_last_error() then holds a message (per calling thread).
 *  - One context may be used by one host thread at a time.  Calls on one
 *    context must be ordered (same stream, or synchronised by the caller).
 *  - Stream capture (HIP graphs): once a build of the same (n, cell, pbc)
 *    and the same call in the same mode have completed on the context
 *    (so that every buffer exists), d3_build_neighbors, d3_coordination,
 *    d3_energy_forces_virial and d3_evaluate (n > 0, flags without
 *    D3_AUTO_REBUILD, timing off; D3_REBUILD allowed) enqueue kernels
 *    only: no allocation,
 *    memset, copy or synchronisation, so they may be captured and the
 *    graph replayed on new positions written into the same buffers.
 *    d3_status, d3_list_stats, the first build of a geometry and
 *    D3_AUTO_REBUILD synchronise and must stay outside a capture.
 */
#ifndef D3_MI355X_H
#define D3_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define D3_MAX_REF 5   /* reference CNs per element */
#define D3_MAX_ELEM 16 /* elements per table */

typedef enum d3_status_code {
    D3_OK = 0,
    D3_ERR_INVALID_ARG = -1, /* bad pointer, size, parameter or cell */
    D3_ERR_HIP = -2,         /* a HIP runtime call failed */
    D3_ERR_CAPACITY = -3,    /* neighbour list overflowed (rebuild) */
    D3_ERR_STALE = -4,       /* an atom moved > skin/2 since the build */
    D3_ERR_CELL = -5,        /* singular cell or too many images */
    D3_ERR_STATE = -6,       /* call out of order (e.g. no build yet) */
    D3_ERR_NOT_TRAINED = -7, /* surrogate used before training/loading */
    D3_ERR_SPECIES = -8      /* a species index outside [0, n_elem) */
} d3_status_code;

/* Arithmetic of the pair pass. */
typedef enum d3_mode {
    D3_MODE_PLAIN_F64 = 0, /* everything in FP64 */
    D3_MODE_PREC_F32 = 1,  /* pair arithmetic in FP32, FP64 cutoff tests,
                              Gaussian weights and reductions */
    D3_MODE_SURROGATE = 2, /* C6 and its CN derivatives from the learned
                              per-element-pair MLP, exact Eq. 3 outside
                              the trained CN range */
    D3_MODE_LITERAL = 3    /* FP64 like D3_MODE_PLAIN_F64, but C6 from
                              Eq. 3 as printed: K_i K_j Gaussian weights
                              per pair instead of the factorised per-atom
                              weights (a reference; the same result up to
                              rounding, several times slower) */
} d3_mode;

/* Flags of d3_energy_forces_virial. */
#define D3_ACCUMULATE 1u   /* add into energy/forces/virial/atom_energy
                              instead of overwriting (Eq. 9: U = U_NEP+U_D3) */
#define D3_AUTO_REBUILD 2u /* rebuild the neighbour lists first if any atom
                              moved more than skin/2 since the last build
                              (synchronises the stream once) */
#define D3_REBUILD 4u      /* rebuild the neighbour lists from pos first, as
                              d3_build_neighbors would with the species, cell
                              and pbc of the last build, without a
                              synchronisation: one call per new configuration
                              (single-point evaluations).  List overflow is
                              then reported by d3_status, as after a build */

/* Two-body damping (d3_params.damping). */
#define D3_DAMP_BJ 0   /* Becke-Johnson, Eq. 2 */
#define D3_DAMP_ZERO 1 /* zero damping: -s_n C_n f_n / r^n with
                          f_n = 1 / (1 + 6 (r / (s_r,n R0))^-alpha_n),
                          alpha_6 = 14, alpha_8 = 16 (the variant the paper
                          sets aside before Eq. 1, as defined by the D3
                          reference it cites, Grimme et al. 2010) */

/* Damping parameters (Eq. 2) and cutoffs.  a2, r_pot, r_cn, skin, r_atm in
 * Angstrom; s6, a1, s8, rs6, rs8, s9 dimensionless.  Requires r_pot > 0,
 * r_cn > 0, skin >= 0.  Lists hold pairs within r_pot + skin and r_cn +
 * skin.  damping: D3_DAMP_BJ (uses a1, a2) or D3_DAMP_ZERO (uses rs6, rs8
 * > 0; R0 as for BJ, sqrt(3 r2r4_i r2r4_j)).  s9 != 0 adds the three-body
 * Axilrod-Teller-Muto term (also set aside by the paper; same reference):
 * over triangles whose three sides are below r_atm (0 < r_atm <= r_cn),
 * s9 sqrt(C6_AB C6_BC C6_CA) (1 + 3 cos A cos B cos C) / (r_AB r_BC
 * r_CA)^3 f3, f3 = 1 / (1 + 6 (rbar / (4/3 R0bar))^-16) with rbar and
 * R0bar the geometric means of the sides and of the pair radii, C6 from
 * Eq. 3 (exact in every mode), its CN dependence carried into the forces;
 * each atom of a triangle takes a third of its energy and virial. */
typedef struct d3_params {
    double s6, a1, s8, a2;
    double r_pot, r_cn, skin;
    int32_t mode;    /* d3_mode */
    int32_t damping; /* D3_DAMP_BJ or D3_DAMP_ZERO */
    double rs6, rs8; /* zero damping: s_r,6 and s_r,8 */
    double s9;       /* three-body scale; 0 = no three-body term */
    double r_atm;    /* three-body cutoff, 0 < r_atm <= r_cn when s9 != 0 */
} d3_params;

/* Reference table (Eqs. 3-4, host memory, copied by d3_create):
 *   n_ref[e]                 number of reference CNs of element e, 1..5
 *   cn_ref[e*5 + a]          reference CN a of element e
 *   c6_ref[((e*ne+f)*5+a)*5+b]  C6 reference of (e,a) with (f,b), Hartree
 *                            bohr^6; must satisfy c6_ref(e,f,a,b) =
 *                            c6_ref(f,e,b,a)
 *   rcov[e]                  effective covalent radius, Angstrom
 *   r2r4[e]                  sqrt(<r^4>/<r^2>)-type ratio, bohr; R0^2 =
 *                            3 r2r4_i r2r4_j and C8 = C6 R0^2 */
typedef struct d3_table {
    int32_t n_elem;
    const int32_t *n_ref;
    const double *cn_ref;
    const double *c6_ref;
    const double *rcov;
    const double *r2r4;
} d3_table;

typedef struct d3_ctx d3_ctx;

/* Create a context on the current HIP device.  Copies params and table
 * (converted to eV/Angstrom in FP64) to the device.  *out receives the
 * context; it owns all device scratch memory.  Errors: INVALID_ARG for a
 * NULL pointer, n_elem outside 1..D3_MAX_ELEM, n_ref outside 1..5,
 * non-positive cutoffs or negative skin, an asymmetric c6_ref; HIP. */
int d3_create(const d3_params *params, const d3_table *table, d3_ctx **out);

/* Free the context and its device scratch (synchronises the device).
 * NULL is accepted. */
void d3_destroy(d3_ctx *ctx);

/* Message for the last non-zero return on the calling thread. */
const char *d3_last_error(void);

/* Switch the pair-pass arithmetic (d3_mode) of an existing context. */
int d3_set_mode(d3_ctx *ctx, int32_t mode);

/* Bin the atoms of a periodic (or partly open) cell and build the
 * neighbour lists (cutoffs r_pot + skin and r_cn + skin).  n >= 0 atoms;
 * pos: device (n,3) FP64; type: device int32[n], element indices; cell:
 * host double[9]; pbc: host int32[3], 1 = periodic along that lattice
 * vector.  Atoms may lie outside the cell; they are wrapped on periodic
 * axes.  Along open axes the cell only sets the bin layout (atoms outside
 * it are still handled exactly, at some cost).  The first build for a new
 * (n, cell, pbc, cutoff) geometry sizes the lists and synchronises the
 * stream once; later builds are asynchronous.  Errors: INVALID_ARG, CELL
 * (singular cell, or n * images beyond the 32-bit list encoding), HIP.
 * Paper: the two neighbour sets within R_pot and R_cn (Eqs. 2 and 4). */
int d3_build_neighbors(d3_ctx *ctx, int64_t n, const double *pos,
                       const int32_t *type, const double *cell,
                       const int32_t *pbc, void *stream);

/* The positions the current neighbour lists were built from, exactly as
 * the caller passed them (unwrapped), in the caller's atom order.
 * pos_out: device (n,3) FP64.  A build from these positions gives the same
 * bins, sorted order and lists, so an MD checkpoint that keeps them next to
 * the positions and velocities resumes bit for bit: build from them with
 * d3_build_neighbors, then continue with d3_md_nve (whose stale test
 * measures displacements from them).  Asynchronous.  Errors: STATE (no
 * build), INVALID_ARG, HIP. */
int d3_build_positions(d3_ctx *ctx, double *pos_out, void *stream);

/* Coordination numbers, Eq. 4, for positions pos (device (n,3), same
 * atoms as the last build).  Keeps n_i in the context; if cn_out (device
 * double[n]) is not NULL, writes them there in the caller's atom order.
 * Errors: STATE (no build), INVALID_ARG, HIP. */
int d3_coordination(d3_ctx *ctx, const double *pos, double *cn_out,
                    void *stream);

/* Energy (Eqs. 1-2), forces (exact negative gradient: Eqs. 5-6 with the
 * chain term through the coordination numbers) and virial (Eq. 7 summed
 * over atoms, W = -dE/d(strain), eV) for positions pos (device (n,3)).
 * energy: device double[1]; forces: device double[n*3]; virial: device
 * double[9] row-major; atom_energy: device double[n] or NULL (site
 * energies U_i of Eq. 2).  Any output pointer except energy may be NULL.
 * flags: D3_ACCUMULATE, D3_AUTO_REBUILD, D3_REBUILD (which takes
 * precedence over D3_AUTO_REBUILD).  Errors: STATE, INVALID_ARG, HIP;
 * CAPACITY when the last build overflowed the lists and no rebuild flag is
 * given, or (D3_AUTO_REBUILD) when a rebuild could not fit them. */
int d3_energy_forces_virial(d3_ctx *ctx, const double *pos, double *energy,
                            double *forces, double *virial,
                            double *atom_energy, uint32_t flags,
                            void *stream);

/* Output pointers of d3_evaluate.  All are device memory in the caller's
 * atom order; energy is required, every other pointer may be NULL. */
typedef struct d3_outputs {
    double *energy;       /* double[1]: E, Eq. 1 (eV) */
    double *forces;       /* (n,3): exact negative gradient (eV/A) */
    double *virial;       /* double[9] row-major: Eq. 7 summed over atoms (eV) */
    double *atom_energy;  /* double[n]: site energies U_i, Eq. 2 (eV) */
    double *atom_virial;  /* (n,9) row-major per atom: W_i of Eq. 7 (eV) */
    const double *velocities; /* (n,3), any unit; read only for heat_current */
    double *heat_current; /* (n,3): J_i = W_i v_i, Eq. 8 (eV x velocity unit) */
} d3_outputs;

/* d3_energy_forces_virial with the per-atom virial of Eq. 7 and the
 * per-atom heat current of Eq. 8 as further optional outputs.  W_i is the
 * share of atom i in the virial: every entry (i, j, T) of i contributes
 * -1/2 [phi'(r) 1(r < R_pot) + (G_i + G_j) f'(r) 1(r < R_cn)] r (x) r / r
 * (each pair's term split evenly between its atoms), so sum_i W_i equals
 * the virial; for the direct part this is r_ij (x) dU_j/dr_ji as in Eq. 7.
 * J_i = W_i v_i needs velocities.  With D3_ACCUMULATE every requested
 * output is added to.  Requesting atom_virial or heat_current runs
 * variants of the dispersion and chain passes that also sum six tensor
 * components per atom; without them this call is d3_energy_forces_virial.
 * Errors: as d3_energy_forces_virial; INVALID_ARG if out or out->energy
 * is NULL or heat_current is given without velocities. */
int d3_evaluate(d3_ctx *ctx, const double *pos, const d3_outputs *out,
                uint32_t flags, void *stream);

/* Synchronise the stream of the last call and report (then clear) the
 * conditions the device recorded: SPECIES, INVALID_ARG (a non-finite
 * position: that atom was left out of every list and its results are not
 * meaningful), CAPACITY, STALE, or 0.  Writes into the lists stay within
 * their capacity; once an overflow has been seen, the lists count as
 * truncated: evaluations without D3_REBUILD or D3_AUTO_REBUILD return
 * CAPACITY until a build (which then sizes the lists again) replaces
 * them. */
int d3_status(d3_ctx *ctx);

/* Statistics of the last build: max and mean list lengths of the R_pot
 * and R_cn lists, number of bins, number of lattice images.  out: host
 * double[6].  Synchronises. */
int d3_list_stats(d3_ctx *ctx, double *out);

/* The bin layout a build would use, computed on the host only (no device
 * work; for inspection and tests).  cell: host double[9]; pbc: host
 * int32[3]; rlist: the longer list cutoff (R_pot or R_cn, plus the skin);
 * rcn: the R_cn list cutoff (<= rlist); n atoms.  Out: nb[3] bins and
 * reach[3] stencil reach along each lattice vector; *nrows rows of the
 * stencil row table (0: no table, the kernel walks the full stencil), of
 * which the first *ncnrows can hold pairs within rcn; rows (host int32
 * [4*max_rows] or NULL) receives (d1, d2, lo, hi) per row: bins (b0 + lo ..
 * b0 + hi, b1 + d1, b2 + d2) of home bin (b0, b1, b2), those whose nearest
 * points lie within rlist.  Errors: INVALID_ARG, CELL. */
int d3_bin_plan(const double *cell, const int32_t *pbc, double rlist,
                double rcn, int64_t n, int32_t *nb, int32_t *reach,
                int32_t *nrows, int32_t *ncnrows, int32_t *rows,
                int32_t max_rows);

/* Per-phase timing with HIP events recorded on the caller's stream around
 * each group of launches: 0 binning and counting sort of a neighbour
 * build, 1 position update, 2 CN and weights, 3 dispersion pass, 4 chain
 * pass with the final reductions, 5 list construction of a neighbour build
 * (a build is phases 0 and 5), 6 three-body pass.  enable = 1 starts (and
 * clears) the accumulation, 0 stops it. */
#define D3_N_PHASES 7
int d3_set_timing(d3_ctx *ctx, int32_t enable);

/* Summed milliseconds and number of timed calls per phase since timing was
 * enabled (host double[D3_N_PHASES], int64[D3_N_PHASES]).  Synchronises. */
int d3_get_timing(d3_ctx *ctx, double *ms, int64_t *calls);

/* ------------------------------------------------------------------------
 * Allocation-free evaluation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  One call does what d3_create, d3_build_neighbors and
 * d3_energy_forces_virial do together, for one small configuration and
 * without a context: every device buffer the library needs (converted
 * table, bins, lists, per-atom intermediates, partial sums, status) is
 * carved from one static device array of D3_NOALLOC_SCRATCH_BYTES, which
 * the library holds on each GPU it runs on until the process ends, and the
 * host side uses the stack only (about 150 KB).  No hipMalloc, hipFree or
 * other allocating routine is called.
 *   params, table: as for d3_create (mode PLAIN_F64, PREC_F32 or LITERAL;
 *     skin is used as in a build);  n <= D3_NOALLOC_MAX_ATOMS;
 *   pos, type, cell, pbc: as for d3_build_neighbors;
 *   energy, forces, virial, atom_energy: as for d3_energy_forces_virial
 *     (only energy is required);  flags: 0 or D3_ACCUMULATE.
 * The call synchronises the stream and returns the conditions the device
 * recorded (as d3_status would).  Because it synchronises, and copies the
 * converted table from host memory on every call, it is not itself meant
 * to be recorded into a HIP graph: it serves code around a capture (or in
 * a serving loop) that must not allocate.  Errors: INVALID_ARG (n beyond the limit,
 * surrogate mode, bad arguments), CAPACITY (more bins than 65536, more than
 * 1024 periodic images, or neighbour lists beyond the space left in the
 * array: about 7 million entries in all), CELL, SPECIES, HIP.  Calls on one
 * GPU share its array: calls that overlap on one GPU (two threads, or
 * unordered streams) race. */
#define D3_NOALLOC_MAX_ATOMS 4096
#define D3_NOALLOC_SCRATCH_BYTES (32u << 20)
int d3_energy_forces_virial_noalloc(const d3_params *params,
                                    const d3_table *table, int64_t n,
                                    const double *pos, const int32_t *type,
                                    const double *cell, const int32_t *pbc,
                                    double *energy, double *forces,
                                    double *virial, double *atom_energy,
                                    uint32_t flags, void *stream);

/* ------------------------------------------------------------------------
 * Learned C6 surrogate (per element pair: MLP (n_i, n_j) -> (C6,
 * dC6/dn_i, dC6/dn_j), widths 2 -> 32 -> 32 -> 3, SiLU).  Not part of the
 * paper: an approximation of Eq. 3 trained on samples that the exact
 * interpolation itself labels.
 * --------------------------------------------------------------------- */

#define D3_MLP_HIDDEN 32
/* parameters per element pair: 2*32+32 + 32*32+32 + 32*3+3 */
#define D3_MLP_PARAMS 1251

typedef struct d3_train_cfg {
    int64_t n_samples; /* total over all element pairs (>= pairs) */
    int32_t epochs;    /* passes over the sample set */
    int32_t batch;     /* samples per element pair per step (<= 1024) */
    double lr;         /* Adam step size */
    double lr_final;   /* step size at the last step (cosine decay) */
    uint64_t seed;     /* sample draw and shuffling */
    double cn_hi;      /* samples uniform in [0, cn_hi]^2; also the
                          trust box: pairs outside use exact Eq. 3 */
} d3_train_cfg;

/* Initialise the surrogate weights (Glorot-uniform, zero biases) from
 * seed, for all n_elem*(n_elem+1)/2 element pairs. */
int d3_c6_surrogate_init(d3_ctx *ctx, uint64_t seed);

/* Draw cfg->n_samples CN pairs, label them with exact Eq. 3 on the GPU,
 * and train every element pair's network with the library's own forward,
 * backward and Adam kernels (FP32).  final_loss: host double[1], the mean
 * standardised squared error of the last epoch.  Synchronises. */
int d3_c6_surrogate_train(d3_ctx *ctx, const d3_train_cfg *cfg,
                          double *final_loss, void *stream);

/* Evaluate the surrogate for m queries: elem_i, elem_j device int32[m];
 * cn_i, cn_j device float[m]; out device float[m*3] = (C6 in eV A^6,
 * dC6/dn_i, dC6/dn_j).  precision: 0 = FP32 reference forward, 1 = the
 * BF16-MFMA inference kernel used inside the pair pass. */
int d3_c6_surrogate_eval(d3_ctx *ctx, int64_t m, const int32_t *elem_i,
                         const int32_t *elem_j, const float *cn_i,
                         const float *cn_j, float *out, int32_t precision,
                         void *stream);

/* Exact Eq. 3 at the same queries (device buffers as above; out FP64
 * (m,3)), the surrogate's training labels and judge. */
int d3_c6_exact_eval(d3_ctx *ctx, int64_t m, const int32_t *elem_i,
                     const int32_t *elem_j, const double *cn_i,
                     const double *cn_j, double *out, void *stream);

/* Copy the FP32 master weights and standardisation constants to/from host
 * memory.  Layout: for each pair p (e <= f, row-major over e then f):
 * W1[2][32], b1[32], W2[32][32], b2[32], W3[32][3], b3[3] (= 1251 floats),
 * then for all pairs the 3 output means and 3 output scales, then the
 * trust bound cn_hi.  bytes must equal d3_c6_surrogate_bytes(ctx). */
int64_t d3_c6_surrogate_bytes(d3_ctx *ctx);
int d3_c6_surrogate_get_weights(d3_ctx *ctx, float *host_buf, int64_t bytes);
int d3_c6_surrogate_set_weights(d3_ctx *ctx, const float *host_buf,
                                int64_t bytes);

/* One training step on explicit samples (tests: gradient check against
 * the CPU reference).  x: device float[m*2], the network inputs (cn_i,
 * cn_j) already mapped to [-1, 1] by x = 2 cn / cn_hi - 1; y: device
 * float[m*3] standardised targets, pair: device int32[m]; grads: device
 * float[pairs*1251] receives the mean-squared-error gradient; loss: device
 * float[1].  No weight update. */
int d3_c6_surrogate_grad(d3_ctx *ctx, int64_t m, const int32_t *pair,
                         const float *x, const float *y, float *grads,
                         float *loss, void *stream);

/* One training step on explicit samples (tests: the optimiser against the
 * CPU reference).  m, pair, x, y as for d3_c6_surrogate_grad.  Computes
 * each pair's mean-squared-error gradient over its samples, then applies
 * the update d3_c6_surrogate_train makes: Adam (moment decays 0.9 and
 * 0.999, epsilon 1e-8, bias corrections for step + 1) with the cosine step
 * size of step `step` (0-based) of total_steps, lr_final + (lr - lr_final)
 * (1 + cos(pi step / total_steps)) / 2.  Updates the context's FP32
 * weights, Adam moments (zeroed by d3_c6_surrogate_init) and inference
 * weights; pairs without samples are left unchanged.  Synchronises.
 * Errors: INVALID_ARG (sizes, step outside 0..total_steps, lr <= 0),
 * NOT_TRAINED (no init), HIP. */
int d3_c6_surrogate_adam_step(d3_ctx *ctx, int64_t m, const int32_t *pair,
                              const float *x, const float *y, int64_t step,
                              int64_t total_steps, double lr,
                              double lr_final, void *stream);

/* ------------------------------------------------------------------------
 * Velocity-Verlet NVE molecular dynamics driven by the D3 forces (the MD
 * use of the paper's Sec. II D, here without thermostat).
 * pos, vel: device (n,3) FP64, updated in place (Angstrom, Angstrom/fs);
 * mass: device double[n] (amu); dt in fs.  Runs n_steps steps, rebuilding
 * the lists when an atom moved more than skin/2.  thermo: host double
 * array of (n_steps/every + 1) * 3 values (potential, kinetic, total
 * energy, eV) recorded every `every` steps from step 0, or NULL.
 * rebuilds: host int64[1] or NULL, the number of list builds made.  A build
 * must precede the first call.  The decision to rebuild is taken on the
 * device each step (no host synchronisation); the stream is synchronised
 * every 16 steps, at thermo records and at the end, and a list overflow
 * found there sends the run back to the state saved at the previous such
 * point, with grown lists.  Errors: STATE, INVALID_ARG, HIP; CAPACITY if
 * the lists overflowed repeatedly; after the run, SPECIES or INVALID_ARG if
 * the device recorded a bad species index or a non-finite position during
 * it (the run then went on with contained values and its results are not
 * meaningful). */
int d3_md_nve(d3_ctx *ctx, int64_t n_steps, double dt, double *pos,
              double *vel, const double *mass, int32_t every, double *thermo,
              int64_t *rebuilds, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* D3_MI355X_H */
