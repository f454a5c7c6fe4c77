/*
 * dao.h -- C ABI of the MI355X (gfx950) column-generation direct aperture
 * optimisation library.
 *
 * Model (Men, Jia & Jiang, "GPU-based ultra-fast direct aperture
 * optimization for online adaptive radiation therapy"):
 *   - Section 2.1, eq. 1 and eq. 2: voxel dose z_j = sum_k D_kj y_k with the
 *     aperture coefficients D_kj = sum_{i in A_k} D_ij; eq. 7: beamlet
 *     intensity x_i = sum_{k in K_i} y_k, so z = D x.
 *   - Discussion, eq. 9 and eq. 10: per-structure one-sided quadratic
 *     penalties (under-dose on targets, over-dose on every structure), each
 *     weight divided by the structure's voxel count.
 *   - eq. 6: min F(z) over y >= 0 with z defined by eq. 1.
 *   - Section 2.2 and Section 2.3: column generation; the master is solved by
 *     gradient projection, the pricing sub-problem (eq. 8) by a per-row
 *     minimum-sum leaf interval and a per-beam argmin.
 *
 * Conventions shared by every call
 *   - Voxels are numbered 0..n_vox-1 in the caller's order; beamlets
 *     0..n_blt-1 beam by beam, then MLC row by row, then position within the
 *     row (each row is a contiguous run of beamlet numbers).
 *   - Leaf positions are row-local, 0-based, half-open [L, R); a closed row
 *     is (0, 0).  An aperture is one beam plus one (L, R) pair per row of that
 *     beam.
 *   - "ctx type" is the storage/arithmetic type chosen at create time:
 *     DAO_F64 -> double, DAO_F32 -> float.  Device vectors passed to
 *     dao_dose / dao_gradient use the ctx type.  Objective values, reduced
 *     costs, gaps, intensities y and the master's dose are always double.
 *   - Device pointers are plain HIP device addresses (for example a torch
 *     tensor's data_ptr()).  All device work is enqueued on the stream given
 *     to dao_create; calls that return host values synchronise that stream.
 *   - A context is not thread-safe; use one per plan and per host thread.
 *   - Every call returns a dao_status.  On failure the context keeps a
 *     message readable with dao_last_error(); dao_create failures are
 *     described by dao_create_error() (thread-local).
 */
#ifndef DAO_H
#define DAO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dao_ctx dao_ctx;

typedef enum {
    DAO_OK = 0,
    DAO_EOPTIMAL = 1,   /* dao_solve stopped: no aperture prices below -tau */
    DAO_ESTALLED = 2,   /* dao_solve stopped: pricing kept returning a pool member */
    DAO_ENOTCONV = 3,   /* dao_master_solve stopped at max_steps with the KKT residual still
                           above tol; the state is valid (not an error) */
    DAO_EINVAL = -1,    /* malformed argument; nothing was changed */
    DAO_ENOMEM = -2,    /* device allocation failed or exceeded mem_cap_bytes */
    DAO_EDEVICE = -3,   /* a HIP call failed */
    DAO_ESTATE = -4     /* call not valid in the context's current state */
} dao_status;

typedef enum { DAO_F64 = 0, DAO_F32 = 1 } dao_dtype;

/* Beamlet dose matrix D (eq. 2's D_ij): voxel-row CSR on the host.
 * row_ptr[n_vox + 1] non-decreasing from 0 to nnz; col[nnz] strictly
 * increasing inside each row, each in [0, n_blt); val[nnz] finite and >= 0.
 * Limits: n_blt <= 65535 (columns are stored as 16-bit indices on the
 * device), nnz < 2^31.  Values are rounded to the ctx type on upload. */
typedef struct {
    int64_t n_vox, n_blt, nnz;
    const int64_t* row_ptr;
    const int32_t* col;
    const double* val;
} dao_matrix;

/* Beam and MLC geometry (Section 2.3: rows of n beamlets per beam).
 * rows_per_beam[n_beams] >= 1 each; row_len[sum rows_per_beam] in [1, 64];
 * sum(row_len) must equal n_blt. */
typedef struct {
    int32_t n_beams;
    const int32_t* rows_per_beam;
    const int32_t* row_len;
} dao_beams;

/* Structure label of every voxel (eq. 9 and eq. 10's v_s): vox_struct[n_vox]
 * in [-1, n_struct), -1 = in no structure.  n_struct <= 255.
 * vox_struct2 (optional, NULL = none): a second label per voxel for
 * overlapping structures, whose terms add to the first label's (eq. 10 sums
 * over every structure containing the voxel; nested targets such as PTV1
 * inside PTV2, Section 3).  -1, or a structure other than the voxel's first
 * label, which must then be set.  |v_s| counts both labels.  At most 255
 * distinct (first, second) pairs plus single labels.
 * vox_shift (optional, NULL = none): per-voxel threshold shift tau_j (finite):
 * every threshold of voxel j is T_s + tau_j (eq. 3 and eq. 4's per-voxel
 * T_j).  The re-optimization mode of the Discussion (alpha_j = beta_j = 1,
 * T_j = the deformed dose of the original plan) is one target structure and
 * one structure for all other voxels, thresholds 0, weights equal to the
 * structure sizes, and tau = T. */
typedef struct {
    int32_t n_struct;
    const int16_t* vox_struct;
    const int16_t* vox_struct2;
    const double* vox_shift;
} dao_structures;

/* One prescription per structure (eq. 9 and eq. 10): targets (is_target != 0)
 * are penalised below t_under with weight w_under and above t_over with
 * weight w_over; other structures only above t_over.  Weights are divided by
 * the structure's voxel count on the device.  Requires finite values,
 * w_under, w_over >= 0, and t_under <= t_over for targets. */
typedef struct {
    int32_t is_target;
    double t_under, t_over, w_under, w_over;
} dao_prescription;

/* Options; fill with dao_default_options() and change what you need. */
typedef struct {
    int32_t dtype;          /* DAO_F64 or DAO_F32 (default DAO_F32) */
    int32_t max_apertures;  /* pool capacity, 1..256 (default 64) */
    double eps;             /* master stops at KKT residual <= eps * |rc_1| (1e-6) */
    int32_t max_steps;      /* master steps per round (500) */
    double tau_rel;         /* aperture enters iff rc < -tau_rel * |rc_1| (1e-10) */
    int32_t max_tighten;    /* eps tightenings on a duplicate aperture (3) */
    int32_t refresh_every;  /* recompute d = D(A y) every this many steps (50) */
    int32_t ls_slots;       /* line-search launches per master cycle (2) */
    int64_t mem_cap_bytes;  /* fail dao_create with DAO_ENOMEM above this device footprint; 0 = none */
    int32_t master;         /* DAO_MASTER_APERTURE (default) or DAO_MASTER_BEAMLET, see below */
    int32_t d_format;       /* storage of D's values: DAO_DFMT_NATIVE (default: the ctx
                               dtype) or, for DAO_F32 with the aperture master,
                               DAO_DFMT_F16 / DAO_DFMT_BF16, see below */
    int32_t d_residual;     /* with a 16-bit d_format: 1 also stores the FP16 residual and
                               uses it in every product; 0 (default) the 16-bit values only;
                               2 stores it and uses it selectively: in the plan's last
                               residual_rounds rounds (where D_K is also rebuilt in FP32 when
                               dk_format is DAO_DFMT_F16), and to price again any earlier
                               decision whose gap is within the 16-bit values' rounding bound
                               (4 u sum_{i in A} (D^T |grad F|)_i, u = 2^-11 FP16, 2^-8 BF16) */
    int32_t persistent;     /* aperture master: 2 (default) runs each master solve as one
                               cooperative launch when the device supports it, each
                               workgroup holding its rows of D_K, d and q in LDS when they
                               fit, else only its d, q and classes (D_K streamed), else as 1;
                               1 is that launch streaming D_K, d and q from device memory on
                               every pass; 0 launches each phase of each step separately */
    int32_t product_tune;   /* 1 (default): dao_create times the variants of the two
                               sparse products (how many loads each thread keeps in
                               flight, and for native values whether x is staged on
                               chip) and keeps the fastest; 0: the two fields below
                               choose.  The variants add the same terms in the same
                               order, so results do not depend on the choice */
    int32_t dose_variant;   /* with product_tune 0: forward product variant, 0 (default)
                               x staged on chip, 4 slices of 64 rows per workgroup;
                               1 as 0 with 8 entries per lane in flight; 2 x read from
                               device memory with 8 in flight (native d_format only);
                               3 as 0 with 8 slices per workgroup; 4, 5, 6 whole rows
                               per lane (every entry group of a row in flight, x staged
                               once per workgroup) on a grid of 1, 2 or 4 workgroups of
                               256 threads per compute unit, each walking slices with
                               the grid's stride; 7, 8 as 5, 6 with each wavefront's
                               slices from a list balanced by slice width at creation
                               (widest first, to the least-loaded wavefront) */
    int32_t gradient_depth; /* with product_tune 0: transposed product entries per thread
                               in flight, 4 (default), 8 or 16 */
    int32_t direction;      /* master search direction (Section 2.3, gradient projection):
                               DAO_DIR_CONJUGATE (default) or DAO_DIR_STEEPEST, see below */
    int32_t apertures_per_round; /* 1 (default): one aperture enters per round (Section 2.3).
                               m in [2, 16]: after it, the beams ranked 2..m by their best
                               aperture's value (ties to the lowest beam) add their
                               apertures too, each if its value is below -tau, it is not
                               pooled and the budget allows; one master solve follows */
    int32_t dk_format;      /* storage of the aperture dose matrix D_K (eq. 1 and eq. 2) the
                               aperture master streams: DAO_DFMT_NATIVE (default: the ctx
                               dtype) or, for DAO_F32, DAO_DFMT_F16: FP16 values of D_K over
                               the largest entry of D (half the bytes per master pass, about
                               2.4e-4 relative rounding per entry); products accumulate in
                               FP32 / FP64 as before; or, for DAO_F32, DAO_DFMT_AUTO: a plan
                               starts with D_K in FP32 and moves it to FP16 (its columns
                               rebuilt once) before the first column that would make the pool
                               too large for the persistent master's on-chip form (from the
                               start when that form is off: persistent 0 or 1); the buffer is
                               FP32-sized.  dao_info_t.dk_format reports the storage now */
    int32_t residual_rounds; /* with d_residual 2: the plan's last this many rounds (5) run in
                               the accurate form, see d_residual */
    int32_t graphs;         /* 1: the pricing sequence of every round (exact FP64 dose,
                               objective, FP64 prices, pricing scan, result copy) replays,
                               on the context stream, a HIP graph captured at its first use
                               (one per residual setting) on a stream the context creates
                               for that; 0 (default): the same launches one by one.  Same
                               results */
} dao_options;

/* Search direction of the master's gradient projection.  r is the projected
 * negative gradient over the pool: r_k = -dF/dy_k, except 0 where y_k = 0 and
 * dF/dy_k >= 0.  DAO_DIR_STEEPEST moves along r.  DAO_DIR_CONJUGATE moves along
 * r + beta p_prev, with beta = max(0, r.(r - r_prev) / r_prev.r_prev), when the
 * pool's previous step did not block and had the same free set (where r may
 * be non-zero) and the result is a descent direction; otherwise along r.  The
 * memory is cleared when an aperture enters the pool, on dao_reset and
 * dao_set_state, and after a blocking step.  It is kept across consecutive
 * dao_master_step / dao_master_solve calls on the same pool. */
enum { DAO_DIR_STEEPEST = 0, DAO_DIR_CONJUGATE = 1 };

/* How the restricted master evaluates its two products per step.
 * DAO_MASTER_APERTURE keeps the aperture dose matrix D_K (eq. 1 and eq. 2:
 * D_kj = sum_{i in A_k} D_ij) on the device, one column per pool aperture,
 * appended when the aperture enters; each step streams it twice
 * (q = D_K p, dF/dy = D_K^T grad F).  Needs max_apertures <= 64.
 * DAO_MASTER_BEAMLET evaluates the same products through the beamlet
 * matrix and the pool map: q = D (A p), dF/dy = A^T (D^T grad F) (eq. 7). */
enum { DAO_MASTER_APERTURE = 0, DAO_MASTER_BEAMLET = 1 };

/* Reduced-precision storage of D (products accumulate in FP32; the
 * objective total, line search, convergence and reduced-cost tests stay
 * FP64).  Each beamlet column i gets an FP32 scale s_i = max_j D_ij (1 for
 * an empty column); each entry stores hi = RNE(D_ij / s_i) in FP16 or BF16
 * and, with d_residual, lo = RNE_FP16(D_ij / s_i - hi), so that
 * D_ij ~= s_i (hi + lo).  The scale is applied to x before the forward
 * product and to each column sum of the transposed product.  Needs
 * n_blt * 4 bytes of x to fit the on-chip staging (n_blt <= 12288). */
enum { DAO_DFMT_NATIVE = 0, DAO_DFMT_F16 = 1, DAO_DFMT_BF16 = 2, DAO_DFMT_AUTO = 3 /* dk_format only */ };

/* The host encoder of that storage, for inspection and tests: for each of
 * n ratios r[i] (finite, >= 0) writes hi[i] (the 16-bit pattern of
 * RNE(r) in d_format) and, if lo is not NULL, lo[i] (the FP16 pattern of
 * RNE(r - hi)).  DAO_EINVAL for a native or unknown format or a bad r. */
dao_status dao_encode_values(int32_t d_format, int64_t n, const double* r, uint16_t* hi, uint16_t* lo);

void dao_default_options(dao_options* opt);

/* Validate the inputs, build the device layouts and upload them (one copy;
 * the caller keeps ownership of every host array).  `stream` is a
 * hipStream_t (NULL = default stream) on the current HIP device.  On
 * success *out owns all device memory until dao_destroy.  Returns DAO_EINVAL
 * for any malformed input before touching the device. */
dao_status dao_create(const dao_matrix* D, const dao_beams* beams,
                      const dao_structures* structs, const dao_prescription* presc,
                      const dao_options* opt, void* stream, dao_ctx** out);
void dao_destroy(dao_ctx* ctx);
const char* dao_last_error(const dao_ctx* ctx);
const char* dao_create_error(void);

/* Sizes and device footprint. */
typedef struct {
    int64_t n_vox, n_vox_nonempty, n_blt, nnz, n_rows;
    int32_t n_beams, max_rows_per_beam, dtype, n_slices;
    int64_t sell_entries;     /* stored forward-layout entries incl. padding */
    int64_t device_bytes;     /* device memory held by the context */
    int32_t d_format;         /* storage of D's values (DAO_DFMT_*) */
    int32_t d_residual;       /* 1 when the FP16 residual is stored and used */
    int64_t bytes_dose;       /* algorithmic HBM bytes of one forward product */
    int64_t bytes_gradient;   /* algorithmic HBM bytes of one transposed product */
    int32_t dose_variant;     /* forward product variant in use (as dao_options.dose_variant) */
    int32_t gradient_depth;   /* transposed product: entries per thread in flight (4, 8, 16) */
    int32_t last_master_form; /* how the last master solve ran: -1 none yet, 0 one launch per
                                 phase, 1 persistent launch streaming D_K, d and q, 2 persistent
                                 launch with each workgroup's rows (D_K, d, q) on chip, 5
                                 persistent launch streaming D_K with each workgroup's d and q
                                 on chip, 3 / 4 / 6 the batched launch in forms 1 / 2 / 5 */
    int32_t onchip_lds_bytes; /* dynamic LDS a workgroup of the persistent launch may use for
                                 its rows (0: the on-chip form is unavailable) */
    int32_t dk_format;        /* storage of D_K now (DAO_DFMT_NATIVE or DAO_DFMT_F16) */
    int32_t residual_reprices; /* d_residual 2: decisions priced again with the residual in the
                                 last plan (or since the last reset) */
} dao_info_t;
dao_status dao_info(const dao_ctx* ctx, dao_info_t* out);

/* d = D x (eq. 1 and eq. 2 with x from eq. 7).  x_dev: n_blt values, d_dev:
 * n_vox values, both ctx type, caller-order, device.  Every d entry is
 * written (voxels no beamlet reaches get 0). */
dao_status dao_dose(dao_ctx* ctx, const void* x_dev, void* d_dev);

/* g = D^T grad F(d) (eq. 8's w_i with pi = grad F) and F(d) over all voxels
 * (eq. 9 and eq. 10).  d_dev: n_vox ctx-type values; g_dev: n_blt ctx-type
 * values; *F receives the objective (double). */
dao_status dao_gradient(dao_ctx* ctx, const void* d_dev, void* g_dev, double* F);

/* Pricing sub-problem (eq. 8, Section 2.3) on prices g (n_blt doubles on the
 * device): per row the minimum-sum leaf interval (ties: smallest right end,
 * then smallest left end; a row with no negative interval stays closed),
 * per-beam sums, argmin over beams (ties: lowest beam).  Outputs the beam,
 * leaves[2 * rows of that beam] as (L, R) pairs, the reduced cost *rc (the
 * beam value) and the decision gap *gap (distance to the runner-up beam or
 * to the runner-up interval of any chosen row, whichever is smaller). */
dao_status dao_price(dao_ctx* ctx, const double* g_dev, int32_t* beam, int16_t* leaves,
                     double* rc, double* gap);

/* For callers that cannot allocate device memory or call allocating library
 * routines during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid it): dao_price with the same arguments,
 * outputs and errors, whose pricing launch keeps its scratch (per-row
 * records, the result and the arrival counters) in a static device array of
 * the library instead of the context's buffers.  The call allocates nothing;
 * the array's address is looked up once per device when the first context on
 * that device is created.  Limit: at most 4096 MLC rows (DAO_EINVAL above).
 * Every call on one device uses the same array and leaves its contents
 * behind (the counters are cleared at the start of each call): calls that
 * overlap on one device, from any thread or stream, race. */
dao_status dao_price_noalloc(dao_ctx* ctx, const double* g_dev, int32_t* beam, int16_t* leaves,
                             double* rc, double* gap);

/* Master state.  dao_reset empties the pool (y = 0, dose 0).
 * dao_add_aperture appends an aperture with y = 0 (leaves as in dao_price;
 * DAO_EINVAL for a malformed aperture, DAO_ESTATE when the pool is full). */
dao_status dao_reset(dao_ctx* ctx);
dao_status dao_add_aperture(dao_ctx* ctx, int32_t beam, const int16_t* leaves);

/* One gradient-projection iteration of the restricted master (Section 2.3)
 * over the current pool: gradient over the pool, projected direction,
 * longest feasible step, exact line search, update.  Returns the objective
 * after the step (*F), the KKT residual max_k |min(y_k, dF/dy_k)| after the
 * step (*kkt) and the step length (*step, 0 if already at a KKT point). */
dao_status dao_master_step(dao_ctx* ctx, double* F, double* kkt, double* step);

/* Gradient projection until KKT residual <= tol or max_steps steps.
 * Returns DAO_OK when the residual reached tol (or the projected direction
 * vanished) and DAO_ENOTCONV when the step cap ended the solve first. */
dao_status dao_master_solve(dao_ctx* ctx, double tol, int32_t max_steps,
                            int32_t* steps, double* kkt, double* F);

/* Prices at the current intensities in FP64 and returns the entering
 * aperture (same outputs as dao_price).  The master dose is first
 * recomputed as D (A y) with FP64 products and sums (eq. 7, eq. 1), so the
 * prices (eq. 8 with pi = grad F) are those of the current y, not of the
 * master's incrementally updated dose; the master continues from that dose. */
dao_status dao_price_current(dao_ctx* ctx, int32_t* beam, int16_t* leaves,
                             double* rc, double* gap);

/* Copy the pool (entry order) and intensities to the host.  beams[cap],
 * leaves[cap * 2 * max_rows_per_beam] (row-major per aperture, unused rows
 * left as is), y[cap]; *n receives the pool size.  Any pointer may be NULL. */
dao_status dao_get_pool(dao_ctx* ctx, int32_t cap, int32_t* n, int32_t* beams,
                        int16_t* leaves, double* y);

/* Master dose (double, caller voxel order, n_vox values) into a device
 * buffer, and the objective at it. */
dao_status dao_get_dose(dao_ctx* ctx, double* d_dev, double* F);

/* Mean device time, in microseconds, of `iters` back-to-back launches of one
 * product kernel on the context stream, measured with HIP events: kernel 0
 * is the forward product d = D x (Section 2.1, eq. 1, eq. 2, eq. 7; the
 * kernel behind dao_dose), kernel 1 the transposed product g = D^T u (the
 * w_i of eq. 8; the kernel behind dao_gradient).  Inputs are the master's
 * current vectors, outputs go to context scratch memory.  For measurement
 * only; the master state is left unchanged. */
dao_status dao_time_product(dao_ctx* ctx, int32_t kernel, int32_t iters, double* us_per_launch);

/* As dao_time_product, with the caches cold: before each of the `iters`
 * launches a kernel reads scrub_bytes (>= 1 MiB, a multiple of 16) of the
 * caller-owned device buffer `scrub`, displacing D and the vectors from the
 * L2 and last-level caches with clean lines; only the product launch is
 * timed (one event pair per launch, the mean is returned).  The scrub
 * buffer is only read (its first 16 bytes may be written in the unlikely
 * case that a thread's XOR of its words hits a fixed pattern).  DAO_EINVAL
 * for a bad kernel, iters < 1 or a bad scrub size. */
dao_status dao_time_product_cold(dao_ctx* ctx, int32_t kernel, int32_t iters, void* scrub,
                                 int64_t scrub_bytes, double* us_per_launch);

/* The reference for those figures: a plain streaming read (16-byte loads,
 * grid-stride, 2048 workgroups of 256 threads, the kernel that scrubs) of
 * the first `bytes` bytes of the caller-owned device buffer `buf`, timed as
 * dao_time_product_cold times a product (scrub read first, one event pair
 * per launch); *us_per_launch is the mean.  buf is only read (its first 16
 * bytes may be written as for the scrub buffer).  bytes >= 16, a multiple
 * of 16; DAO_EINVAL otherwise or for a bad scrub size or iters < 1. */
dao_status dao_time_read_cold(dao_ctx* ctx, void* buf, int64_t bytes, int32_t iters, void* scrub,
                              int64_t scrub_bytes, double* us_per_launch);

/* Launch-level measurement of one kernel of the aperture-matrix master
 * (Section 2.3's master, evaluated as in DAO_MASTER_APERTURE): after
 * dao_profile_start(ctx, kernel) every launch of that kernel is bracketed by
 * HIP events on the context stream, and the kernel accumulates its
 * algorithmic bytes on the device (launches that find nothing to do add
 * none).  kernel: 0 update pass (apply step, grad F, F, grad_y partials),
 * 1 q pass (q = D_K p with the first line-search evaluation), 2 line-search
 * pass, 3 direction, 4 the persistent master (one launch per master solve;
 * its bytes are the sum over its update, q and line-search passes).  dao_profile_stop synchronises and returns the number
 * of launches, how many did work, their summed event time (us) and summed
 * algorithmic bytes, then disables the events.  DAO_ESTATE for the beamlet
 * master or a stop without a start.  For measurement runs only: the events
 * add a little host and queue overhead. */
dao_status dao_profile_start(dao_ctx* ctx, int32_t kernel);
dao_status dao_profile_stop(dao_ctx* ctx, int64_t* launches, int64_t* working_launches,
                            double* total_us, double* total_bytes);

/* Split of the persistent master's time in the last profiling window of
 * kernel 4, as seen by its workgroup 0 (device wall clock), into us[7]:
 * update passes, their grid reductions, direction, first line-search passes
 * (q = D_K p), line-search grid reductions, final decisions and y updates,
 * later line-search passes (with the decision before each).  Zeros when
 * the last window was another kernel's.  Reductions include waiting for the
 * slowest workgroup. */
dao_status dao_profile_phases(dao_ctx* ctx, double* us);

/* Per-round log and outcome of dao_solve.  The arrays are caller-owned with
 * room for n_apertures entries each; any may be NULL. */
typedef struct {
    int32_t rounds;           /* apertures added */
    int32_t stop;             /* DAO_OK (budget reached), DAO_EOPTIMAL or DAO_ESTALLED */
    double F;                 /* final objective */
    double rc1;               /* reduced cost of round 1 */
    int64_t total_steps;      /* master steps over all rounds */
    int64_t total_ls_evals;   /* line-search evaluations over all rounds */
    int32_t* round_beam;
    double* round_rc;
    double* round_gap;
    int32_t* round_steps;
    double* round_kkt;
    double* round_F;
    double price_s;           /* host wall-clock seconds in pricing (incl. the gradient refresh) */
    double master_s;          /* host wall-clock seconds in column building and master solves */
    int32_t* round_stop;      /* why each round's master stopped: 1 KKT residual <= tol,
                                 2 step cap (max_steps) reached first, 3 zero projected direction */
    int32_t capped_rounds;    /* rounds whose master stopped at the step cap */
} dao_plan;

/* Column generation (Section 2.2, Section 2.3) from an empty pool: round 1
 * prices at zero dose; each round prices in FP64, stops when rc >= -tau
 * (DAO_EOPTIMAL), tightens the master tolerance and re-solves when pricing
 * returns a pool member (at most max_tighten times, then DAO_ESTALLED),
 * otherwise adds the aperture and solves the master to
 * eps * |rc_1| or max_steps.  Stops after n_apertures apertures. */
dao_status dao_solve(dao_ctx* ctx, int32_t n_apertures, dao_plan* out);

/* Checkpoint and resume of a plan (also used to restore an arbitrary pool and
 * intensities, e.g. a reference solve's state, before pricing or a master
 * solve).  The state is the pool in entry order, y, and the column-generation
 * loop's scalars below; the dose is not part of it: dao_set_state recomputes
 * it as D (A y) in FP64, which is also the dose every round's pricing uses,
 * so a plan resumed from a checkpoint taken between rounds repeats the
 * uninterrupted plan. */
typedef struct {
    int32_t n;          /* pool size */
    int32_t tighten;    /* master tolerance tightenings so far */
    double rc1;         /* reduced cost of round 1 (NaN: no round priced yet) */
    double eps;         /* current master tolerance factor (tolerance = eps * |rc1|) */
    double last_step;   /* length of the last master step (0 if none) */
    double prev_step;   /* length of the step before it (the next line search starts there) */
} dao_state_info;

/* Copy the state out: beams[cap], leaves[cap * 2 * max_rows_per_beam]
 * (layout of dao_get_pool), y[cap] and *info.  DAO_EINVAL if cap is smaller
 * than the pool. */
dao_status dao_get_state(dao_ctx* ctx, int32_t cap, int32_t* beams, int16_t* leaves, double* y,
                         dao_state_info* info);

/* Replace the pool and intensities by info->n apertures (arrays laid out as
 * dao_get_state's) and y[info->n] (finite, >= 0), and set the loop scalars.
 * Rebuilds the aperture dose matrix, the dose D (A y) (FP64), the objective
 * and the prices.  DAO_EINVAL for a malformed aperture or value (nothing is
 * changed then). */
dao_status dao_set_state(dao_ctx* ctx, const dao_state_info* info, const int32_t* beams,
                         const int16_t* leaves, const double* y);

/* Column generation continued from the current pool (dao_set_state or an
 * earlier solve) under dao_solve's rules, with the loop's rc1, eps and
 * tightenings carried over, until the pool holds n_apertures.  The plan's
 * round arrays cover the rounds of this call. */
dao_status dao_solve_resume(dao_ctx* ctx, int32_t n_apertures, dao_plan* out);

/* Several independent solves advanced together (the serving form): each
 * round prices every live solve and adds its column, then one cooperative
 * launch runs all their master solves, the grid's workgroups shared out in
 * proportion to their voxel rows; a solve leaves when it stops.  Every solve
 * follows exactly dao_solve's rules, so each plan is the one dao_solve gives
 * (up to the order of floating-point sums, which depends on how many
 * workgroups a solve gets).  Contexts must be distinct and share the dtype;
 * the shared launch needs the persistent aperture master on one stream
 * (otherwise the master solves run one after another).  plans[i] receives
 * solve i's log (may be NULL); the return is DAO_OK or the first error. */
dao_status dao_solve_batch(dao_ctx* const* ctxs, int32_t n, const int32_t* n_apertures, dao_plan* plans);

/* Serving loop (continuous batching).  Requests are queued in arrival order.
 * The server's admission threads (`workers`) take them in that order while
 * fewer than max_live solves are live, admitted or being built.  Each lays
 * out the request's inputs on the host, reserves the context's predicted
 * device footprint under hbm_cap_bytes (0: no cap; a request whose
 * footprint does not fit waits until retirements free enough memory, and
 * fails with DAO_ENOMEM if it exceeds the cap alone), then allocates and
 * uploads on a stream of its own; a request is admitted when its context is
 * ready, so requests built at the same time may be admitted out of arrival
 * order.  Context creation thus overlaps the device work of the live
 * solves.  Each dao_server_step takes the admitted contexts in and advances
 * every live solve by one column-generation round.  With batch_masters the
 * master solves of the small solves (fewer than 4 row batches per workgroup
 * of the whole grid) share one launch as in dao_solve_batch and each larger
 * one keeps the whole grid; otherwise they all run one after another.  A solve that stops is retired at once: its
 * context (dose matrix, dose, master state) is destroyed and its result is
 * kept for dao_server_poll.  Each result is the plan dao_solve gives for the
 * same request up to the order of floating-point sums.  The host arrays of
 * a request must stay valid until its ticket is admitted.  All work runs on
 * `stream`; the server's calls are made from one thread. */
typedef struct dao_server dao_server;
typedef struct {
    int32_t max_live;        /* solves advanced together, 1..64 */
    int32_t batch_masters;   /* 1: the round's master solves share one launch (dao_solve_batch);
                                0: each runs with the whole grid, one after another */
    int64_t hbm_cap_bytes;   /* device bytes of the admitted contexts; 0 = no cap */
    int32_t workers;         /* admission threads building contexts at once, 0..16 (0: 4) */
} dao_server_options;
dao_status dao_server_create(const dao_server_options* opt, void* stream, dao_server** out);
void dao_server_destroy(dao_server* srv);
/* Queue one request (dao_solve of n_apertures on these inputs and options,
 * NULL options = defaults); *ticket identifies it. */
dao_status dao_server_submit(dao_server* srv, const dao_matrix* D, const dao_beams* beams,
                             const dao_structures* structs, const dao_prescription* presc,
                             const dao_options* opt, int32_t n_apertures, int64_t* ticket);
/* Admit, then one round of every live solve.  *n_live: live solves after the
 * step; *n_done: solves retired in it.  A device error ends every live solve
 * with that error and is returned. */
dao_status dao_server_step(dao_server* srv, int32_t* n_live, int32_t* n_done);
/* *state: 0 queued, 1 live, 2 done.  When done, fills *out (arrays as in
 * dao_solve, may be NULL), forgets the ticket and returns the solve's status
 * (DAO_OK, DAO_EOPTIMAL, DAO_ESTALLED or an error).  DAO_EINVAL for an unknown
 * or already collected ticket. */
dao_status dao_server_poll(dao_server* srv, int64_t ticket, int32_t* state, dao_plan* out);
dao_status dao_server_info(const dao_server* srv, int32_t* queued, int32_t* live, int64_t* used_bytes);

#ifdef __cplusplus
}
#endif
#endif /* DAO_H */
