/*
 * bf.h - C ABI of the MI355X (gfx950) N-term bilateral filter library.
 *
 * The filter is Eq. (BF) of Dai, Yuan, Zhang, "Speeding up the Bilateral
 * Filter: A Joint Acceleration Way" (IEEE TIP; arXiv 1803.00004):
 *
 *   out(p) = sum_q K_s(p - q) K_r(I(p) - I(q)) I(q) / sum_q K_s(p - q) K_r(I(p) - I(q))
 *
 * over the in-image pixels q of the (2r+1)^2 window, with K_s replaced by its
 * best N_s-term Haar expansion (Sec. IV-B, Eq. Haar_N_terms, box form of
 * App. A) and K_r by its best N_r-term truncated cosine expansion (Sec. IV-C,
 * Eq. trigonometric_N_terms).  The cosine shift identity (Eq. 1D_N_terms)
 * turns each range term into four linear filters of modulated images, each
 * evaluated as a sum of 2-D box sums read from summed-area tables (Sec.
 * III-D, Eqs. sum_sat_2D .. sum_sat_sum_region_2D).
 *
 * A plan selects the kernels (Gaussian or exponential, bf_kernel_t, or
 * tables of any symmetric kernels, bf_plan_create_tabulated) and the
 * way the filter is computed: the N-term expansion above (default); Eq. BF
 * summed directly (BF_FLAG_DIRECT / _AUTO); the paper's own 8-bit regime
 * with the range box over the 256 intensity levels (BF_FLAG_RANGE_BOX); the
 * expansion for 8-bit input with its range terms folded per output level
 * (BF_FLAG_LEVEL_FOLD); or the expansion with FP16 term images
 * (BF_PREC_REDUCED).
 *
 * Conventions (all functions):
 *  - Images are row-major and contiguous (pitch = W elements), H x W, with
 *    1 <= H, W <= 32768.  Pointers named I/out/ws are DEVICE pointers.
 *  - Intensities are float32 in [0, span] (default span 1) or uint8 (read as
 *    byte / 255).  Values outside [0, span] or NaN give an unspecified (but
 *    memory-safe) result.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *    Filtering calls only enqueue work and never synchronise the host; a
 *    device fault shows up as BF_ERR_DEVICE from the launch check or at the
 *    caller's next synchronisation.
 *  - Every function returns a bf_status_t; on an error nothing is enqueued.
 *  - Plans are immutable after creation and may be shared by threads, except
 *    that bf_filter (no workspace argument) grows a workspace owned by the
 *    plan and is therefore not safe to call concurrently on one plan;
 *    concurrent callers use bf_filter_ws with their own workspaces.
 */
#ifndef BF_H
#define BF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bf_plan_s *bf_plan_t;

typedef enum {
  BF_OK = 0,
  BF_ERR_INVALID_ARG = 1,   /* bad pointer, size, parameter, or workspace too small */
  BF_ERR_OUT_OF_MEMORY = 2, /* a device or host allocation failed */
  BF_ERR_DEVICE = 3,        /* a HIP call or kernel launch failed */
  BF_ERR_UNSUPPORTED = 4    /* valid request the library does not implement */
} bf_status_t;

/* Kernel shapes.  Eq. BF takes symmetric kernels decreasing on R+ and the
 * expansions of Sec. III-IV take any such kernel (only their coefficients
 * change):
 *   GAUSSIAN     G_sigma(x) = exp(-x^2 / 2 sigma^2) (Sec. I); as K_s the
 *                separable exp(-(dx^2 + dy^2) / 2 sigma_s^2); K^{-1}(eps) =
 *                sigma sqrt(2 ln(1/eps)).
 *   EXPONENTIAL  exp(-|x| / sigma); as K_s the radial, not separable
 *                exp(-sqrt(dx^2 + dy^2) / sigma_s), whose 2-D Haar
 *                coefficients are integrated numerically (radius <= 511);
 *                K^{-1}(eps) = sigma ln(1/eps).
 * K_s and K_r are chosen independently.  Other kernels are given as tables
 * (bf_plan_create_tabulated). */
typedef enum { BF_KERNEL_GAUSSIAN = 0, BF_KERNEL_EXPONENTIAL = 1 } bf_kernel_t;

/* Expansion sizes: n_range cosine terms (1..64) of K_r, n_spatial Haar level
 * groups (1..(J+2)^2, J = floor(log2(radius + 1/2))) of K_s.  A level group is
 * every 2-D Haar function phi/psi_{j,.}(x) times phi/psi_{j',.}(y) of one pair
 * of levels; groups are kept in decreasing L2 energy (best N-term, Sec. III-A). */
typedef struct {
  int n_range;
  int n_spatial;
} bf_terms_t;

typedef enum { BF_IN_F32 = 0, BF_IN_U8 = 1 } bf_dtype_t;

/* PLAIN: int32 summed-area tables (exact box sums), FP32 tap sums and
 * accumulation; max-abs error against the FP64 expanded form about 1e-6.  REDUCED: the term images are
 * stored once in FP16 (2 bytes per pixel and table, no halo copies) and the
 * lookup kernel builds each table of its output tile in LDS from them (exact
 * int32 sums of the FP16 values); the error is the FP16 rounding of the term
 * values, a few 1e-5.  REDUCED needs every tap in a symmetric quadruplet
 * (at most 12) and a region of at most 128 x 128 for its 32 x 32 output
 * tiles (radius <= 48), and neither DIRECT nor RANGE_BOX (BF_ERR_INVALID_ARG);
 * else BF_ERR_UNSUPPORTED.  Workspace: n_images H W 2 bytes; no pre-computed
 * tables, no autotuning. */
typedef enum { BF_PREC_PLAIN = 0, BF_PREC_REDUCED = 1 } bf_precision_t;

#define BF_FLAG_HOST_ONLY 0x1u /* fit tables on the host only; no device work, no filtering */
/* Direct summation (the paper's brute-force baseline "BFT"): Eq. BF itself
 * with the exact K_s on the square window [-r, r]^2 and the exact K_r (either
 * kind), summed in FP32 over in-image neighbours -- the true bilateral
 * filter rather than its N-term expansion, and no workspace.  radius <= 32.
 * DIRECT always filters this way; DIRECT_AUTO does so where its estimated
 * cost, 8.5 (2r + 1)^2 vector operations per pixel, is below the expansion's,
 * (1700 + n_images (85 + 10 quadruplets)) (1 + r / 120) (both fitted to
 * MI355X timings): small windows, and mid-size ones with many range terms.
 * bf_plan_info_t.direct says which. */
#define BF_FLAG_DIRECT 0x2u
#define BF_FLAG_DIRECT_AUTO 0x4u
/* The paper's own regime for 8-bit input (Eq. trigonometric_N_terms with its
 * range box, Eqs. 1D_box_N_terms / numerator_2D_box_N_terms): the range
 * series lies on [-T_r, T_r] (T = T_r; span is ignored) and a source pixel q
 * counts for output p only when |Z(p) - Z(q)| <= 255 T_r in levels.  Few
 * range terms then suffice whatever sigma_r (five give a kernel error of
 * 3.8e-3 at sigma_r = 0.1).  The cube sums over the promoted intensity axis
 * are taken as rectangle sums of the level-window slab per output level (the
 * sliding z window), with the range terms folded into one weight per level
 * difference: one kernel, no workspace, two tables of (32 + 2r + 1)^2 per
 * distinct level of each 32 x 32 output tile, whatever the number of terms.
 * BF_IN_U8 only (BF_ERR_UNSUPPORTED otherwise), radius <= 48, not with the
 * DIRECT flags (BF_ERR_INVALID_ARG); no pre-computed tables, no autotuning.
 * bf_plan_info_t.range_box and .box_levels (floor(255 T_r), at most 255)
 * describe it. */
#define BF_FLAG_RANGE_BOX 0x8u
/* 8-bit input in the default regime (T = max(T_r, span), no range box), with
 * the range terms folded per output level: for an output of level L every
 * source contributes K_s W(L - Z(q)) with W(d) = sum_k a_k cos(omega_k d/255),
 * which is the same filter as the term-by-term expansion (Eq. 1D_N_terms;
 * only the order of the sums over k and over the boxes changes), computed by
 * the range-box kernel with its level window open to every difference.  Cost
 * independent of N_r, proportional to the distinct levels per output tile:
 * faster than the term tables where N_r is large.  BF_IN_U8 only
 * (BF_ERR_UNSUPPORTED otherwise), radius <= 48, not with DIRECT, RANGE_BOX or
 * REDUCED (BF_ERR_INVALID_ARG).  bf_plan_info_t.level_fold says so. */
#define BF_FLAG_LEVEL_FOLD 0x10u

typedef struct {
  bf_dtype_t in_dtype;      /* input element type, default BF_IN_F32 */
  bf_precision_t precision; /* default BF_PREC_PLAIN */
  double eps;               /* kernel truncation level (Sec. IV-A); 0 -> 0.01 */
  double span;              /* intensity span D; range series on [-T, T], T = max(T_r, D); 0 -> 1 */
  int tile;                 /* output tile edge of the summed-area tables (multiple of 64);
                               0 -> chosen per image (see bf_image_geometry) */
  unsigned flags;           /* BF_FLAG_* */
} bf_plan_opts_t;

/* Create a plan: FP64 host fit of both expansions (Sec. IV, App. B), tap
 * compilation, and upload of the tables to the current HIP device.
 *   sigma_s, sigma_r > 0 and finite (sigma_r in intensity units of [0, span]);
 *   radius >= 0 (0 -> ceil(K_s^{-1}(eps)), e.g. ceil(sigma_s sqrt(2 ln(1/eps)))
 *     for the Gaussian);
 *   opts may be NULL (all defaults).
 * Errors: BF_ERR_INVALID_ARG for a NULL plan pointer or out-of-range
 * parameter, BF_ERR_UNSUPPORTED for another kernel kind (or an EXPONENTIAL
 * K_s with radius > 511), BF_ERR_OUT_OF_MEMORY,
 * BF_ERR_DEVICE.  The plan owns its device tables until bf_plan_destroy. */
bf_status_t bf_plan_create(bf_plan_t *plan, bf_kernel_t K_s, bf_kernel_t K_r, double sigma_s,
                           double sigma_r, int radius, bf_terms_t N, const bf_plan_opts_t *opts);

/* Create a plan of two tabulated kernels (arbitrary kernels: Secs. I, IV-B
 * and VI; the expansions and every kernel of the path are unchanged, only
 * the coefficients come from the tables).  Host arrays, read during the
 * call only (the caller keeps ownership):
 *   K_s[(2 radius + 1)^2], row-major, K_s[(dy + radius)(2 radius + 1) + dx +
 *     radius] = weight of offset (dy, dx); radius in [1, 511].  The kernel is
 *     taken as constant on the unit square around each offset, so its Haar
 *     coefficients are exact sums over the finest Haar cells.  Weights must be
 *     finite and >= 0, the centre > 0, and the table even in dy and in dx
 *     (bitwise equal mirrored entries).
 *   K_r[n_r], n_r in [2, 16385]: K_r(i step_r), i = 0 .. n_r - 1, for
 *     differences t >= 0 in the plan's intensity units ([0, 1] for uint8
 *     input, where one level is 1/255); linear between samples, even in t,
 *     zero past T_r = (n_r - 1) step_r.  Samples finite and >= 0, K_r(0) > 0.
 *     The cosine coefficients are the exact integrals of the linear pieces.
 *     The series lies on [-T, T], T = max(T_r, span) (RANGE_BOX: T = T_r).
 * eps is not used (the tables fix both supports).  Every option and flag of
 * bf_plan_create applies except DIRECT (BF_ERR_UNSUPPORTED: direct
 * summation evaluates the analytic kernels only); DIRECT_AUTO never chooses
 * it.  Errors as bf_plan_create; BF_ERR_INVALID_ARG for a NULL table or a
 * table that breaks the rules above. */
bf_status_t bf_plan_create_tabulated(bf_plan_t *plan, const double *K_s, int radius, const double *K_r,
                                     int n_r, double step_r, bf_terms_t N, const bf_plan_opts_t *opts);

/* Release a plan and everything it owns (waits for nothing; the caller must
 * not destroy a plan while work that uses it is in flight).  NULL is a no-op. */
bf_status_t bf_plan_destroy(bf_plan_t plan);

/* Bytes of device workspace bf_filter_ws needs for an H x W image. */
bf_status_t bf_workspace_size(bf_plan_t plan, int H, int W, size_t *bytes);

/* Filter one image: out[H*W] (float32, same units as float input, [0, 1] for
 * uint8 input) from I[H*W] (type fixed by the plan).  I and out are device
 * pointers and must not overlap.  Uses one workspace owned by the plan, grown
 * on demand: the first call at a larger size waits for the device to finish
 * what it has queued, frees the old workspace and allocates a new one (not
 * under graph capture; use bf_filter_ws there).  Calls on one plan share that
 * workspace, so they must be ordered on one stream (or by the caller). */
bf_status_t bf_filter(bf_plan_t plan, const void *I, float *out, int H, int W, void *stream);

/* As bf_filter with a caller-owned device workspace of ws_bytes >=
 * bf_workspace_size(plan, H, W), which must not overlap I or out.  Allocates
 * nothing.  Calls that share a workspace must be ordered on one stream. */
bf_status_t bf_filter_ws(bf_plan_t plan, const void *I, float *out, int H, int W, void *ws,
                         size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): as
 * bf_filter_ws, with the workspace taken from a device array of
 * BF_NOALLOC_SCRATCH_BYTES (256 MiB) that the library holds on each GPU from
 * its first use until the process ends.  Allocates nothing: no hipMalloc, no
 * hipFree.  BF_ERR_INVALID_ARG, with nothing enqueued, when
 * bf_workspace_size(plan, H, W) exceeds BF_NOALLOC_SCRATCH_BYTES.  Every call
 * on one GPU uses that GPU's one array, which keeps the last call's tables:
 * calls that overlap on one GPU (other streams, or other host threads without
 * ordering) race, so order them on one stream.  The result is bitwise the
 * one bf_filter_ws gives. */
#define BF_NOALLOC_SCRATCH_BYTES (256ull << 20)
bf_status_t bf_filter_noalloc(bf_plan_t plan, const void *I, float *out, int H, int W, void *stream);

/* As bf_filter_ws, also writing the numerator and denominator of Eq. BF
 * (device float32 arrays of H*W; either may be NULL).  For validation. */
bf_status_t bf_filter_parts(bf_plan_t plan, const void *I, float *out, float *num, float *den,
                            int H, int W, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes for a batch (host arrays H[n], W[n]). */
bf_status_t bf_batch_workspace_size(const bf_plan_t *plans, int n, const int *H, const int *W,
                                    size_t *bytes);

/* Filter n images of possibly different sizes and plans.  plans, I, out, H, W
 * are HOST arrays of n entries (I[i], out[i] are device pointers); ws is a
 * device workspace of >= bf_batch_workspace_size bytes.  No output may
 * overlap another output, any input or the workspace.  If any entry is
 * invalid the whole batch is rejected before anything is enqueued.  Output i
 * is bitwise identical to bf_filter_ws(plans[i], I[i], out[i], H[i], W[i]). */
bf_status_t bf_filter_batch(const bf_plan_t *plans, int n, const void *const *I, float *const *out,
                            const int *H, const int *W, void *ws, size_t ws_bytes, void *stream);

/* Batch launch form, process-wide (default 0).  0: a batch group of one input
 * type is one table-kernel launch followed by persistent lookup launches, one
 * per lookup kernel class.  1: where every image of a group is looked up by
 * the LDS tile kernel (double-buffered, or with regions up to 164 rows at
 * pitch 176), with at most 8 quadruplets and table rows of at most 1024
 * columns, the group is ONE persistent launch (after a small counter-reset
 * launch) that builds the tables and looks them up, an output tile starting
 * as soon as the tables of its table tile are published (per-tile ready
 * counters, release/acquire at device scope); other groups as with 0.
 * Results are bitwise the same either way (Secs. III-IV).  The batch's first
 * 40 workspace bytes are its queues, counters and error word.  Returns
 * BF_ERR_INVALID_ARG for values other than 0 and 1. */
bf_status_t bf_batch_set_fused(int fused);

/* Plan introspection (host side; valid for BF_FLAG_HOST_ONLY plans too). */
typedef struct {
  int radius;         /* window radius r */
  int n_range;        /* cosine terms kept */
  int n_spatial;      /* Haar level groups kept */
  int n_taps;         /* nonzero summed-area-table taps of the spatial expansion */
  int n_tap_rows;     /* distinct tap row offsets */
  int n_tap_cols;     /* distinct tap column offsets */
  int n_images;       /* term images per filter call: 4 n_range - 3 */
  int tile;           /* fixed output tile edge, 0 when chosen per image */
  int sat_shift;      /* q (term values stored as round(v 2^q)); -1: chosen per image */
  double T_s;         /* spatial truncation r + 1/2 */
  double T_r;         /* K_r^{-1}(eps) */
  double T;           /* range series half-interval max(T_r, span) */
  double den_floor;   /* out = I where den <= den_floor (1e-7 sum |K~_s|) */
  int n_quads;        /* taps grouped in symmetric quadruplets (one box sum each) */
  int n_single;       /* taps outside any quadruplet: always 0 (plans whose taps do not all pair
                         into quadruplets are refused with BF_ERR_UNSUPPORTED) */
  int lookup_kernel;  /* 1: LDS tile lookup kernel, 0: per-pixel lookup kernel */
  int direct;         /* 1: filters by direct summation (BF_FLAG_DIRECT / _AUTO) */
  int range_box;      /* 1: the 8-bit range-box regime (BF_FLAG_RANGE_BOX) */
  int box_levels;     /* its level window half-width floor(255 T_r); -1 otherwise */
  int box_tile;       /* its output tile edge (64, or 32 where a 64 tile's region exceeds LDS) */
  int reduced;        /* 1: BF_PREC_REDUCED (FP16 term images, tables built in LDS) */
  int level_fold;     /* 1: BF_FLAG_LEVEL_FOLD (8-bit, range terms folded per output level) */
  int lds_pitch;      /* LDS tile lookup kernel: row pitch (int32) of its staged table region
                         (128, 160, 176 or 192); 0 when the per-pixel kernel is used */
  int lds_double_buffered; /* 1: two staged regions fit in LDS (pitch 128) */
  int lattice;        /* 1: the lattice lookup kernel applies (quadruplet rows on a lattice of step
                         lattice_step <= 16, at most 4 rows and 4 columns of boxes) */
  int lattice_step;
  int default_lookup; /* lookup kernel of an untuned image: 0 per-pixel, 1 LDS tile double-buffered,
                         2 LDS tile single-buffered or overlap-staged, 3 lattice (where the LDS tile
                         kernel is not double-buffered and the plan has more than 8 quadruplets, or
                         where the LDS tile kernel does not apply) */
} bf_plan_info_t;

bf_status_t bf_plan_query(bf_plan_t plan, bf_plan_info_t *info);

/* Tiling of an H x W image under a plan: the table tile edge, the shift q
 * and the workspace bytes.  Term values are stored as round(v 2^q) in int32
 * tables summed with wrapping 32-bit adds; the kernels use only box
 * differences of a table, exact modulo 2^32, so q is the largest shift with
 * (2r + 1)^2 (gmax 2^q + 1) <= 2^31 - 1 (at most 24) and does not depend on
 * the tile (the FP32 rounding of the quantised products is allowed for by a
 * factor 1 + 2^-20 on gmax).  Any pointer may be NULL. */
bf_status_t bf_image_geometry(bf_plan_t plan, int H, int W, int *tile, int *sat_shift,
                              size_t *ws_bytes);

/* The lookup kernel an H x W image runs under a plan, as bf_filter would
 * launch it now (after bf_autotune or bf_tuning_set, the tuned one):
 * *kind = 0 per-pixel, 1 LDS tile double-buffered, 2 LDS tile single-buffered
 * or overlap-staged, 3 lattice; -1 for plans that keep no tables (direct
 * summation, range-box and level-fold regimes, reduced precision).  All
 * lookup kernels give the same bits.  BF_ERR_INVALID_ARG for a null plan or
 * kind, or sizes outside [1, 32768]. */
bf_status_t bf_image_lookup_kernel(bf_plan_t plan, int H, int W, int *kind);

/* Range terms: k[i], a[i] (coefficient a_k) and omega[i] = pi k / T, i < n_range. */
bf_status_t bf_plan_range_terms(bf_plan_t plan, int *k, double *a, double *omega, int capacity);

/* Sampled spatial expansion K~_s(dy, dx) for dy, dx in [-r, r]:
 * K[(dy + r)(2r + 1) + dx + r], capacity >= (2r + 1)^2. */
bf_status_t bf_plan_spatial_kernel(bf_plan_t plan, double *K, int capacity);

/* Summed-area-table taps: corr(p) = sum_i w[i] S(p_y + dy[i], p_x + dx[i])
 * with S the exclusive table S(Y, X) = sum_{y < Y, x < X} g(y, x), indices
 * clamped to [0, H] x [0, W]. */
bf_status_t bf_plan_taps(bf_plan_t plan, int *dy, int *dx, double *w, int capacity);

/* Selected Haar level groups as (level_x, level_y) pairs, level -1 = phi. */
bf_status_t bf_plan_spatial_groups(bf_plan_t plan, int *level_x, int *level_y, int capacity);

/* Autotuner.  Times the candidate launch shapes for H x W images under this
 * plan -- table tiles of 64, 128, 256 and 512, and for a plan the lattice
 * kernel applies to, the multiples of 64 up to 576 that hold whole lattice
 * tiles (tile + 2r + 1 <= 1024), each
 * with one range term, one table or one cosine or sine pair of tables per
 * table-kernel wave, and with every
 * lookup kernel the plan can use (LDS tile double- or single-buffered,
 * lattice; all give the same bits) --
 * on a temporary mid-grey image (reps launches each, at least
 * 3) and keeps the fastest (among shapes within 1% of it, the one with the
 * smallest workspace), process-wide, for the plan's shape class (the
 * radius, term and quadruplet counts, input type) and images in the same
 * 256-pixel size bucket of H and W.  From then on every call path (bf_filter,
 * bf_filter_ws, bf_filter_batch, bf_workspace_size, the request loop) uses
 * it, so the workspace size of those images may change: size workspaces
 * after tuning.  Results do not change: only plans whose taps all belong to
 * quadruplets are tuned, and their outputs do not depend on the tiling.
 * Other plans (a tile fixed in the options) are left as they are.  Allocates and frees device memory and synchronises `stream`; not for
 * use under graph capture.  *tile (may be NULL) receives the chosen tile. */
bf_status_t bf_autotune(bf_plan_t plan, int H, int W, int reps, void *stream, int *tile);
/* Set the launch shape for this plan's shape class and H x W's size bucket
 * by hand, as bf_autotune would: table tile (a multiple of 64 with
 * tile + 2r + 1 <= 1024), kb_single (the lookup kernel: 0 the default
 * choice, 1 the LDS tile kernel single-buffered, 2 the lattice kernel; a
 * kernel the plan cannot use falls back to the default), ka_one (table-kernel
 * waves: 0 one range term each, 1 one table, 2 the cosine pair C I, C or the
 * sine pair S I, S of a term; BF_ERR_INVALID_ARG otherwise).  BF_ERR_UNSUPPORTED for plans
 * that are not tuned (a fixed tile, direct, range-box or reduced plans). */
bf_status_t bf_tuning_set(bf_plan_t plan, int H, int W, int tile, int kb_single, int ka_one);
/* Forget every tuned shape. */
bf_status_t bf_autotune_clear(void);

/* ------------------------------------------------------------------------
 * Pre-computed tables (Case 1 of Sec. V-C).  The term tables of an image
 * depend on the image, the range terms k and T only (not on the spatial
 * kernel or on sigma_r while T = max(T_r, span) stays the same), so tables
 * built once under `tables_plan` serve later filters of the same image under
 * any `plan` that is compatible: same input type, radius <= tables_plan's,
 * and range terms equal to the first terms of tables_plan's
 * (same k, same T).  Only the lookup kernel runs.  The result equals
 * bf_filter(plan) up to the fixed-point shift, which here is tables_plan's
 * (within 1e-6 of it; not bitwise).
 * ------------------------------------------------------------------------ */
/* Workspace bytes of the tables of an H x W image under tables_plan. */
bf_status_t bf_precompute_size(bf_plan_t tables_plan, int H, int W, size_t *bytes);
/* Build the tables (table kernel only) into ws (>= bf_precompute_size). */
bf_status_t bf_precompute(bf_plan_t tables_plan, const void *I, int H, int W, void *ws, size_t ws_bytes,
                          void *stream);
/* BF_OK if tables built under tables_plan serve plan; else BF_ERR_INVALID_ARG
 * (BF_ERR_UNSUPPORTED for direct, range-box or reduced plans). Host only. */
bf_status_t bf_precomputed_compatible(bf_plan_t tables_plan, bf_plan_t plan);
/* Filter I (the image the tables were built from) under plan, reading the
 * tables in ws; lookup kernel only. */
bf_status_t bf_filter_precomputed(bf_plan_t tables_plan, bf_plan_t plan, const void *I, float *out, int H,
                                  int W, const void *ws, size_t ws_bytes, void *stream);

/* Per-kernel timing for measurement.  While enabled, every filter call
 * records HIP events around each of its kernels on the call's stream (all
 * work still runs); bf_profile_read waits for the recorded events, returns
 * the summed milliseconds and launch counts per kernel (index 0: summed-area
 * tables, 1: tap lookup and normalisation) and clears them.  Process-wide,
 * not thread-safe; for benchmarks. */
bf_status_t bf_profile_enable(int on);
bf_status_t bf_profile_read(double ms[2], int launches[2]);

/* ------------------------------------------------------------------------
 * Serving: a request loop over bf_filter_batch.
 *
 * Requests (plan, device image, device output) are queued in arrival order.
 * Whenever a stream is free, the longest prefix of the queue whose batch
 * workspace fits in the largest free block of the server's workspace arena
 * (and has at most max_batch requests) is launched as one batch on that
 * stream; up to n_streams batches run at once, so requests that arrive while
 * others are on the GPU are admitted as streams and memory free up and
 * their work overlaps on the device.  The queue head is never overtaken
 * (no starvation); a request whose workspace cannot fit the whole arena is
 * completed with BF_ERR_OUT_OF_MEMORY.  Each result is bitwise the one a
 * single bf_filter call produces (bf_filter_batch contract).
 *
 * The server owns its arena (one device allocation of hbm_budget bytes at
 * create) and its streams; the caller owns plans, images and outputs and
 * keeps them alive until the request completes.  The server's streams do not
 * wait for any other stream: a request's input must hold its final values,
 * and no queued work may still write its output, when it is submitted (the
 * caller synchronises the streams that produced them first).  Completions are found by
 * bf_server_poll, which never blocks; `now` is the caller's clock, recorded
 * as the completion time.  Not thread-safe: one thread drives a server.
 *
 * BF_SERVER_DRY_RUN does no device work at all (no arena, no streams, no
 * launches; plans may be host-only and pointers are not dereferenced): a
 * batch completes when `now` passes its simulated end, launch time plus its
 * pixel count / dry_rate.  It exercises the same queue, admission and
 * arena logic, for tests without a GPU.
 * ------------------------------------------------------------------------ */
typedef struct bf_server_s *bf_server_t;

#define BF_SERVER_DRY_RUN 1u

typedef struct {
  size_t hbm_budget; /* workspace arena bytes; 0 -> 16 GiB */
  int max_batch;     /* requests per batch; 0 -> 32 */
  int n_streams;     /* batches in flight at once; 0 -> 2 (at most 8) */
  unsigned flags;    /* BF_SERVER_DRY_RUN */
  double dry_rate;   /* dry run: pixels per second of one batch; 0 -> 1e9 */
} bf_server_opts_t;

typedef struct {
  unsigned long long tag; /* the caller's request tag */
  bf_status_t status;     /* BF_OK or the error of its batch */
  int batch;              /* sequence number of the batch it ran in (-1: none) */
  int batch_size;         /* requests in that batch */
  double t_launch;        /* `now` when its batch was launched */
  double t_done;          /* `now` of the poll that found it complete */
} bf_completion_t;

typedef struct {
  long long submitted, completed, batches;
  int peak_batches_in_flight;
  int peak_requests_in_flight;
  size_t peak_arena_bytes; /* high-water mark of arena bytes held by batches */
  size_t arena_bytes;      /* arena size */
  long long batch_size_hist[65]; /* batches of size b (b >= 64 counted at 64) */
} bf_server_stats_t;

bf_status_t bf_server_create(bf_server_t *server, const bf_server_opts_t *opts);
/* Waits for the batches in flight, then frees the arena and the streams. */
bf_status_t bf_server_destroy(bf_server_t server);
/* Queue one request; validated now (plan, sizes, pointers, its input and
 * output not overlapping).  Requests whose buffers overlap each other are
 * completed with BF_ERR_INVALID_ARG together with their batch. */
bf_status_t bf_server_submit(bf_server_t server, bf_plan_t plan, const void *I, float *out, int H,
                             int W, unsigned long long tag, double now);
/* Retire finished batches, launch new ones, and return up to `capacity`
 * completions (the rest are returned by later polls). */
bf_status_t bf_server_poll(bf_server_t server, double now, bf_completion_t *done, int capacity,
                           int *n_done);
/* Requests queued but not launched, and requests in flight. */
bf_status_t bf_server_pending(bf_server_t server, int *queued, int *in_flight);
bf_status_t bf_server_stats(bf_server_t server, bf_server_stats_t *stats);

const char *bf_status_string(bf_status_t s);

/* Library version string. */
const char *bf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BF_H */
