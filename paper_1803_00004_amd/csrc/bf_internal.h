// Internal structures shared by the host plan, the C ABI and the HIP kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "bf.h"

namespace bf {

// Compile-time capacities of the device tables.
constexpr int kMaxTerms = 64;      // cosine terms per plan
constexpr int kMaxTapAxis = 16;    // distinct tap offsets per axis (Haar levels <= 3)
constexpr int kMaxTaps = 256;      // nonzero summed-area-table taps
constexpr int kMaxQuads = kMaxTaps / 4;  // symmetric tap quadruplets
constexpr int kMaxImages = 4 * kMaxTerms;  // term images (tables) per filter call
constexpr int kMaxChunks = 8;      // 256-column chunks of one table row (table width <= 2048)
constexpr int kKA_Threads = 256;   // summed-area-table kernel block size (upper bound)
constexpr int kMaxBatch = 24;      // images per batched launch (descriptors travel as kernel arguments)
constexpr int kLatClasses = 12;            // lattice lookup kernel classes (pitch, rows, columns)
constexpr int kBatchQueues = 8 * (2 + kLatClasses);  // K-B work queues of a batch: 8 per lookup class
constexpr size_t kBatchHeadBytes = 1024;   // batch workspace prefix: the K-B work-queue heads
constexpr int kMaxDirectRadius = 32;     // direct summation window limit
constexpr int kMaxCellFitRadius = 511;   // non-separable K_s: Haar levels <= 8 (cell integrals)

// Host-side result of the FP64 fit (Sec. IV, App. A/B).
struct Fit {
  int radius = 0;
  double T_s = 0, T_r = 0, T = 0, eps = 0.01, span = 1.0;
  // spatial
  std::vector<int> group_lx, group_ly;  // selected Haar level groups (-1 = phi)
  std::vector<double> K;                // (2r+1)^2 sampled expansion, K[(dy+r)(2r+1) + dx+r]
  // taps of the exclusive summed-area table: corr(p) = sum w S(p + (dy, dx))
  std::vector<int> tap_dy, tap_dx;
  std::vector<double> tap_w;
  std::vector<int> row_off, col_off;   // distinct tap offsets per axis (sorted)
  std::vector<double> tap_grid;        // [row_off.size()][col_off.size()] weights (0 = no tap)
  double sum_abs_K = 0;
  // range
  std::vector<int> k;
  std::vector<double> a, omega;
};

// The two kernels of a plan: analytic kinds (bf_kernel_t) with their sigmas,
// or tables.  A spatial table holds (2r + 1)^2 weights, ks[(dy + r)(2r + 1) +
// dx + r], taken as constant on the unit square around each integer offset; a
// range table holds kr_n samples K_r(i kr_step), taken as linear between
// samples and zero past the last.
struct KernelSpec {
  int kind_s = BF_KERNEL_GAUSSIAN, kind_r = BF_KERNEL_GAUSSIAN;
  double sigma_s = 0, sigma_r = 0;
  const double *ks = nullptr;  // tabulated K_s, or null
  const double *kr = nullptr;  // tabulated K_r, or null
  int kr_n = 0;
  double kr_step = 0;
};
constexpr int kMaxRangeSamples = 16385;

// Fit both expansions; returns BF_OK, BF_ERR_INVALID_ARG or BF_ERR_UNSUPPORTED.
bf_status_t fit_plan(const KernelSpec &kern, int radius, bf_terms_t N, double eps, double span, Fit *out);

// Device-side constant tables of a plan (one upload per plan).  Everything
// the kernels read is integer or FP32: the FP64 fit stays on the host.
struct DevTables {
  int n_terms;
  int tap_dy_min, tap_dy_max, tap_dx_min, tap_dx_max;  // extent of the summed-area-table taps
  // The taps of a symmetric kernel come in quadruplets (dy, dx), (1-dy, dx),
  // (dy, 1-dx), (1-dy, 1-dx) with weights w, -w, -w, w: one box sum of the
  // table, differenced exactly in int32, times w.  Each quadruplet is stored
  // as its representative (dy >= 1, dx >= 1).
  int lds_pitch;                       // staged region row pitch; 0: no LDS tile kernel
  // Row lattice of the quadruplets for the lattice lookup kernel (lat = 1):
  // their dy take lat_m values dy_j = lat_dy0 + j lat_s (j < lat_m, lat_s <=
  // 16; values between the plan's rows may carry no quadruplet), their dx the
  // lat_n values lat_dx[i] (padded by repeating the last); the quadruplet
  // (dy_j, lat_dx[i]) has weight lat_w[4 j + i] when bit 4 j + i of lat_mask
  // is set.  lat_g lattice groups of lat_s waves compute; lat_pitch is the
  // staged band's row pitch.
  int lat, lat_s, lat_m, lat_n, lat_g, lat_pitch, lat_dy0, lat_mask;
  int lat_dx[4];
  float lat_w[16];
  int n_quads;
  int quad_dy[kMaxQuads], quad_dx[kMaxQuads];
  float quad_w[kMaxQuads];
  float f_hi[kMaxTerms], f_lo[kMaxTerms];  // f_k = k / (2T) (u8: k / (2T 255)) as two floats
  float a[kMaxTerms];                  // a_k
  int k_is_zero[kMaxTerms];            // term k = 0: one image (I), analytic denominator
  int slot[kMaxTerms];                 // first table of the term
  // table -> (term, part); part 0: C*I, 1: S*I, 2: C, 3: S, 4: I (k = 0)
  int slot_term[kMaxImages], slot_part[kMaxImages];
  // the slot's term values again, indexed by slot, so that a lookup kernel
  // fetches them without first fetching the slot's term
  float slot_fhi[kMaxImages], slot_flo[kMaxImages];
  float slot_a[kMaxImages];
  float gmax;                          // bound of |term value| for [0, span] input
  float den_floor;
  int in_u8;
  int n_images;
  // direct summation (true BF over the (2r+1)^2 window)
  int direct;
  int direct_r;
  int direct_abs;                      // range kernel in |d| (exponential) instead of d^2
  float direct_c;                      // K_r(d) = 2^(c d^2), or 2^(c |d|) when direct_abs
  const float *direct_ks;              // device: K_s(dy, dx) at (dy + r)(2r + 1) + dx + r
                                       // (direct_r also holds the radius of range-box plans)
  // range-box regime for 8-bit input (T = T_r, Eq. 1D_box_N_terms)
  int range_box;
  int box_zr;                          // level window half-width floor(255 T_r), <= 255
  float box_scale;                     // 2^q of the slab tables
  float box_w[511];                    // W(d) = sum_k a_k cos(omega_k d / 255) [|d| <= zr] at d + 255
  int reduced;                         // FP16 term images, tables built in LDS (BF_PREC_REDUCED)
  int level_fold;                      // range_box kernel with the window open (BF_FLAG_LEVEL_FOLD)
};

// Geometry of one image under a plan: tiles of `tile` outputs with their
// tile-relative summed-area tables of E_h x E_w (pitch P_w) int32 entries.
struct Geometry {
  int H, W, tile, radius;
  int sat_shift;                    // q: term values stored as round(v * 2^q)
  int tiles_y, tiles_x, n_images;
  int E_max, pitch;                 // max table edge (tile + 2r + 1) and padded row pitch
  size_t table_elems;               // E_max * pitch per table
  size_t ready_off;                 // bytes of the tables; the fused batch's ready counters follow
  size_t bytes;                     // whole workspace
  int kb_single = 0;                // lookup kernel: 0 the default choice, 1 the LDS tile kernel
                                    // single-buffered, 2 the lattice kernel (lookup_kernel_for)
  int ka_one = 0;                   // table-kernel waves: 0 one range term each, 1 one table,
                                    // 2 a cosine or sine pair of tables
};

Geometry make_geometry(int H, int W, int tile, int radius, int n_images, int sat_shift);

// Table tile and fixed-point shift for one image: `fixed_tile` if nonzero,
// else the largest of 512, 256, 128, 64 that gives >= 2048 term waves with a
// table row of <= 768 columns (the smallest such tile otherwise); with
// row_unit > 0 (the output rows of a lattice-kernel tile) the candidates are
// the multiples of both 64 and row_unit up to 576 instead, where there are any.  Term values
// are stored as round(v * 2^q) in int32 and tables are summed with wrapping
// 32-bit adds.  Every tap belongs to a symmetric quadruplet, so the kernels
// only ever use box differences, which are exact modulo 2^32 whenever the box
// fits in int32: q is the largest shift (<= 24) with
// (2r + 1)^2 (gmax 2^q (1 + 2^-20) + 1) <= 2^31 - 1 (the factor covers the
// FP32 rounding of the products that are quantised), independent of the tile.
// A pure function of its arguments, so every call path tiles an image alike.
void choose_tiling(int H, int W, int radius, int n_terms, int fixed_tile, double gmax, int row_unit, int *tile,
                   int *sat_shift);

// Row pitch (int32 elements) of the LDS tile kernel's staged table region for
// a region `width` columns wide: one of the compiled pitches, or 0 if none fits.
int lds_pitch_for(int width);

// The range-box regime (host.range_box) of an 8-bit image: one launch, no
// workspace; BF_ERR_UNSUPPORTED when its staged region exceeds LDS.
bf_status_t launch_rangebox(const DevTables *dev, const DevTables &host, const void *I, float *out, float *num,
                            float *den, int H, int W, void *stream);
size_t rangebox_lds_bytes(const DevTables &host);
int rangebox_tile(const DevTables &host);  // output tile edge of the range-box kernel (0: does not fit)
constexpr int kMaxRangeBoxRadius = 48;

// Reduced precision (host.reduced): FP16 term images in ws ([table][H][W]),
// then the lookup kernel with tables built in LDS.  Output tile edge 64 or 32
// (0: the region does not fit); workspace bytes for an H x W image.
bf_status_t launch_reduced(const DevTables *dev, const DevTables &host, const Geometry &g, const void *I,
                           float *out, float *num, float *den, void *ws, void *stream);
int reduced_tile(const DevTables &host);
size_t reduced_workspace_bytes(const DevTables &host, int H, int W);

// Direct summation of Eq. BF for a plan with host.direct set.
bf_status_t launch_direct(const DevTables &host, const void *I, float *out, float *num, float *den,
                          int H, int W, void *stream);

// The table kernel alone (tables of `host`'s terms, geometry g) and the
// lookup kernel alone (taps and terms of `host`, reading tables laid out by
// geometry g, which may hold more tables than `host` reads).
bf_status_t launch_tables(const DevTables *dev, const DevTables &host, const Geometry &g,
                          const void *I, int32_t *ws, void *stream);
bf_status_t launch_lookup(const DevTables *dev, const DevTables &host, const Geometry &g,
                          const void *I, float *out, float *num, float *den, const int32_t *ws,
                          void *stream);

// Launch the two kernels of one image on `stream` (hipStream_t): `dev` is
// the device copy of `host`.
bf_status_t launch_filter(const DevTables *dev, const DevTables &host, const Geometry &g,
                          const void *I, float *out, float *num, float *den, int32_t *ws,
                          void *stream);

// One image of a batch: its plan tables (device and host copies), geometry,
// buffers and its own region of the batch workspace.
struct BatchItem {
  const DevTables *dev;
  const DevTables *host;
  Geometry g;
  const void *I;
  float *out;
  int32_t *ws;
};

// Launch a batch on `stream`: per group of at most kMaxBatch images of one
// input type one K-A launch and one K-B launch per lookup class (or one fused
// launch, bf_batch_set_fused); table-free requests (direct summation,
// range-box regime) and reduced-precision requests share launches per kind.
// `heads` is kBatchHeadBytes of device memory for the work queues.
bf_status_t launch_batch(const BatchItem *items, int n, uint32_t *heads, void *stream);
// bf_batch_set_fused: 1 runs eligible batch groups as one fused launch
void set_fused_batch(int on);

// Which lookup kernel a plan's images use: 1 the LDS tile kernel, 0 the
// per-pixel kernel.
int lookup_kernel_kind(const DevTables &h);
// The lookup kernel an image runs: 0 per-pixel, 1 LDS tile double-buffered,
// 2 LDS tile single-buffered, 3 lattice (Geometry.kb_single selects among
// the eligible ones; 0 there: the double-buffered LDS tile kernel where it
// applies, else the lattice kernel for plans of more than 8 quadruplets where
// it applies, else the LDS tile kernel, else the lattice kernel).
int lookup_kernel_for(const DevTables &h, int kb_single);
// output rows of one lattice-kernel tile (s U G)
int lattice_rows(const DevTables &h);
bool lattice_eligible(const DevTables &h);
size_t lattice_lds_bytes(const DevTables &h);
bool kb_tile_eligible(const DevTables &h);
bool kb_double_buffered(const DevTables &h);  // two staged regions fit in LDS
bool kb_overlap_staged(const DevTables &h, int pitch);  // overlap staging applies at this pitch

// Device workspace of bf_filter_noalloc: kScratchBytes of a static device
// array, resolved once per device (the current one); BF_ERR_DEVICE if the
// symbol cannot be resolved.
constexpr size_t kScratchBytes = size_t(BF_NOALLOC_SCRATCH_BYTES);
bf_status_t scratch_workspace(void **ptr);

// Optional per-kernel event recording (bf_profile_enable); kernel 0 / 1.
void profile_mark(int kernel, int begin, void *stream);

}  // namespace bf

struct bf_plan_s {
  bf::Fit fit;
  bf_dtype_t in_dtype = BF_IN_F32;
  bf_precision_t precision = BF_PREC_PLAIN;
  int tile = 0;        // fixed table tile, 0 = chosen per image
  double gmax = 1.0;
  unsigned flags = 0;
  bf::DevTables host_tables{};
  bf::DevTables *dev_tables = nullptr;  // device copy
  float *dev_direct_ks = nullptr;       // device K_s window of a direct plan
  void *own_ws = nullptr;               // workspace grown by bf_filter
  size_t own_ws_bytes = 0;
  int device = 0;
};
