// gfx950 kernels of the N-term bilateral filter.
//
// K-A (ka_sat / ka_body): for one table tile and one range term k, modulate
//   the image (C = cos(omega_k I), S = sin(omega_k I); term values C*I, S*I,
//   C, S, or I alone for k = 0 -- the shift identity of Eq. 1D_N_terms) and
//   build the summed-area table of each term image over the tile plus an
//   r-pixel halo (recurrences of Eq. sum_sat_recurrence_2D: prefix along the
//   row, then accumulation down the columns).  Values are stored as
//   round(v * 2^q) in int32 (the k = 0 image of 8-bit input as the byte
//   itself) and summed with wrapping 32-bit adds, so every box difference is
//   exact; q is chosen so that no box of the window can overflow.
// K-B (kb_tile / kb_body, LDS tile form; kb_lookup, per-pixel form): per
//   output pixel, the box sums of the spatial expansion's tap quadruplets
//   (four-reference box sums of Eq. sum_sat_sum_region_2D), accumulated into
//   the numerator and denominator of Eq. BF over the range terms, and the
//   normalisation.
// Batches (ka_batch, kb_batch) run the same per-image bodies over many
//   images in one launch per kernel.
// Other plan kinds, each one launch per image (their own launches in batches):
//   direct_bf    Eq. BF summed directly over the window (the brute-force
//                baseline, for small windows);
//   kz_rangebox  the paper's own 8-bit regime: range series on [-T_r, T_r]
//                with the range box, cube sums over the promoted intensity
//                axis as per-level slab tables built in LDS;
//   kr_modulate, kr_tile  reduced precision: FP16 term images, tables built
//                in LDS per output tile.
//
// Layout in HBM: one workspace of int32 tables, [tile][image][row][pitch],
// each table (tile + 2r + 1) x pitch with pitch a multiple of 64 elements
// (reduced precision: FP16 term images [table][H][W]).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>
#include <atomic>
#include <mutex>
#include <type_traits>
#include <numeric>
#include <vector>

#include "bf_internal.h"

namespace bf {

// Per-launch scalars of one image.
struct ImageParams {
  int H, W, tile, radius, tiles_x, n_images, pitch, n_terms;
  long long table_elems;
  float sat_scale;      // 2^q
  float inv_sat_scale;  // 2^-q
};

// Phase of term k at intensity x in revolutions, reduced to about [-0.5, 0.5]:
// f_k * x with f_k = f_hi + f_lo carried in two floats (error-free product of
// f_hi and x), so the reduced phase is accurate to a few 1e-8.
__device__ __forceinline__ float phase_rev(float f_hi, float f_lo, float x) {
  const float ph = f_hi * x;
  const float e = __builtin_fmaf(f_hi, x, -ph);
  const float pl = __builtin_fmaf(f_lo, x, e);
  const float n = __builtin_rintf(ph);
  return (ph - n) + pl;
}

template <bool U8>
__device__ __forceinline__ void load_pixel(const void *I, long long idx, float *phase_x,
                                           float *val) {
  if (U8) {
    const float b = (float)static_cast<const uint8_t *>(I)[idx];
    *phase_x = b;  // the u8 plan carries f_k / 255
    *val = b * (1.0f / 255.0f);
  } else {
    const float v = static_cast<const float *>(I)[idx];
    *phase_x = v;
    *val = v;
  }
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP moves: partial
// sums within each 16-lane row (row_shr 1, 2, 3, then 4 and 8 on the upper
// banks), then the row totals carried by row_bcast:15 and row_bcast:31.
// Sums wrap modulo 2^32 (unsigned arithmetic).
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
  uint32_t x = v;
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);   // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);   // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x113, 0xf, 0xf, true);   // row_shr:3
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xe, false);  // row_shr:4, lanes 4..15 of a row
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xc, false);  // row_shr:8, lanes 8..15 of a row
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
  return x;
}

// ---------------------------------------------------------------------------
// K-A: tile-relative int32 summed-area tables of one range term per wave
// (the four term images C*I, S*I, C, S share one phase and one sin/cos; the
// k = 0 term has the single image I).  Lane l owns the 4-column groups
// [4l + 256g, 4l + 256g + 4), g < G, so each int4 store of a row writes 1 KB
// of contiguous memory; the row prefix is an in-lane prefix plus one DPP wave
// scan per 256-column chunk; the column accumulation lives in registers and
// the image rows are prefetched kPF rows ahead.  No barriers: waves are
// independent.  Term values are quantised as round(v * 2^q); values outside
// [-gmax, gmax] (inputs outside [0, span]) are not clamped.
// ---------------------------------------------------------------------------
constexpr int kPF = 4;

// ONE = false: a wave builds the 1 or 4 tables of one range term (one sin/cos
// per pixel for all four); ONE = true: a wave builds one table (4x the waves
// for the same tile, so larger tiles keep the chip busy); PAIR: a wave builds
// the cosine pair (C*I, C) or the sine pair (S*I, S) of a term (2x the waves,
// one of sin/cos per pixel each).  All store the same integers.  One wave
// builds unit `unit` (a term, with ONE a table, with PAIR 2 term + pair) of
// table tile tile_id.  DYN: the wave's 8-bit lookup table lives in the
// dynamic LDS (the fused batch kernel), else in a static array of 4 waves.
template <int G, bool U8, bool ONE, bool DYN, bool PAIR = false>
__device__ __forceinline__ void ka_unit(const void *__restrict__ I, const ImageParams &p,
                                        const DevTables *__restrict__ tab, int32_t *__restrict__ ws,
                                        int tile_id, int unit) {
  // the wave index is uniform; saying so keeps per-term loads scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int term = ONE ? tab->slot_term[unit] : PAIR ? unit >> 1 : unit;
  const int part = ONE ? tab->slot_part[unit] : 0;  // ONE: the table's part (4: k = 0)
  const int half = PAIR ? unit & 1 : 0;              // PAIR: 0 the cosine pair, 1 the sine pair
  const int ty = tile_id / p.tiles_x, tx = tile_id - ty * p.tiles_x;
  const int y0 = ty * p.tile, x0 = tx * p.tile;
  const int y1 = min(p.H, y0 + p.tile), x1 = min(p.W, x0 + p.tile);
  const int oy = max(y0 - p.radius, 0), ox = max(x0 - p.radius, 0);
  const int Eh = min(y1 + p.radius, p.H) - oy + 1;
  const int Ew = min(x1 + p.radius, p.W) - ox + 1;
  const bool k0 = tab->k_is_zero[term] != 0;
  if (PAIR && k0 && half) return;  // the k = 0 term's one table is its first wave's
  const int nimg = (k0 || ONE) ? 1 : PAIR ? 2 : 4;
  const float f_hi = tab->f_hi[term], f_lo = tab->f_lo[term];
  const float scale = p.sat_scale;
  int32_t *base = ws + ((long long)tile_id * p.n_images + (ONE ? unit : tab->slot[term] + half)) * p.table_elems;
  // the wave's m-th table (PAIR: parts half and half + 2 of the term)
  const long long te = (PAIR ? 2 : 1) * (long long)p.table_elems;

  // 8-bit input takes 256 values only: each wave tabulates its term's four
  // quantised values per byte value in LDS, with the very expressions of the
  // per-pixel path below (same integers), and looks them up per pixel.
  int4 *lut;
  if constexpr (!DYN) {
    __shared__ int4 lut8_s[4][256];
    lut = lut8_s[wave];
  } else {
    extern __shared__ int4 lut8_d[];
    lut = lut8_d + 256 * wave;
  }
  if (U8 && !k0) {
    for (int b = lane; b < 256; b += 64) {
      const float px = (float)b;
      const float xs = px * (1.0f / 255.0f) * scale;
      const float fr = phase_rev(f_hi, f_lo, px);
      const float C = __builtin_amdgcn_cosf(fr), S = __builtin_amdgcn_sinf(fr);
      lut[b] = make_int4(__float2int_rn(C * xs), __float2int_rn(S * xs), __float2int_rn(C * scale),
                         __float2int_rn(S * scale));
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the wave's table is in LDS before it reads it
  }

  // raw pixel values (u8 as integer-valued float) of the rows i .. i + kPF - 1
  float pf[kPF][G][4];
  auto load_row = [&](int i, float (&dst)[G][4]) {
    const long long row = (long long)(oy + i - 1) * p.W;
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int j = 4 * lane + 256 * g + c;
        float v = 0.0f;
        if (i < Eh && j >= 1 && j < Ew) {
          const long long idx = row + (ox + j - 1);
          v = U8 ? (float)static_cast<const uint8_t *>(I)[idx] : static_cast<const float *>(I)[idx];
        }
        dst[g][c] = v;
      }
  };
#pragma unroll
  for (int q = 0; q < kPF; ++q) load_row(1 + q, pf[q]);

  uint32_t acc[4][G][4];  // column sums, wrapping modulo 2^32
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int g = 0; g < G; ++g) acc[m][g][0] = acc[m][g][1] = acc[m][g][2] = acc[m][g][3] = 0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int j0 = 4 * lane + 256 * g;
    if (j0 < p.pitch)
      for (int m = 0; m < nimg; ++m) *reinterpret_cast<int4 *>(base + m * te + j0) = make_int4(0, 0, 0, 0);
  }

  for (int i = 1; i < Eh; ++i) {
    float cur[G][4];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int c = 0; c < 4; ++c) cur[g][c] = pf[0][g][c];
#pragma unroll
    for (int q = 0; q + 1 < kPF; ++q)
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int c = 0; c < 4; ++c) pf[q][g][c] = pf[q + 1][g][c];
    load_row(i + kPF, pf[kPF - 1]);

    uint32_t carry[4] = {0, 0, 0, 0};
    int32_t *row = base + (long long)i * p.pitch;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      uint32_t v[4][4];  // [image][column]
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float px = cur[g][c];
        const float xs = (U8 ? px * (1.0f / 255.0f) : px) * scale;  // I * 2^q
        if (k0) {
          // 8-bit input: the k = 0 image is the byte itself, summed exactly
          v[0][c] = U8 ? (uint32_t)px : (uint32_t)__float2int_rn(xs);
          v[1][c] = v[2][c] = v[3][c] = 0;
        } else if (U8) {
          const int4 e = lut[(int)px];
          if (ONE) {
            v[0][c] = (uint32_t)(part == 0 ? e.x : part == 1 ? e.y : part == 2 ? e.z : e.w);
          } else if (PAIR) {
            v[0][c] = (uint32_t)(half ? e.y : e.x);
            v[1][c] = (uint32_t)(half ? e.w : e.z);
          } else {
            v[0][c] = (uint32_t)e.x;
            v[1][c] = (uint32_t)e.y;
            v[2][c] = (uint32_t)e.z;
            v[3][c] = (uint32_t)e.w;
          }
        } else if (ONE) {
          // the one table's value, by the same expressions as below
          const float fr = phase_rev(f_hi, f_lo, px);
          const float t = (part & 1) ? __builtin_amdgcn_sinf(fr) : __builtin_amdgcn_cosf(fr);
          v[0][c] = (uint32_t)__float2int_rn(t * (part < 2 ? xs : scale));
        } else if (PAIR) {
          const float fr = phase_rev(f_hi, f_lo, px);
          const float t = half ? __builtin_amdgcn_sinf(fr) : __builtin_amdgcn_cosf(fr);
          v[0][c] = (uint32_t)__float2int_rn(t * xs);
          v[1][c] = (uint32_t)__float2int_rn(t * scale);
        } else {
          const float fr = phase_rev(f_hi, f_lo, px);
          const float C = __builtin_amdgcn_cosf(fr), S = __builtin_amdgcn_sinf(fr);
          v[0][c] = (uint32_t)__float2int_rn(C * xs);
          v[1][c] = (uint32_t)__float2int_rn(S * xs);
          v[2][c] = (uint32_t)__float2int_rn(C * scale);
          v[3][c] = (uint32_t)__float2int_rn(S * scale);
        }
      }
      const int j0 = 4 * lane + 256 * g;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (m >= nimg) break;
        v[m][1] += v[m][0];
        v[m][2] += v[m][1];
        v[m][3] += v[m][2];
        const uint32_t incl = wave_inclusive_scan(v[m][3]);
        const uint32_t excl = incl - v[m][3] + carry[m];
        carry[m] += (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[m][g][c] += v[m][c] + excl;
        if (j0 < p.pitch)
        {
          typedef int v4i __attribute__((ext_vector_type(4)));
          const v4i val = {(int)acc[m][g][0], (int)acc[m][g][1], (int)acc[m][g][2], (int)acc[m][g][3]};
          __builtin_nontemporal_store(val, reinterpret_cast<v4i *>(row + m * te + j0));
        }
      }
    }
  }
}

// Blocks of 4 waves: wave w builds unit 4 unit_group + w of the tile.
template <int G, bool U8, bool ONE, bool PAIR = false>
__device__ __forceinline__ void ka_body(const void *__restrict__ I, const ImageParams &p,
                                        const DevTables *__restrict__ tab, int32_t *__restrict__ ws,
                                        int tile_id, int unit_group) {
  const int unit = unit_group * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (unit >= (ONE ? p.n_images : PAIR ? 2 * p.n_terms : p.n_terms)) return;
  ka_unit<G, U8, ONE, false, PAIR>(I, p, tab, ws, tile_id, unit);
}

template <int G, bool U8, bool ONE, bool PAIR = false>
__global__ __launch_bounds__(256) void ka_sat(const void *__restrict__ I, ImageParams p,
                                             const DevTables *__restrict__ tab,
                                             int32_t *__restrict__ ws) {
  ka_body<G, U8, ONE, PAIR>(I, p, tab, ws, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// K-B, per-pixel form (plans whose staged region or quadruplet count exceeds
// the LDS tile kernel): one thread per pixel, block 64 x 4 pixels, never
// straddling a tile (tile % 64 == 0).  Table reads are raw buffer loads with
// the table offset as a scalar; corners are clamped to [0, H] x [0, W].
// Quadruplets are box sums differenced in int32 like the tile kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  // raw buffer (stride 0), word 3 = 0x00020000 on gfx9-family targets
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ int load_i32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return (int)__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}

// Box sum from the four corners of a quadruplet, (a - b) - (c - d) modulo
// 2^32: exact whenever the box itself fits in int32, even where table
// entries have wrapped.
__device__ __forceinline__ int box_of(int a, int b, int c, int d) {
  return (int)(((uint32_t)a - (uint32_t)b) - ((uint32_t)c - (uint32_t)d));
}

// Denominator of the k = 0 term at pixel (y, x): K~_s correlated with the
// image of ones, whose box sums are the in-image areas of the quadruplets'
// boxes (corners clamped to [0, H] x [0, W]), exact integers.
__device__ __forceinline__ float k0_denominator(const DevTables *__restrict__ tab, int y, int x, int H, int W) {
  float d0 = 0.0f;
  for (int q = 0; q < tab->n_quads; ++q) {
    const int dy = tab->quad_dy[q], dx = tab->quad_dx[q];
    const int h = min(max(y + dy, 0), H) - min(max(y + 1 - dy, 0), H);
    const int w = min(max(x + dx, 0), W) - min(max(x + 1 - dx, 0), W);
    d0 = __builtin_fmaf(tab->quad_w[q], (float)(h * w), d0);
  }
  return d0;
}

template <bool U8>
__global__ __launch_bounds__(256) void kb_lookup(const void *__restrict__ I, ImageParams p,
                                                 const DevTables *__restrict__ tab,
                                                 const int32_t *__restrict__ ws,
                                                 float *__restrict__ out, float *__restrict__ num_out,
                                                 float *__restrict__ den_out) {
  const int bx0 = blockIdx.x * 64, by0 = blockIdx.y * 4;
  const int x = bx0 + (threadIdx.x & 63);
  const int y = by0 + (threadIdx.x >> 6);
  if (x >= p.W || y >= p.H) return;
  const int ty = by0 / p.tile, tx = bx0 / p.tile;
  const int tile_id = ty * p.tiles_x + tx;
  const int oy = max(ty * p.tile - p.radius, 0), ox = max(tx * p.tile - p.radius, 0);
  const uint32_t te4 = (uint32_t)p.table_elems * 4u;
  const __amdgpu_buffer_rsrc_t rsrc =
      make_rsrc(ws + (long long)tile_id * p.n_images * p.table_elems, te4 * (uint32_t)p.n_images);
  auto corner = [&](int dy, int dx) {
    const int Y = min(max(y + dy, 0), p.H) - oy, X = min(max(x + dx, 0), p.W) - ox;
    return (uint32_t)(Y * p.pitch + X) * 4u;
  };
  const int nq = tab->n_quads;

  float px, xv;
  load_pixel<U8>(I, (long long)y * p.W + x, &px, &xv);
  const float inv = p.inv_sat_scale;
  float num = 0.0f, den = 0.0f;
  for (int t = 0; t < p.n_terms; ++t) {
    const uint32_t sb = (uint32_t)tab->slot[t] * te4;
    const bool k0 = tab->k_is_zero[t] != 0;
    const int nimg = k0 ? 1 : 4;
    float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int q = 0; q < nq; ++q) {
      const int dy = tab->quad_dy[q], dx = tab->quad_dx[q];
      const uint32_t oa = corner(dy, dx), ob = corner(1 - dy, dx);
      const uint32_t oc = corner(dy, 1 - dx), od = corner(1 - dy, 1 - dx);
      const float w = tab->quad_w[q];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (m >= nimg) break;
        const uint32_t so = sb + (uint32_t)m * te4;
        const int box = box_of(load_i32(rsrc, oa, so), load_i32(rsrc, ob, so), load_i32(rsrc, oc, so),
                               load_i32(rsrc, od, so));
        s[m] = __builtin_fmaf(w, (float)box, s[m]);
      }
    }
    const float a = tab->a[t];
    if (k0) {
      // numerator a_0 (K * I); denominator a_0 (K * 1)
      num = __builtin_fmaf(a * (U8 ? 1.0f / 255.0f : inv), s[0], num);
      den = __builtin_fmaf(a, k0_denominator(tab, y, x, p.H, p.W), den);
      continue;
    }
    const float fr = phase_rev(tab->f_hi[t], tab->f_lo[t], px);
    const float C = __builtin_amdgcn_cosf(fr), S = __builtin_amdgcn_sinf(fr);
    num = __builtin_fmaf(a * inv, C * s[0] + S * s[1], num);
    den = __builtin_fmaf(a * inv, C * s[2] + S * s[3], den);
  }
  const long long idx = (long long)y * p.W + x;
  out[idx] = den > tab->den_floor ? num / den : xv;
  if (num_out) num_out[idx] = num;
  if (den_out) den_out[idx] = den;
}

// ---------------------------------------------------------------------------
// K-B (LDS tile form): one block per 64 x 64 output tile; tables are the
// outer loop.  For each table the block copies the region its taps read --
// (64 + dy span) rows x (64 + dx span) columns, border clamp applied through
// the per-lane source columns -- from the workspace straight into LDS with
// buffer-to-LDS loads (no registers, no vector instructions), then every
// pixel reads its taps from LDS.  Symmetric quadruplets of taps are one box
// sum differenced exactly in int32 and one FP32 FMA.  Each thread owns the
// pixels (wave + 16 i, lane), i < 4, of the tile: one precomputed LDS address
// per quadruplet corner serves all four through instruction offsets.  When
// two regions fit in LDS they are double-buffered with their rows
// interleaved (row r of buffer b at (2r + b) * PITCH), so the second buffer
// is an instruction offset too and each table costs one barrier; the copy of
// table m + 1 runs while table m is read.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void_t;

// How the LDS tile kernel stages each table's region:
// - single: copies straight into one LDS buffer after the barrier that ends
//   the previous table;
// - double: two interleaved LDS buffers, the next table's copy running while
//   the current one is read;
// - overlap: where two regions do not fit, two layouts that overlap, the
//   second kOverlapBase(PITCH) rows below the first.  Tables alternate
//   between them; the rows of the next table that fall outside the current
//   one's are copied straight into LDS while it is read, the overlapping
//   rows are loaded into registers meanwhile and written to LDS after the
//   barrier that ends the current table.
constexpr int kStageSingle = 0, kStageDouble = 1, kStageOverlap = 2;
constexpr int kLdsBytes = 160 * 1024;
// The second layout's first row: as far down as LDS allows for regions 15
// rows shorter than the pitch (the shortest of the pitch's class), but with
// the layout's byte offset plus a thread's pixel offsets (3 x 4 rows)
// within an instruction offset, a multiple of 256 bytes (paired reads count
// offsets in 256-byte units up to 255).  Regions up to kLdsBytes / (4 pitch)
// - kOverlapBase(pitch) rows tall take overlap staging.
__host__ __device__ constexpr int kOverlapBase(int pitch) {
  int ob = kLdsBytes / (pitch * 4) - (pitch - 15);
  while (ob > 0 && ((ob + 12) * pitch * 4 > 65535 || (ob * pitch * 4) % 256 != 0)) --ob;
  return ob;
}
__host__ __device__ constexpr int kOverlapMaxRows(int pitch) { return kLdsBytes / (pitch * 4) - kOverlapBase(pitch); }

// The fold of one table's correlation s (Eq. 1D_N_terms): parts 0 and 1
// (C I, S I) add a_k C s and a_k S s to the numerator, parts 2 and 3 (C, S)
// the same to the denominator, part 4 (I of k = 0) a_0 s to the numerator.
// The wave-uniform part picks the weights (an, ad) = (a, 0) or (0, a) and
// the per-pixel factor; the other accumulator takes 0 * s, which leaves it
// unchanged.  No branch selects the accumulator, so the per-pixel arrays stay
// in registers (a branch that stores to num[i] or den[i] is merged by the
// compiler into one store through a selected pointer, which puts both arrays
// in scratch memory).
__device__ __forceinline__ void fold_weights(int part, float a, float *an, float *ad) {
  const bool to_num = part < 2 || part == 4;
  *an = to_num ? a : 0.0f;
  *ad = to_num ? 0.0f : a;
}

__device__ __forceinline__ void fold_table(int part, float an, float ad, float cs, float sn, float s,
                                           float &num, float &den) {
  const float f = part == 4 ? 1.0f : (part & 1) ? sn : cs;
  num = __builtin_fmaf(an * f, s, num);
  den = __builtin_fmaf(ad * f, s, den);
}

__device__ __forceinline__ int lds_ld(const int *lds, uint32_t byte_addr) {
  return *reinterpret_cast<const int *>(reinterpret_cast<const char *>(lds) + byte_addr);
}

// The 64 x 64 output tile with index L in the XCD-aware order: XCD k takes
// the k-th contiguous eighth of the tiles (L in [k per_xcd, (k + 1) per_xcd)),
// walked in patches of 8 x 4 tiles, so the tiles one XCD runs at the same time
// are neighbours whose staged halos overlap in that XCD's L2.  Patch rows of
// PH tile rows (the last may be shorter); within one, patches of PW tile
// columns (the last may be narrower); tiles row-major in a patch.
__device__ __forceinline__ void kb_tile_origin(int L, int H, int W, int *y0, int *x0) {
  const int ntx = (W + 63) / 64, nty = (H + 63) / 64;
  constexpr int PW = 8, PH = 4;
  const int pr = L / (PH * ntx);
  const int rem = L - pr * PH * ntx;
  const int ph = min(PH, nty - pr * PH);
  const int pc = rem / (PW * ph);
  const int in = rem - pc * PW * ph;
  const int pw = min(PW, ntx - pc * PW);
  *x0 = (pc * PW + in % pw) * 64;
  *y0 = (pr * PH + in / pw) * 64;
}

// One 64 x 64 output tile of one image; L is the tile's index in the
// XCD-aware order (kb_tile_origin).  Every thread of the block calls it.
template <int PITCH, int NQ, int ST, bool U8>
__device__ __forceinline__ void kb_body(const void *__restrict__ I, const ImageParams &p,
                                        const DevTables *__restrict__ tab,
                                        const int32_t *__restrict__ ws, float *__restrict__ out,
                                        float *__restrict__ num_out, float *__restrict__ den_out,
                                        int L) {
  constexpr bool DB = ST == kStageDouble, OV = ST == kStageOverlap;
  constexpr int NW = 16;                          // waves
  constexpr int PX = 64 / NW;                     // rows of the tile per thread
  constexpr int RS = DB ? 2 * PITCH : PITCH;      // LDS row stride (int32 elements)
  constexpr int CC = (PITCH + 63) / 64;           // 64-column chunks of a staged row
  constexpr int OB = OV ? kOverlapBase(PITCH) : 0;  // first row of the second layout
  // a thread's pixels: tile rows wave + NW i, or with overlap staging
  // 16 (wave / 4) + wave % 4 + 4 i (the second layout's offset and the
  // pixels' offsets then both fit an instruction offset)
  constexpr int PROW = OV ? 4 : NW;
  constexpr uint32_t PSTEP = PROW * RS * 4;       // bytes between a thread's pixels
  constexpr uint32_t BSTEP = (OV ? OB * PITCH : PITCH) * 4;  // bytes from buffer 0 to buffer 1
  extern __shared__ int lds[];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int x0, y0;
  kb_tile_origin(L, p.H, p.W, &y0, &x0);
  const int ty = y0 / p.tile, tx = x0 / p.tile;
  const int tile_id = ty * p.tiles_x + tx;
  const int oy = max(ty * p.tile - p.radius, 0), ox = max(tx * p.tile - p.radius, 0);
  const int dy0 = tab->tap_dy_min, dx0 = tab->tap_dx_min;
  const int RH = 64 + tab->tap_dy_max - dy0, RW = 64 + tab->tap_dx_max - dx0;
  const uint32_t te4 = (uint32_t)p.table_elems * 4u;
  const __amdgpu_buffer_rsrc_t rsrc =
      make_rsrc(ws + (long long)tile_id * p.n_images * p.table_elems, te4 * (uint32_t)p.n_images);
  const int x = x0 + lane;
  const bool xin = x < p.W;
  const int prow0 = OV ? 16 * (wave >> 2) + (wave & 3) : wave;  // tile row of the thread's pixel 0

  // staging: wave w copies region rows w, w + NW, ...; lane l columns l,
  // l + 64, ...  The clamped source column is fixed per lane (vector offset),
  // the table and row part is wave-uniform (scalar offset), the LDS target is
  // the wave-uniform row start plus 4 bytes per lane.
  uint32_t xoff4[CC];
#pragma unroll
  for (int c = 0; c < CC; ++c) xoff4[c] = (uint32_t)(min(max(x0 + dx0 + lane + 64 * c, 0), p.W) - ox) * 4u;
  const uint32_t gp4 = (uint32_t)p.pitch * 4u;
  // where the region's columns need no clamp and start on a 16-byte boundary
  // of the table, a row is one 16-byte copy per lane (lanes 0 .. RW / 4; the
  // last lane's spare columns land in the row's padding)
  const int cx0 = x0 + dx0 - ox;  // table column of region column 0
  const bool wide = x0 + dx0 >= 0 && x0 + dx0 + RW - 1 <= p.W && (cx0 & 3) == 0;
  const uint32_t xoff16 = (uint32_t)(cx0 + 4 * lane) * 4u;
  const bool lane16 = 4 * lane < RW;
  auto copy_row = [&](int *dst, uint32_t soff) {
    if (wide) {
      if (lane16) __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void_t *)dst, 16, xoff16, soff, 0, 0);
    } else {
#pragma unroll
      for (int c = 0; c < CC; ++c)
        if (lane + 64 * c < RW)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void_t *)(dst + 64 * c), 4, xoff4[c], soff, 0, 0);
    }
  };
  auto stage = [&](int m, int buf) {
    const uint32_t sm = (uint32_t)m * te4;
    for (int r = wave; r < RH; r += NW) {
      const int Y = min(max(y0 + dy0 + r, 0), p.H) - oy;
      copy_row(lds + r * RS + buf * PITCH, sm + (uint32_t)Y * gp4);
    }
  };

  // overlap staging: region rows [r0, r1) of table m straight into LDS rows
  // base + r; rows r0 + wave + NW i < r1 (i < RR) into registers and from
  // there into LDS rows base + r
  auto stage_rows = [&](int m, int base, int r0, int r1) {
    const uint32_t sm = (uint32_t)m * te4;
    for (int r = r0 + wave; r < r1; r += NW) {
      const int Y = min(max(y0 + dy0 + r, 0), p.H) - oy;
      copy_row(lds + (base + r) * PITCH, sm + (uint32_t)Y * gp4);
    }
  };
  constexpr int RR = OV ? (kOverlapMaxRows(PITCH) - OB + NW - 1) / NW : 1;
  int rv[RR][CC];
  // (every register is loaded, rows past the range from clamped rows of the
  // table, and only the range is written to LDS: a load under a condition
  // would make the compiler wait for it to merge the register's two values)
  auto fetch = [&](int m, int r0) {
    const uint32_t sm = (uint32_t)m * te4;
#pragma unroll
    for (int i = 0; i < RR; ++i) {
      const int r = r0 + wave + NW * i;
      const int Y = min(max(y0 + dy0 + r, 0), p.H) - oy;
      const uint32_t soff = sm + (uint32_t)Y * gp4;
#pragma unroll
      for (int c = 0; c < CC; ++c) rv[i][c] = load_i32(rsrc, xoff4[c], soff);
    }
  };
  auto deposit = [&](int base, int r0, int r1) {
#pragma unroll
    for (int i = 0; i < RR; ++i) {
      const int r = r0 + wave + NW * i;
      if (r < r1) {
#pragma unroll
        for (int c = 0; c < CC; ++c)
          if (lane + 64 * c < RW) lds[(base + r) * PITCH + lane + 64 * c] = rv[i][c];
      }
    }
  };

  // LDS byte address of each quadruplet corner for this thread's pixel 0 in
  // buffer 0: region row r holds image row y0 + dy0 + r, so tap (dy, dx) of
  // the pixel in tile row prow0, column lane is at element
  // (prow0 + dy - dy0) * RS + lane + dx - dx0.  Padding quadruplets read one
  // valid element four times with weight 0.
  const uint32_t lb = (uint32_t)(prow0 * RS + lane) * 4u;
  const int nq = tab->n_quads;
  uint32_t qa[NQ][4];
  float qw[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (q < nq) {
      const int dy = tab->quad_dy[q], dx = tab->quad_dx[q];
      const int ra = dy - dy0, rb = 1 - dy - dy0, ca = dx - dx0, cb = 1 - dx - dx0;
      qa[q][0] = lb + (uint32_t)(ra * RS + ca) * 4u;
      qa[q][1] = lb + (uint32_t)(rb * RS + ca) * 4u;
      qa[q][2] = lb + (uint32_t)(ra * RS + cb) * 4u;
      qa[q][3] = lb + (uint32_t)(rb * RS + cb) * 4u;
      qw[q] = tab->quad_w[q];
    } else {
      qa[q][0] = qa[q][1] = qa[q][2] = qa[q][3] = lb;
      qw[q] = 0.0f;
    }
  }

  float pxv[PX];
  float num[PX], den[PX];
#pragma unroll
  for (int i = 0; i < PX; ++i) {
    const int y = y0 + prow0 + PROW * i;
    pxv[i] = 0.0f;
    if (xin && y < p.H) {
      float px, v;
      load_pixel<U8>(I, (long long)y * p.W + x, &px, &v);
      pxv[i] = px;
    }
    num[i] = 0.0f;
    den[i] = 0.0f;
  }
  const float inv = p.inv_sat_scale;
  float cs[PX], sn[PX];
#pragma unroll
  for (int i = 0; i < PX; ++i) cs[i] = sn[i] = 0.0f;
  // the pixels have landed before the table loop: otherwise the first use of
  // a pixel inside the loop waits for every load in flight, the next table's
  // region included
#pragma unroll
  for (int i = 0; i < PX; ++i) asm volatile("" ::"v"(pxv[i]));

  // one table: box sums of every quadruplet, then the fold of Eq. 1D_N_terms
  // into the numerator / denominator
  auto body = [&](int m, auto BUF) {
    constexpr uint32_t bo = decltype(BUF)::value * BSTEP;
    const int part = tab->slot_part[m];
    const float fhi = tab->slot_fhi[m], flo = tab->slot_flo[m];
    const float at = tab->slot_a[m];
    if (part == 0) {
#pragma unroll
      for (int i = 0; i < PX; ++i) {
        const float fr = phase_rev(fhi, flo, pxv[i]);
        cs[i] = __builtin_amdgcn_cosf(fr);
        sn[i] = __builtin_amdgcn_sinf(fr);
      }
    }
    float s[PX];
#pragma unroll
    for (int i = 0; i < PX; ++i) s[i] = 0.0f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
      for (int i = 0; i < PX; ++i) {
        const uint32_t o = i * PSTEP + bo;
        const int box = box_of(lds_ld(lds, qa[q][0] + o), lds_ld(lds, qa[q][1] + o),
                               lds_ld(lds, qa[q][2] + o), lds_ld(lds, qa[q][3] + o));
        s[i] = __builtin_fmaf(qw[q], (float)box, s[i]);
      }
    }
    // software pipeline of the quadruplet loop: the reads of D quadruplets
    // first, then the arithmetic of quadruplet q beside the reads of q + D
    // (D = 1 with overlap staging at pitch 160, where it measured faster)
    constexpr int D = OV && PITCH == 160 ? 1 : 2;
    __builtin_amdgcn_sched_group_barrier(0x100, 8 * D, 0);
#pragma unroll
    for (int q = 0; q + D < NQ; ++q) {
      __builtin_amdgcn_sched_group_barrier(0x002, 5 * PX, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x002, 5 * D * PX, 0);
    // the box sums are complete here (an empty statement that keeps the
    // compiler from interleaving the pixels' quadruplet chains, which spills)
#pragma unroll
    for (int i = 0; i < PX; ++i) asm volatile("" : "+v"(s[i]));
    // the k = 0 table of 8-bit input holds bytes: scale 1/255 instead of 2^-q
    const float ai = at * (U8 && part == 4 ? 1.0f / 255.0f : inv);
    float an, ad;
    fold_weights(part, ai, &an, &ad);
#pragma unroll
    for (int i = 0; i < PX; ++i) fold_table(part, an, ad, cs[i], sn[i], s[i], num[i], den[i]);
    if (part == 4) {
      // denominator of the k = 0 term: a_0 (K * 1)
#pragma unroll
      for (int i = 0; i < PX; ++i)
        den[i] = __builtin_fmaf(at, k0_denominator(tab, y0 + prow0 + PROW * i, x, p.H, p.W), den[i]);
    }
  };

  const int n = tab->n_images;  // this plan's tables (the workspace may hold more: p.n_images)
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, 1>;
  if (DB) {
    stage(0, 0);
    for (int m = 0; m < n; m += 2) {
      // this wave's copy of table m has landed; after the barrier every
      // wave's has, and every wave is done reading buffer 1 (table m - 1)
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (m + 1 < n) stage(m + 1, 1);
      body(m, B0{});
      if (m + 1 < n) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (m + 2 < n) stage(m + 2, 0);
        body(m + 1, B1{});
      }
    }
  } else if (OV) {
    // table m in layout m & 1 (LDS rows (m & 1) OB + r).  Table m + 1 in
    // layout 1: rows [nov, RH) fall below table m's rows, [0, nov) on them;
    // in layout 0: rows [0, OB) fall above table m's rows, [OB, RH) on them
    // (none when RH <= OB).
    const int nov = max(RH - OB, 0);
    stage_rows(0, 0, 0, RH);
    for (int m = 0; m < n; ++m) {
      const int b = m & 1;
      __syncthreads();  // every wave is done reading table m - 1
      if (m > 0) deposit(b ? OB : 0, b ? 0 : OB, b ? nov : RH);
      __builtin_amdgcn_s_waitcnt(0);  // this wave's copies and writes of table m are done
      __syncthreads();                // table m is whole in LDS
      // table m + 1 (the last table loads itself again, unused)
      if (m + 1 < n) stage_rows(m + 1, b ? 0 : OB, b ? 0 : nov, b ? min(OB, RH) : RH);
      fetch(min(m + 1, n - 1), b ? OB : 0);
      // the loads of table m + 1 stay ahead of the reads of table m
      __builtin_amdgcn_sched_barrier(0);
      if (b) body(m, B1{});
      else body(m, B0{});
    }
  } else {
    for (int m = 0; m < n; ++m) {
      __syncthreads();  // every wave is done reading table m - 1
      stage(m, 0);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      body(m, B0{});
    }
  }
#pragma unroll
  for (int i = 0; i < PX; ++i) {
    const int y = y0 + prow0 + PROW * i;
    if (!xin || y >= p.H) continue;
    const long long idx = (long long)y * p.W + x;
    const float xv = U8 ? pxv[i] * (1.0f / 255.0f) : pxv[i];
    out[idx] = den[i] > tab->den_floor ? num[i] / den[i] : xv;
    if (num_out) num_out[idx] = num[i];
    if (den_out) den_out[idx] = den[i];
  }
}

// Blocks are dispatched round-robin over the 8 XCDs: block b runs on XCD
// b % 8 and takes the (b / 8)-th tile of that XCD's eighth.
template <int PITCH, int NQ, int ST, bool U8>
__global__ __launch_bounds__(1024) void kb_tile(const void *__restrict__ I, ImageParams p,
                                               const DevTables *__restrict__ tab,
                                               const int32_t *__restrict__ ws,
                                               float *__restrict__ out, float *__restrict__ num_out,
                                               float *__restrict__ den_out) {
  const int n_tiles = ((p.W + 63) / 64) * ((p.H + 63) / 64);
  const int per_xcd = (n_tiles + 7) / 8;
  const int L = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (L >= n_tiles) return;
  kb_body<PITCH, NQ, ST, U8>(I, p, tab, ws, out, num_out, den_out, L);
}

// ---------------------------------------------------------------------------
// K-B, lattice form.  For plans whose quadruplet rows lie on a lattice, dy_j
// = dy_0 + j s (j < M), every thread owns U = 8 pixels of one column spaced
// s rows apart: pixel u's top corner of row j (1 - dy_j) and pixel u''s with
// u' - j' = u - j are the same table row, and likewise at the bottom, so the
// U pixels' boxes read only U + M - 1 distinct rows per side, and each row's
// difference between a box's right and left corner columns, h = S(row, R_i)
// - S(row, L_i), is taken once and serves up to min(U, M) boxes:
//   box(u, j, i) = h(bottom row u + j, i) - h(top row u + M - 1 - j, i),
// exact in int32 like the four-corner form (the same integer).  At r = 48
// (s = 12, M = N = 4) that is 22 table reads per pixel and table against the
// four-corner form's 48.
//
// The block stages the whole region of a table (TR + dy span rows) in LDS,
// its rows stored by residue modulo s, so a thread's U + M - 1 top rows are
// consecutive LDS rows, and so are its bottom rows: every offset of one side
// is an instruction immediate from one address per corner column.  A table
// is read in two phases, the top rows' differences first (kept in
// registers), then the bottom rows, the boxes and the fold.  The region's
// first B0 rows hold top corners only, and with one lattice group the rows of
// residue rho are read only by wave rho: each wave copies those rows of the
// next table as soon as its own top phase has read them, so that copy runs
// beside the bottom phase; the other rows are copied after the barrier that
// ends the table.
//
// Output tiles are TR = s U G rows (G groups of s waves) by 64 columns,
// clipped to the table tile they lie in.  The block has NWV waves: all
// copy, the first s G compute (NWV = 16, or 12 where s G = 12 for the N_s = 8
// box pattern, so no wave only copies).  Each pixel sums its boxes in (dy, dx) order, the
// order of the plan's quadruplet list, so the result is bitwise that of the
// LDS tile kernel.
// ---------------------------------------------------------------------------
constexpr int kLatU = 8;
// lattice box mask (bit 4 j + i) of the N_s = 8 Gaussian expansion: its
// eight level groups leave no box whose row and column indices are both 0 or
// 2 (offsets of 1 and 3 lattice steps)
constexpr uint32_t kLatMaskNs8 = 0xFAFAu;

// LDS of the lattice kernel: the region's rows, every residue class modulo s
// padded to the same count
size_t lattice_lds_bytes(const DevTables &h) {
  const int RH = h.lat_s * kLatU * h.lat_g + h.tap_dy_max - h.tap_dy_min;
  const int KB = (RH + h.lat_s - 1) / h.lat_s;
  return (size_t)h.lat_s * KB * h.lat_pitch * sizeof(int32_t);
}

// Output-tile grid of the lattice kernel for an image: rows of tiles per table
// tile (nsub), tile rows in all (nty) and columns (ntx).
struct LatGrid {
  int TR, nsub, nty, ntx;
};
__host__ __device__ inline LatGrid lat_grid(int H, int W, int tile, int s, int g) {
  LatGrid q;
  q.TR = s * kLatU * g;
  q.nsub = (tile + q.TR - 1) / q.TR;
  const int tty = (H + tile - 1) / tile;
  const int last = H - (tty - 1) * tile;
  q.nty = (tty - 1) * q.nsub + (last + q.TR - 1) / q.TR;
  q.ntx = (W + 63) / 64;
  return q;
}

// MASK: bit 4 j + i set where the plan may have a box (dy_j, dx_i); boxes
// outside it have weight 0 and are skipped (adding 0 changes no bit).
template <int PITCH, int M, int N, bool U8, uint32_t MASK = 0xFFFFu, int NWV = 16>
__device__ __forceinline__ void kl_body(const void *__restrict__ I, const ImageParams &p,
                                        const DevTables *__restrict__ tab,
                                        const int32_t *__restrict__ ws, float *__restrict__ out,
                                        float *__restrict__ num_out, float *__restrict__ den_out, int L) {
  constexpr int U = kLatU;
  constexpr int KT = U + M - 1;      // distinct corner rows per side and thread
  constexpr uint32_t P4 = PITCH * 4u;
  constexpr int CC = (PITCH + 63) / 64;
  extern __shared__ int lds[];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int s = tab->lat_s, G = tab->lat_g;
  const LatGrid lg = lat_grid(p.H, p.W, p.tile, s, G);
  // XCD-aware patches of one table tile each (or of its first rows, to fit
  // the 32 CUs of an XCD): the tiles one XCD runs at the same time read one
  // tile's tables, whose halo rows and columns they share in that XCD's L2
  const int PW = p.tile / 64;
  int PH = lg.nsub;
  while (PH > 1 && PW * PH > 32) PH = (PH + 1) / 2;
  const int pr = L / (PH * lg.ntx);
  const int rem = L - pr * PH * lg.ntx;
  const int ph = min(PH, lg.nty - pr * PH);
  const int pc = rem / (PW * ph);
  const int in = rem - pc * PW * ph;
  const int pw = min(PW, lg.ntx - pc * PW);
  const int bx = pc * PW + in % pw, by = pr * PH + in / pw;
  const int tyt = by / lg.nsub, ksub = by - tyt * lg.nsub;
  const int y0 = tyt * p.tile + ksub * lg.TR;                 // tile rows [y0, y1)
  const int y1 = min(min(y0 + lg.TR, (tyt + 1) * p.tile), p.H);
  const int x0 = bx * 64, txt = x0 / p.tile;
  const int tile_id = tyt * p.tiles_x + txt;
  const int oy = max(tyt * p.tile - p.radius, 0), ox = max(txt * p.tile - p.radius, 0);
  const int dy0 = tab->tap_dy_min, dx0 = tab->tap_dx_min;
  const int RW = 64 + tab->tap_dx_max - dx0;
  const int dymax = tab->lat_dy0 + (M - 1) * s;
  const int B0 = tab->lat_dy0 - dy0;                          // region row of the first bottom corner
  const int RH = lg.TR + dymax - dy0;                          // region rows (image rows y0 + dy0 + R)
  const int KB = (RH + s - 1) / s;                             // LDS rows per residue class
  const int erows = (int)(p.table_elems / p.pitch);            // rows of a table
  const uint32_t te4 = (uint32_t)p.table_elems * 4u;
  const __amdgpu_buffer_rsrc_t rsrc =
      make_rsrc(ws + (long long)tile_id * p.n_images * p.table_elems, te4 * (uint32_t)p.n_images);
  const int x = x0 + lane;
  const bool xin = x < p.W;

  // Copies.  Region row R of table m goes to LDS row (R mod s) KB + R div s.
  uint32_t xoff4[CC];
#pragma unroll
  for (int c = 0; c < CC; ++c) xoff4[c] = (uint32_t)(min(max(x0 + dx0 + lane + 64 * c, 0), p.W) - ox) * 4u;
  const uint32_t gp4 = (uint32_t)p.pitch * 4u;
  // where the region's columns need no clamp and start on a 16-byte boundary
  // of the table, a row is one 16-byte copy per lane (lanes 0 .. RW/4)
  const int cx0 = x0 + dx0 - ox;  // table column of region column 0
  const bool wide = x0 + dx0 >= 0 && x0 + dx0 + RW - 1 <= p.W && (cx0 & 3) == 0;
  const uint32_t xoff16 = (uint32_t)(cx0 + 4 * lane) * 4u;
  const bool lane16 = 4 * lane < RW;
  const int nchunk = (RW + 63) / 64;
  auto copy_row = [&](int m, int R, int lrow) {
    const int Y = min(min(max(y0 + dy0 + R, 0), p.H) - oy, erows - 1);
    const uint32_t soff = (uint32_t)m * te4 + (uint32_t)Y * gp4;
    int *dst = lds + lrow * PITCH;
    if (wide) {
      if (lane16) __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void_t *)dst, 16, xoff16, soff, 0, 0);
    } else {
#pragma unroll
      for (int c = 0; c < CC; ++c)
        if (c < nchunk && lane + 64 * c < RW)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void_t *)(dst + 64 * c), 4, xoff4[c], soff, 0, 0);
    }
  };
  // rows [lo, RH) of table m: wave w copies rows lo + w, lo + w + NWV, ...
  const int d16 = NWV / s, m16 = NWV - d16 * s;
  auto stage_from = [&](int m, int lo) {
    int R = lo + wave;
    int rq = R / s, rr = R - rq * s;
    for (; R < RH; R += NWV) {
      copy_row(m, R, rr * KB + rq);
      rq += d16;
      rr += m16;
      if (rr >= s) {
        rr -= s;
        ++rq;
      }
    }
  };

  // this wave's pixels: group g, residue rho; pixel u at tile row g s U + rho + u s
  const bool comp = wave < s * G;
  const int g = comp ? wave / s : 0, rho = comp ? wave - (wave / s) * s : 0;
  const int tq = rho * KB + g * U;             // LDS row of the thread's first top corner row
  const int cb = B0 + rho;                      // region row of its first bottom corner row (group 0)
  const int bq = (cb % s) * KB + cb / s + g * U;  // its LDS row
  uint32_t aTL[N], aTR[N], aBL[N], aBR[N];      // LDS byte addresses per corner column
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int dx = tab->lat_dx[i];
    const uint32_t cl = (uint32_t)(lane + 1 - dx - dx0) * 4u, cr = (uint32_t)(lane + dx - dx0) * 4u;
    aTL[i] = tq * P4 + cl;
    aTR[i] = tq * P4 + cr;
    aBL[i] = bq * P4 + cl;
    aBR[i] = bq * P4 + cr;
  }
  float wq[M][N];
#pragma unroll
  for (int j = 0; j < M; ++j)
#pragma unroll
    for (int i = 0; i < N; ++i) wq[j][i] = tab->lat_w[4 * j + i];

  float pxv[U], num[U], den[U], cs[U], sn[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int y = y0 + g * s * U + rho + u * s;
    pxv[u] = 0.0f;
    if (comp && xin && y < y1) {
      float px, v;
      load_pixel<U8>(I, (long long)y * p.W + x, &px, &v);
      pxv[u] = px;
    }
    num[u] = den[u] = 0.0f;
    cs[u] = sn[u] = 0.0f;
  }
  const float inv = p.inv_sat_scale;

  const int n = tab->n_images;  // this plan's tables (the workspace may hold more: p.n_images)
  const bool own = G == 1;      // copy of the top-only rows by their one reader
  stage_from(0, 0);
  for (int m = 0; m < n; ++m) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of table m have landed
    __syncthreads();                // every wave's have
    const bool ahead = m + 1 < n;
    if (comp) {
      const int part = tab->slot_part[m];
      const float fhi = tab->slot_fhi[m], flo = tab->slot_flo[m];
      const float at = tab->slot_a[m];
      if (part == 0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const float fr = phase_rev(fhi, flo, pxv[u]);
          cs[u] = __builtin_amdgcn_cosf(fr);
          sn[u] = __builtin_amdgcn_sinf(fr);
        }
      }
      // top phase: the differences of the thread's top corner rows
      int ht[KT][N];
#pragma unroll
      for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int i = 0; i < N; ++i)
          ht[kt][i] = (int)((uint32_t)lds_ld(lds, aTR[i] + kt * P4) - (uint32_t)lds_ld(lds, aTL[i] + kt * P4));
      if (own && ahead) {
        // the top rows are in registers before the next table's copy lands on them
#pragma unroll
        for (int kt = 0; kt < KT; ++kt)
#pragma unroll
          for (int i = 0; i < N; ++i) asm volatile("" : "+v"(ht[kt][i]));
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
        for (int R = rho, q = 0; R < B0; R += s, ++q) copy_row(m + 1, R, rho * KB + q);
      }
      // bottom phase: the boxes and the fold
      float sv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) sv[u] = 0.0f;
      // two rows at a time (their reads pair into one instruction per column)
#pragma unroll
      for (int k2 = 0; k2 < KT; k2 += 2) {
        uint32_t hb[2][N];
#pragma unroll
        for (int t = 0; t < 2 && k2 + t < KT; ++t)
#pragma unroll
          for (int i = 0; i < N; ++i)
            hb[t][i] = (uint32_t)lds_ld(lds, aBR[i] + (k2 + t) * P4) - (uint32_t)lds_ld(lds, aBL[i] + (k2 + t) * P4);
        // one difference per row, shared by the row's boxes (the compiler
        // would otherwise fold it into each box as an add and a subtract)
#pragma unroll
        for (int t = 0; t < 2 && k2 + t < KT; ++t)
#pragma unroll
          for (int i = 0; i < N; ++i) asm volatile("" : "+v"(hb[t][i]));
#pragma unroll
        for (int t = 0; t < 2 && k2 + t < KT; ++t) {
          const int kb = k2 + t;
#pragma unroll
          for (int i = 0; i < N; ++i) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const int j = kb - u;
              if (j < 0 || j >= M || !((MASK >> (4 * j + i)) & 1u)) continue;
              // pairs without a quadruplet carry weight 0 (adding 0 changes no bit)
              const int box = (int)(hb[t][i] - (uint32_t)ht[u + M - 1 - j][i]);
              sv[u] = __builtin_fmaf(wq[j][i], (float)box, sv[u]);
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) asm volatile("" : "+v"(sv[u]));
      // the k = 0 table of 8-bit input holds bytes: scale 1/255 instead of 2^-q
      const float ai = at * (U8 && part == 4 ? 1.0f / 255.0f : inv);
      float an, ad;
      fold_weights(part, ai, &an, &ad);
#pragma unroll
      for (int u = 0; u < U; ++u) fold_table(part, an, ad, cs[u], sn[u], sv[u], num[u], den[u]);
      if (part == 4) {
        // denominator of the k = 0 term: a_0 (K * 1)
#pragma unroll
        for (int u = 0; u < U; ++u)
          den[u] = __builtin_fmaf(at, k0_denominator(tab, y0 + g * s * U + rho + u * s, x, p.H, p.W), den[u]);
      }
    }
    __syncthreads();  // every wave is done reading table m
    if (ahead) stage_from(m + 1, own ? B0 : 0);
  }
  if (!comp || !xin) return;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int y = y0 + g * s * U + rho + u * s;
    if (y >= y1) continue;
    const long long idx = (long long)y * p.W + x;
    const float xv = U8 ? pxv[u] * (1.0f / 255.0f) : pxv[u];
    out[idx] = den[u] > tab->den_floor ? num[u] / den[u] : xv;
    if (num_out) num_out[idx] = num[u];
    if (den_out) den_out[idx] = den[u];
  }
}

template <int PITCH, int M, int N, bool U8, uint32_t MASK = 0xFFFFu, int NWV = 16>
__global__ __launch_bounds__(64 * NWV) void kl_tile(const void *__restrict__ I, ImageParams p,
                                               const DevTables *__restrict__ tab,
                                               const int32_t *__restrict__ ws,
                                               float *__restrict__ out, float *__restrict__ num_out,
                                               float *__restrict__ den_out, int n_tiles) {
  const int per_xcd = (n_tiles + 7) / 8;
  const int L = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (L >= n_tiles) return;
  kl_body<PITCH, M, N, U8, MASK, NWV>(I, p, tab, ws, out, num_out, den_out, L);
}

// ---------------------------------------------------------------------------
// Direct summation of Eq. BF (the brute-force baseline of the paper): one
// thread per pixel, 64 x 4 pixels per block; the block's image tile with an
// r-pixel halo and the K_s window are staged in LDS.  Neighbours outside the
// image are staged as a large value whose range weight underflows to 0, so
// the inner loop has no branch: w = K_s(d) 2^(c (v - v0)^2) (Gaussian K_r;
// 2^(c |v - v0|) for the exponential), num += w v, den += w, in FP32
// (den >= 1: the centre's weight).
// ---------------------------------------------------------------------------
template <bool U8, bool ABS>
__device__ __forceinline__ void direct_body(const void *__restrict__ I, int H, int W, int r,
                                            const float *__restrict__ Ks, float c, float *__restrict__ out,
                                            float *__restrict__ num_out, float *__restrict__ den_out,
                                            int bx, int by) {
  extern __shared__ float sh[];
  const int K = 2 * r + 1, TW = 64 + 2 * r, TH = 4 + 2 * r;
  float *ks = sh;
  float *t = sh + K * K;
  const int x0 = bx * 64, y0 = by * 4;
  for (int i = threadIdx.x; i < K * K; i += 256) ks[i] = Ks[i];
  for (int i = threadIdx.x; i < TW * TH; i += 256) {
    const int ty = i / TW, tx = i - ty * TW;
    const int y = y0 - r + ty, x = x0 - r + tx;
    float v = 1e18f;  // outside the image: (v - v0)^2 c underflows the weight to 0
    if (y >= 0 && y < H && x >= 0 && x < W) {
      const long long idx = (long long)y * W + x;
      v = U8 ? (float)static_cast<const uint8_t *>(I)[idx] : static_cast<const float *>(I)[idx];
    }
    t[i] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, row = threadIdx.x >> 6;
  const int x = x0 + lane, y = y0 + row;
  if (x >= W || y >= H) return;
  const float *base = t + row * TW + lane;  // window corner (dy = -r, dx = -r)
  const float v0 = base[r * TW + r];
  float nu = 0.0f, de = 0.0f;
  for (int dy = 0; dy < K; ++dy) {
    const float *rowp = base + dy * TW;
    const float *krow = ks + dy * K;
    for (int dx = 0; dx < K; ++dx) {
      const float v = rowp[dx];
      const float d = v - v0;
      const float w = krow[dx] * __builtin_amdgcn_exp2f(ABS ? c * __builtin_fabsf(d) : c * d * d);
      nu = __builtin_fmaf(w, v, nu);
      de += w;
    }
  }
  const long long idx = (long long)y * W + x;
  const float s = U8 ? 1.0f / 255.0f : 1.0f;
  out[idx] = nu / de * s;
  if (num_out) num_out[idx] = nu * s;
  if (den_out) den_out[idx] = de;
}

template <bool U8, bool ABS>
__global__ __launch_bounds__(256) void direct_bf(const void *__restrict__ I, int H, int W, int r,
                                                 const float *__restrict__ Ks, float c,
                                                 float *__restrict__ out, float *__restrict__ num_out,
                                                 float *__restrict__ den_out) {
  direct_body<U8, ABS>(I, H, W, r, Ks, c, out, num_out, den_out, blockIdx.x, blockIdx.y);
}

// Direct summation for the requests of a batch, one launch: a flat grid over
// every image's 64 x 4 blocks (image i owns blocks [start[i], start[i + 1])),
// the single-image body, so each output is bitwise its single-image call.
struct DirectImage {
  const void *I;
  float *out;
  const float *Ks;
  float c;
  int H, W, r;
};
struct DirectBatchArgs {
  int n;
  int start[kMaxBatch + 1];
  DirectImage img[kMaxBatch];
};

template <bool U8, bool ABS>
__global__ __launch_bounds__(256) void direct_batch(DirectBatchArgs a) {
  const int b = blockIdx.x;
  int i = 0;
  while (i + 1 < a.n && b >= a.start[i + 1]) ++i;
  const DirectImage &im = a.img[i];
  const int lb = b - a.start[i], bxs = (im.W + 63) / 64;
  direct_body<U8, ABS>(im.I, im.H, im.W, im.r, im.Ks, im.c, im.out, nullptr, nullptr, lb % bxs, lb / bxs);
}

// The direct-summation requests of a batch (host tables, inputs, outputs):
// one launch per input type and range kernel kind, at most kMaxBatch images each.
bf_status_t launch_direct_batch(const DevTables *const *host, const void *const *I, float *const *out,
                                const int *H, const int *W, int n, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int kind = 0; kind < 4; ++kind) {
    const bool u8 = kind & 1, abs_kind = kind & 2;
    DirectBatchArgs a{};
    size_t lds = 0;
    auto flush = [&]() -> bool {
      if (!a.n) return true;
      const int blocks = a.start[a.n];
      auto go = [&](auto kernel) {
        if (hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
          return false;
        hipLaunchKernelGGL(kernel, dim3(blocks), dim3(256), lds, s, a);
        return hipGetLastError() == hipSuccess;
      };
      const bool ok = u8 ? (abs_kind ? go(direct_batch<true, true>) : go(direct_batch<true, false>))
                         : (abs_kind ? go(direct_batch<false, true>) : go(direct_batch<false, false>));
      a = DirectBatchArgs{};
      lds = 0;
      return ok;
    };
    for (int j = 0; j < n; ++j) {
      const DevTables &h = *host[j];
      if ((h.in_u8 != 0) != u8 || (h.direct_abs != 0) != abs_kind) continue;
      const int r = h.direct_r, K = 2 * r + 1;
      DirectImage &im = a.img[a.n];
      im.I = I[j];
      im.out = out[j];
      im.Ks = h.direct_ks;
      im.c = h.direct_c;
      im.H = H[j];
      im.W = W[j];
      im.r = r;
      a.start[a.n + 1] = a.start[a.n] + ((W[j] + 63) / 64) * ((H[j] + 3) / 4);
      lds = std::max(lds, ((size_t)K * K + (size_t)(64 + 2 * r) * (4 + 2 * r)) * sizeof(float));
      if (++a.n == kMaxBatch && !flush()) return BF_ERR_DEVICE;
    }
    if (!flush()) return BF_ERR_DEVICE;
  }
  return BF_OK;
}

bf_status_t launch_direct(const DevTables &host, const void *I, float *out, float *num, float *den,
                          int H, int W, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int r = host.direct_r, K = 2 * r + 1;
  const size_t lds = ((size_t)K * K + (size_t)(64 + 2 * r) * (4 + 2 * r)) * sizeof(float);
  dim3 grid((W + 63) / 64, (H + 3) / 4), block(256);
  profile_mark(1, 1, stream);
  auto go = [&](auto kernel) {
    if (hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return false;
    hipLaunchKernelGGL(kernel, grid, block, lds, s, I, H, W, r, host.direct_ks, host.direct_c, out, num, den);
    return true;
  };
  bool ok;
  if (host.in_u8)
    ok = host.direct_abs ? go(direct_bf<true, true>) : go(direct_bf<true, false>);
  else
    ok = host.direct_abs ? go(direct_bf<false, true>) : go(direct_bf<false, false>);
  if (!ok) return BF_ERR_DEVICE;
  const hipError_t e = hipGetLastError();
  profile_mark(1, 0, stream);
  return e == hipSuccess ? BF_OK : BF_ERR_DEVICE;
}

// ---------------------------------------------------------------------------
// K-Z: the paper's own regime for 8-bit images (range series on [-T_r, T_r]
// times the range box, Eqs. 1D_box_N_terms / numerator_2D_box_N_terms).  A
// cube sum over a Haar rectangle and the level window [z_p - zr, z_p + zr] of
// the auxiliary volume F(y, z) = G(y) delta_{Z(y)}(z) is, for an output pixel
// of level L, the rectangle sum of the slab G(y) [|Z(y) - L| <= zr] (the
// sliding window over the promoted intensity axis).  For 8-bit input the
// output's modulation cos / sin(omega_k L) is fixed by L, so the range terms
// fold into one weight per level difference before the box sums:
//   num(p) = sum_rect w_rect sum_{y in rect} W(L - Z(y)) I(y),
//   den(p) = sum_rect w_rect sum_{y in rect} W(L - Z(y)),
//   W(d) = sum_k a_k cos(omega_k d / 255) [|d| <= zr]   (tabulated on the host),
// two tables per output level whatever the number of range terms.  One block
// per 32 x 32 output tile stages the levels of the region its taps read; for
// every level L among its outputs it builds both slab tables at once in LDS
// (int2 entries; row pass then column pass, each a DPP wave scan with int32
// wrapping adds of round(v 2^q)) and the pixels of level L read their
// quadruplet boxes.  No workspace.
// ---------------------------------------------------------------------------
// Output tiles of 64 x 64 (1024 threads) where their region fits in LDS, else
// 32 x 32 (512 threads); the region is at most 128 x 128 levels either way.
constexpr int kZMaxRegion = 128;
constexpr int kZPitch = kZMaxRegion + 2;

// Inclusive prefix sum within each 16-lane row of a wave (the first steps of
// wave_inclusive_scan).
__device__ __forceinline__ uint32_t row16_inclusive_scan(uint32_t v) {
  uint32_t x = v;
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true);   // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true);   // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x113, 0xf, 0xf, true);   // row_shr:3
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xe, false);  // row_shr:4, lanes 4..15 of a row
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xc, false);  // row_shr:8, lanes 8..15 of a row
  return x;
}

// One block of the regime: block blk of an image's tiles x nsplit blocks.
template <int kZTile, int kZThreads>
__device__ __forceinline__ void kz_body(const uint8_t *__restrict__ I, int H, int W,
                                        const DevTables *__restrict__ tab, int nsplit, float *__restrict__ out,
                                        float *__restrict__ num_out, float *__restrict__ den_out, int blk) {
  constexpr int kZWaves = kZThreads / 64;
  static_assert(kZWaves <= 16, "segment carries are scanned in 16-lane rows");
  constexpr int kZSeg = kZMaxRegion / kZWaves;      // region rows per wave
  constexpr int PPT = kZTile * kZTile / kZThreads;  // pixels per thread
  extern __shared__ int4 kz_lds4[];
  // two buffers of [264] (num, den) slab values by source level (the current
  // level's and the next one's); zero outside the level window and at 256
  // (sources outside the region)
  int2 *luts = reinterpret_cast<int2 *>(kz_lds4);
  uint32_t *mask = reinterpret_cast<uint32_t *>(luts + 2 * 264);    // 256 bits of output levels
  int2 *sat = reinterpret_cast<int2 *>(mask + 8);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tiles_x = (W + kZTile - 1) / kZTile;
  // nsplit blocks share a tile (small images): block part takes the tile's
  // levels part, part + nsplit, ...
  const int tile = blk / nsplit, part = blk - tile * nsplit;
  const int ty0 = (tile / tiles_x) * kZTile, tx0 = (tile % tiles_x) * kZTile;
  const int cy0 = min(max(ty0 + tab->tap_dy_min, 0), H), cy1 = min(max(ty0 + kZTile - 1 + tab->tap_dy_max, 0), H);
  const int cx0 = min(max(tx0 + tab->tap_dx_min, 0), W), cx1 = min(max(tx0 + kZTile - 1 + tab->tap_dx_max, 0), W);
  const int RS = cy1 - cy0, RC = cx1 - cx0;  // source rows / columns of the region (<= 128 each)
  const int P = kZPitch;                     // table pitch in int2: every lane's two columns fit
  int2 *tot = sat + (RS + 1) * P;            // [kZWaves][P]: column totals of each wave's segment
  int *start = reinterpret_cast<int *>(tot + kZWaves * P);  // [257]: first list slot per level
  int *cursor = start + 257;                                 // [256]
  int *levels = cursor + 256;                                // [256]: the output levels present
  uint16_t *list = reinterpret_cast<uint16_t *>(levels + 256);        // [kZTile^2]: tile pixels by level
  uint8_t *lv = reinterpret_cast<uint8_t *>(sat);  // the region's levels, staged before the tables exist
  const float scale = tab->box_scale;
  // wave w builds the region rows [w seg, (w + 1) seg) with sums restarting at
  // its first row; lane l holds the columns 2l, 2l + 1
  const int seg = (RS + kZWaves - 1) / kZWaves;
  const int ry0 = wave * seg, nrows = max(0, min(seg, RS - ry0));

  for (int i = tid; i < RS * RC; i += kZThreads) {
    const int y = i / RC, x = i - y * RC;
    lv[i] = I[(long long)(cy0 + y) * W + cx0 + x];
  }
  for (int i = tid; i < 257 + 256; i += kZThreads) start[i] = 0;  // start and cursor
  if (tid < 8) mask[tid] = 0;
  __syncthreads();
  // the wave's levels in registers as byte offsets into the slab values, two
  // columns per lane (level 256: outside the region)
  uint32_t zq[kZSeg];
#pragma unroll
  for (int i = 0; i < kZSeg; ++i) {
    const int y = ry0 + i, x = 2 * lane;
    const uint32_t a = (i < nrows && x < RC) ? lv[y * RC + x] : 256u;
    const uint32_t b = (i < nrows && x + 1 < RC) ? lv[y * RC + x + 1] : 256u;
    zq[i] = (a * 8u) | ((b * 8u) << 16);
  }
  int zp[PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int pi = tid + kZThreads * i;
    const int py = ty0 + pi / kZTile, px = tx0 + pi % kZTile;
    zp[i] = (py < H && px < W) ? (int)I[(long long)py * W + px] : -1;
    if (zp[i] >= 0) {
      atomicOr(&mask[zp[i] >> 5], 1u << (zp[i] & 31));
      atomicAdd(&cursor[zp[i]], 1);
    }
  }
  __syncthreads();  // the staged levels are in registers: the table rows may be cleared
  for (int x = tid; x < P; x += kZThreads) sat[x] = make_int2(0, 0);  // table row 0 and column 0 stay zero
  for (int y = tid; y <= RS; y += kZThreads) sat[y * P] = make_int2(0, 0);
  if (wave == 0) {  // exclusive prefix of the level counts and the list of levels: four per lane
    int c[4], t = 0, np = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      c[k] = cursor[4 * lane + k];
      t += c[k];
      np += c[k] > 0;
    }
    int e = (int)wave_inclusive_scan((uint32_t)t) - t;
    int el = (int)wave_inclusive_scan((uint32_t)np) - np;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      start[4 * lane + k] = e;
      cursor[4 * lane + k] = e;
      e += c[k];
      if (c[k] > 0) levels[el++] = 4 * lane + k;
    }
    if (lane == 63) start[256] = e;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PPT; ++i)
    if (zp[i] >= 0) list[atomicAdd(&cursor[zp[i]], 1)] = (uint16_t)(tid + kZThreads * i);
  int nlev = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) nlev += __builtin_popcount(mask[k]);
  nlev = __builtin_amdgcn_readfirstlane(nlev);

  // slab values of level L into buffer b, by the threads 0 .. 256
  auto fill_lut = [&](int L, int b) {
    int2 *lut = luts + 264 * b;
    if (tid < 256) {
      const int z = tid;
      const float w = tab->box_w[L - z + 255];  // zero outside the window
      lut[z] = make_int2(__float2int_rn(w * ((float)z * (1.0f / 255.0f)) * scale), __float2int_rn(w * scale));
    } else if (tid == 256) {
      lut[256] = make_int2(0, 0);
    }
  };
  if (part < nlev) fill_lut(__builtin_amdgcn_readfirstlane(levels[part]), 0);
  const int nq = tab->n_quads;
  for (int li = part, it = 0; li < nlev; li += nsplit, ++it) {
    __syncthreads();  // the lists, the level's slab values, the cleared tables; the last level's reads are done
    const int L = __builtin_amdgcn_readfirstlane(levels[li]);
    // the segment's slab values in registers and their column totals; each
    // segment's table starts from the totals of the segments above, so the
    // column sums run down the wave's rows and one row scan per row across
    // the lanes gives the table itself
    uint32_t an[kZSeg], ad[kZSeg], bn[kZSeg], bd[kZSeg];
    {
      const char *lb = reinterpret_cast<const char *>(luts + 264 * (it & 1));
      uint32_t s0n = 0, s0d = 0, s1n = 0, s1d = 0;
#pragma unroll
      for (int i = 0; i < kZSeg; ++i) {  // rows past the segment read the zero entry 256
        const int2 va = *reinterpret_cast<const int2 *>(lb + (zq[i] & 0xffffu));
        const int2 vb = *reinterpret_cast<const int2 *>(lb + (zq[i] >> 16));
        an[i] = (uint32_t)va.x;
        ad[i] = (uint32_t)va.y;
        bn[i] = (uint32_t)vb.x;
        bd[i] = (uint32_t)vb.y;
        s0n += an[i];
        s0d += ad[i];
        s1n += bn[i];
        s1d += bd[i];
      }
      tot[wave * P + 2 * lane] = make_int2((int)s0n, (int)s0d);
      tot[wave * P + 2 * lane + 1] = make_int2((int)s1n, (int)s1d);
    }
    __syncthreads();  // the totals are in
    {
      uint32_t c0n = 0, c0d = 0, c1n = 0, c1d = 0;
      for (int w = 0; w < wave; ++w) {
        const int2 ta = tot[w * P + 2 * lane], tb = tot[w * P + 2 * lane + 1];
        c0n += (uint32_t)ta.x;
        c0d += (uint32_t)ta.y;
        c1n += (uint32_t)tb.x;
        c1d += (uint32_t)tb.y;
      }
#pragma unroll
      for (int i = 0; i < kZSeg; ++i) {
        if (i < nrows) {  // wave-uniform
          c0n += an[i];
          c0d += ad[i];
          c1n += bn[i];
          c1d += bd[i];
          const uint32_t tn = c0n + c1n, td = c0d + c1d;
          const uint32_t en = wave_inclusive_scan(tn) - tn, ed = wave_inclusive_scan(td) - td;
          int2 *row = sat + (ry0 + i + 1) * P + 2 * lane + 1;  // columns past the region: padding
          row[0] = make_int2((int)(en + c0n), (int)(ed + c0d));
          row[1] = make_int2((int)(en + tn), (int)(ed + td));
        }
      }
    }
    // the next level's slab values go to the other buffer meanwhile
    if (li + nsplit < nlev) fill_lut(__builtin_amdgcn_readfirstlane(levels[li + nsplit]), (it + 1) & 1);
    __syncthreads();
    auto corner = [&](int Y, int X) -> int2 { return sat[Y * P + X]; };  // table entry (Y, X) of level L
    // the pixels of level L, one per thread
    const int s0 = start[L], cnt = start[L + 1] - s0;
    for (int j = tid; j < cnt; j += kZThreads) {
      const int pi = list[s0 + j];
      const int py = ty0 + pi / kZTile, px = tx0 + pi % kZTile;
      float num = 0.0f, den = 0.0f;
      for (int q = 0; q < nq; ++q) {
        const int dy = tab->quad_dy[q], dx = tab->quad_dx[q];
        const int Ya = min(max(py + dy, 0), H) - cy0, Yb = min(max(py + 1 - dy, 0), H) - cy0;
        const int Xa = min(max(px + dx, 0), W) - cx0, Xb = min(max(px + 1 - dx, 0), W) - cx0;
        const int2 a = corner(Ya, Xa), b = corner(Yb, Xa), c = corner(Ya, Xb), d = corner(Yb, Xb);
        const float w = tab->quad_w[q];
        num = __builtin_fmaf(w, (float)box_of(a.x, b.x, c.x, d.x), num);
        den = __builtin_fmaf(w, (float)box_of(a.y, b.y, c.y, d.y), den);
      }
      const float inv = 1.0f / scale;  // a power of two: exact
      num *= inv;
      den *= inv;
      const long long idx = (long long)py * W + px;
      out[idx] = den > tab->den_floor ? num / den : (float)L * (1.0f / 255.0f);
      if (num_out) num_out[idx] = num;
      if (den_out) den_out[idx] = den;
    }
  }
}

template <int kZTile, int kZThreads>
__global__ __launch_bounds__(kZThreads) void kz_rangebox(const uint8_t *__restrict__ I, int H, int W,
                                                         const DevTables *__restrict__ tab, int nsplit,
                                                         float *__restrict__ out, float *__restrict__ num_out,
                                                         float *__restrict__ den_out) {
  kz_body<kZTile, kZThreads>(I, H, W, tab, nsplit, out, num_out, den_out, blockIdx.x);
}

// The range-box requests of a batch in one launch per output-tile size: a
// flat grid over every image's blocks (image i owns [start[i], start[i + 1])),
// the single-image body, so each output is bitwise its single-image call.
struct ZImage {
  const uint8_t *I;
  float *out;
  const DevTables *tab;
  int H, W, nsplit;
};
struct ZBatchArgs {
  int n;
  int start[kMaxBatch + 1];
  ZImage img[kMaxBatch];
};

template <int kZTile, int kZThreads>
__global__ __launch_bounds__(kZThreads) void kz_batch(ZBatchArgs a) {
  const int b = blockIdx.x;
  int i = 0;
  while (i + 1 < a.n && b >= a.start[i + 1]) ++i;
  const ZImage &im = a.img[i];
  kz_body<kZTile, kZThreads>(im.I, im.H, im.W, im.tab, im.nsplit, im.out, nullptr, nullptr, b - a.start[i]);
}

template <int TE, int NT>
static size_t rangebox_lds(const DevTables &host) {
  const int RS = TE - 1 + host.tap_dy_max - host.tap_dy_min;  // largest region
  const int RC = TE - 1 + host.tap_dx_max - host.tap_dx_min;
  if (RS > kZMaxRegion || RC > kZMaxRegion) return (size_t)-1;
  const int P = kZPitch;
  const size_t lists = (257 + 256 + 256) * 4 + TE * TE * 2;
  // the staged levels (RS x RC bytes) share the bytes of the tables
  return 2 * 264 * 8 + 32 + (size_t)(RS + 1) * P * 8 + (size_t)(NT / 64) * P * 8 + lists;
}

constexpr size_t kLdsLimit = 160 * 1024;

size_t rangebox_lds_bytes(const DevTables &host) {
  const size_t a = rangebox_lds<64, 1024>(host);
  return a <= kLdsLimit ? a : rangebox_lds<32, 512>(host);
}

int rangebox_tile(const DevTables &host) {
  if (rangebox_lds<64, 1024>(host) <= kLdsLimit) return 64;
  return rangebox_lds<32, 512>(host) <= kLdsLimit ? 32 : 0;
}

bf_status_t launch_rangebox(const DevTables *dev, const DevTables &host, const void *I, float *out, float *num,
                            float *den, int H, int W, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t l64 = rangebox_lds<64, 1024>(host), l32 = rangebox_lds<32, 512>(host);
  const bool big = l64 <= kLdsLimit;
  const size_t lds = big ? l64 : l32;
  if (lds > kLdsLimit) return BF_ERR_UNSUPPORTED;
  const int te = big ? 64 : 32;
  const int tiles = ((W + te - 1) / te) * ((H + te - 1) / te);
  const int nsplit = std::max(1, std::min(8, 1024 / tiles));  // small images: several blocks per tile
  const int blocks = tiles * nsplit;
  const void *fn = big ? (const void *)kz_rangebox<64, 1024> : (const void *)kz_rangebox<32, 512>;
  profile_mark(1, 1, stream);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return BF_ERR_DEVICE;
  if (big)
    hipLaunchKernelGGL((kz_rangebox<64, 1024>), dim3(blocks), dim3(1024), lds, s, static_cast<const uint8_t *>(I),
                       H, W, dev, nsplit, out, num, den);
  else
    hipLaunchKernelGGL((kz_rangebox<32, 512>), dim3(blocks), dim3(512), lds, s, static_cast<const uint8_t *>(I),
                       H, W, dev, nsplit, out, num, den);
  const hipError_t e = hipGetLastError();
  profile_mark(1, 0, stream);
  return e == hipSuccess ? BF_OK : BF_ERR_DEVICE;
}

// The range-box requests of a batch (device and host tables, inputs,
// outputs): one launch per output-tile size, at most kMaxBatch images each;
// each image split as its single-image call splits it.
bf_status_t launch_rangebox_batch(const DevTables *const *dev, const DevTables *const *host, const void *const *I,
                                  float *const *out, const int *H, const int *W, int n, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int big = 1; big >= 0; --big) {
    ZBatchArgs a{};
    size_t lds = 0;
    auto flush = [&]() -> bool {
      if (!a.n) return true;
      const void *fn = big ? (const void *)kz_batch<64, 1024> : (const void *)kz_batch<32, 512>;
      if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return false;
      if (big)
        hipLaunchKernelGGL((kz_batch<64, 1024>), dim3(a.start[a.n]), dim3(1024), lds, s, a);
      else
        hipLaunchKernelGGL((kz_batch<32, 512>), dim3(a.start[a.n]), dim3(512), lds, s, a);
      a = ZBatchArgs{};
      lds = 0;
      return hipGetLastError() == hipSuccess;
    };
    for (int j = 0; j < n; ++j) {
      const size_t l64 = rangebox_lds<64, 1024>(*host[j]), l32 = rangebox_lds<32, 512>(*host[j]);
      const bool b = l64 <= kLdsLimit;
      if (b != (big != 0)) continue;
      const size_t l = b ? l64 : l32;
      if (l > kLdsLimit) return BF_ERR_UNSUPPORTED;
      const int te = b ? 64 : 32;
      const int tiles = ((W[j] + te - 1) / te) * ((H[j] + te - 1) / te);
      ZImage &im = a.img[a.n];
      im.I = static_cast<const uint8_t *>(I[j]);
      im.out = out[j];
      im.tab = dev[j];
      im.H = H[j];
      im.W = W[j];
      im.nsplit = std::max(1, std::min(8, 1024 / tiles));
      a.start[a.n + 1] = a.start[a.n] + tiles * im.nsplit;
      lds = std::max(lds, l);
      if (++a.n == kMaxBatch && !flush()) return BF_ERR_DEVICE;
    }
    if (!flush()) return BF_ERR_DEVICE;
  }
  return BF_OK;
}

// ---------------------------------------------------------------------------
// Reduced precision: the term images C I, S I, C, S (I alone for k = 0; the
// byte itself for 8-bit input, exact in FP16) are stored once in FP16,
// [table][H][W] with no halo copies, half the bytes of an int32 value.  The
// lookup kernel then builds each table of its output tile in LDS from them:
// the region's values, rounded to round(v 2^q) in int32, summed by column
// in registers down each wave's row segment with one DPP row scan per row,
// each segment starting from the column totals of the segments above (two
// barriers per table), and the box sums and fold of the plain lookup.  The next table's values are loaded while the current one
// is read.  Out-of-image values are zero, so the table's corners need no clamp.
// ---------------------------------------------------------------------------
template <bool U8>
__device__ __forceinline__ void kr_modulate_body(const void *__restrict__ I, int H, int W,
                                                 const DevTables *__restrict__ tab, _Float16 *__restrict__ img,
                                                 int blk) {
  const long long n = (long long)H * W;
  const long long idx = (long long)blk * 256 + threadIdx.x;
  if (idx >= n) return;
  float px, v;
  load_pixel<U8>(I, idx, &px, &v);
  for (int t = 0; t < tab->n_terms; ++t) {
    _Float16 *dst = img + (long long)tab->slot[t] * n + idx;
    if (tab->k_is_zero[t]) {
      dst[0] = (_Float16)(U8 ? px : v);
      continue;
    }
    const float fr = phase_rev(tab->f_hi[t], tab->f_lo[t], px);
    const float C = __builtin_amdgcn_cosf(fr), S = __builtin_amdgcn_sinf(fr);
    dst[0] = (_Float16)(C * v);
    dst[n] = (_Float16)(S * v);
    dst[2 * n] = (_Float16)C;
    dst[3 * n] = (_Float16)S;
  }
}

template <bool U8>
__global__ __launch_bounds__(256) void kr_modulate(const void *__restrict__ I, int H, int W,
                                                   const DevTables *__restrict__ tab,
                                                   _Float16 *__restrict__ img) {
  kr_modulate_body<U8>(I, H, W, tab, img, blockIdx.x);
}

// One TE x TE output tile (index blk) of one image.
template <int TE, int NT, int NQ, bool U8>
__device__ __forceinline__ void kr_body(const void *__restrict__ I, int H, int W, const DevTables *__restrict__ tab,
                                        const _Float16 *__restrict__ img, float scale, float inv_scale,
                                        float *__restrict__ out, float *__restrict__ num_out,
                                        float *__restrict__ den_out, int blk) {
  constexpr int NW = NT / 64;              // waves: one row segment each
  static_assert(NW <= 16, "segment carries are scanned in 16-lane rows");
  constexpr int SEGMAX = kZMaxRegion / NW;  // rows per segment
  constexpr int PPT = TE * TE / NT;        // pixels per thread
  constexpr int RSTEP = NT / TE;           // tile rows between a thread's pixels
  constexpr int P = kZPitch;               // table pitch (int32): every lane's two columns fit
  extern __shared__ int kr_lds[];
  uint32_t *tot = reinterpret_cast<uint32_t *>(kr_lds);  // [NW][P]: column totals of each wave's segment
  int *sat = kr_lds + NW * P;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tiles_x = (W + TE - 1) / TE;
  const int ty0 = (blk / tiles_x) * TE, tx0 = (blk % tiles_x) * TE;
  const int dy0 = tab->tap_dy_min, dx0 = tab->tap_dx_min;
  const int Y0 = ty0 + dy0, X0 = tx0 + dx0;  // image position of table corner (0, 0)
  const int RS = TE - 1 + tab->tap_dy_max - dy0, RC = TE - 1 + tab->tap_dx_max - dx0;  // <= 128 each
  const long long npx = (long long)H * W;
  const int seg = (RS + NW - 1) / NW;
  const int ry0 = wave * seg, nrows = max(0, min(seg, RS - ry0));
  const int xs0 = X0 + 2 * lane, xs1 = xs0 + 1;  // this lane's source columns
  const bool c0ok = 2 * lane < RC && xs0 >= 0 && xs0 < W;
  const bool c1ok = 2 * lane + 1 < RC && xs1 >= 0 && xs1 < W;

  for (int x = tid; x < P; x += NT) sat[x] = 0;  // table row 0 and column 0 stay zero
  for (int y = tid; y <= RS; y += NT) sat[y * P] = 0;

  _Float16 h0[SEGMAX], h1[SEGMAX];
  auto load = [&](int m) {
    const _Float16 *base = img + (long long)m * npx;
#pragma unroll
    for (int i = 0; i < SEGMAX; ++i) {
      const int y = Y0 + ry0 + i;
      const bool rok = i < nrows && y >= 0 && y < H;
      h0[i] = (rok && c0ok) ? base[(long long)y * W + xs0] : (_Float16)0.0f;
      h1[i] = (rok && c1ok) ? base[(long long)y * W + xs1] : (_Float16)0.0f;
    }
  };

  // the thread's pixels: tile row prow + RSTEP i, column pcol; table corner
  // (y + dy - Y0, x + dx - X0) of tap (dy, dx)
  const int prow = tid / TE, pcol = tid % TE;
  const uint32_t lb = (uint32_t)(prow * P + pcol);
  const int nq = tab->n_quads;
  uint32_t qa[NQ][4];
  float qw[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (q < nq) {
      const int dy = tab->quad_dy[q], dx = tab->quad_dx[q];
      const int ra = dy - dy0, rb = 1 - dy - dy0, ca = dx - dx0, cb = 1 - dx - dx0;
      qa[q][0] = (lb + (uint32_t)(ra * P + ca)) * 4u;
      qa[q][1] = (lb + (uint32_t)(rb * P + ca)) * 4u;
      qa[q][2] = (lb + (uint32_t)(ra * P + cb)) * 4u;
      qa[q][3] = (lb + (uint32_t)(rb * P + cb)) * 4u;
      qw[q] = tab->quad_w[q];
    } else {
      qa[q][0] = qa[q][1] = qa[q][2] = qa[q][3] = lb * 4u;
      qw[q] = 0.0f;
    }
  }
  float pxv[PPT], cs[PPT], sn[PPT];
  float num[PPT], den[PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    cs[i] = sn[i] = 0.0f;
    const int y = ty0 + prow + RSTEP * i, x = tx0 + pcol;
    pxv[i] = 0.0f;
    if (y < H && x < W) {
      float px, v;
      load_pixel<U8>(I, (long long)y * W + x, &px, &v);
      pxv[i] = px;
    }
    num[i] = 0.0f;
    den[i] = 0.0f;
    cs[i] = sn[i] = 0.0f;
  }

  const int n = tab->n_images;
  load(0);
  for (int m = 0; m < n; ++m) {
    const int part = tab->slot_part[m];
    const float fhi = tab->slot_fhi[m], flo = tab->slot_flo[m];
    const float at = tab->slot_a[m];
    const float sc = (U8 && part == 4) ? 1.0f : scale;  // 8-bit k = 0: exact byte sums
    // the segment's fixed-point values and their column totals; the totals of
    // the segments above are the columns' carry into this segment
    uint32_t v0[SEGMAX], v1[SEGMAX], s0 = 0, s1 = 0;
#pragma unroll
    for (int i = 0; i < SEGMAX; ++i) {
      v0[i] = (uint32_t)__float2int_rn((float)h0[i] * sc);  // zero outside the segment and the image
      v1[i] = (uint32_t)__float2int_rn((float)h1[i] * sc);
      s0 += v0[i];
      s1 += v1[i];
    }
    tot[wave * P + 2 * lane] = s0;
    tot[wave * P + 2 * lane + 1] = s1;
    __syncthreads();  // the totals are in, and the previous table's reads are done
    {
      uint32_t c0 = 0, c1 = 0;
      for (int w = 0; w < wave; ++w) {
        c0 += tot[w * P + 2 * lane];
        c1 += tot[w * P + 2 * lane + 1];
      }
#pragma unroll
      for (int i = 0; i < SEGMAX; ++i) {
        if (i < nrows) {  // wave-uniform
          c0 += v0[i];
          c1 += v1[i];
          const uint32_t tt = c0 + c1;
          const uint32_t e = wave_inclusive_scan(tt) - tt;
          int *row = sat + (ry0 + i + 1) * P + 2 * lane + 1;  // columns past the region: padding
          row[0] = (int)(e + c0);
          row[1] = (int)(e + tt);
        }
      }
    }
    if (m + 1 < n) load(m + 1);  // in flight during the lookups
    __syncthreads();
    if (part == 0) {
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        const float fr = phase_rev(fhi, flo, pxv[i]);
        cs[i] = __builtin_amdgcn_cosf(fr);
        sn[i] = __builtin_amdgcn_sinf(fr);
      }
    }
    float sv[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) sv[i] = 0.0f;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
      for (int i = 0; i < PPT; ++i) {
        const uint32_t o = i * RSTEP * P * 4u;
        const int box = box_of(lds_ld(sat, qa[q][0] + o), lds_ld(sat, qa[q][1] + o),
                               lds_ld(sat, qa[q][2] + o), lds_ld(sat, qa[q][3] + o));
        sv[i] = __builtin_fmaf(qw[q], (float)box, sv[i]);
      }
    }
    const float ai = at * (U8 && part == 4 ? 1.0f / 255.0f : inv_scale);
    float an, ad;
    fold_weights(part, ai, &an, &ad);
#pragma unroll
    for (int i = 0; i < PPT; ++i) fold_table(part, an, ad, cs[i], sn[i], sv[i], num[i], den[i]);
    if (part == 4) {
      // denominator of the k = 0 term (table of ones)
#pragma unroll
      for (int i = 0; i < PPT; ++i)
        den[i] = __builtin_fmaf(at, k0_denominator(tab, ty0 + prow + RSTEP * i, tx0 + pcol, H, W), den[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int y = ty0 + prow + RSTEP * i, x = tx0 + pcol;
    if (y >= H || x >= W) continue;
    const long long idx = (long long)y * W + x;
    const float xv = U8 ? pxv[i] * (1.0f / 255.0f) : pxv[i];
    out[idx] = den[i] > tab->den_floor ? num[i] / den[i] : xv;
    if (num_out) num_out[idx] = num[i];
    if (den_out) den_out[idx] = den[i];
  }
}

// 32 x 32 output tiles (512 threads, two pixels each): 64 x 64 tiles with four
// pixels per thread exceed 128 registers and spill.
template <int TE, int NT, int NQ, bool U8>
__global__ __launch_bounds__(NT) void kr_tile(const void *__restrict__ I, int H, int W,
                                              const DevTables *__restrict__ tab,
                                              const _Float16 *__restrict__ img, float scale, float inv_scale,
                                              float *__restrict__ out, float *__restrict__ num_out,
                                              float *__restrict__ den_out) {
  kr_body<TE, NT, NQ, U8>(I, H, W, tab, img, scale, inv_scale, out, num_out, den_out, blockIdx.x);
}

// The reduced-precision requests of a batch: one modulation launch and one
// table-and-lookup launch per input type, flat grids over the images' blocks
// (image i owns [mstart[i], mstart[i + 1]) and [tstart[i], tstart[i + 1])),
// the single-image bodies, so each output is bitwise its single-image call.
struct RImage {
  const void *I;
  float *out;
  const DevTables *tab;
  _Float16 *img;
  float scale, inv;
  int H, W;
};
struct RBatchArgs {
  int n;
  int mstart[kMaxBatch + 1], tstart[kMaxBatch + 1];
  RImage im[kMaxBatch];
};

template <bool U8>
__global__ __launch_bounds__(256) void kr_modulate_batch(RBatchArgs a) {
  const int b = blockIdx.x;
  int i = 0;
  while (i + 1 < a.n && b >= a.mstart[i + 1]) ++i;
  const RImage &m = a.im[i];
  kr_modulate_body<U8>(m.I, m.H, m.W, m.tab, m.img, b - a.mstart[i]);
}

template <int TE, int NT, int NQ, bool U8>
__global__ __launch_bounds__(NT) void kr_tile_batch(RBatchArgs a) {
  const int b = blockIdx.x;
  int i = 0;
  while (i + 1 < a.n && b >= a.tstart[i + 1]) ++i;
  const RImage &m = a.im[i];
  kr_body<TE, NT, NQ, U8>(m.I, m.H, m.W, m.tab, m.img, m.scale, m.inv, m.out, nullptr, nullptr, b - a.tstart[i]);
}

int reduced_tile(const DevTables &host) {
  if (31 + host.tap_dy_max - host.tap_dy_min <= kZMaxRegion && 31 + host.tap_dx_max - host.tap_dx_min <= kZMaxRegion)
    return 32;
  return 0;
}

size_t reduced_workspace_bytes(const DevTables &host, int H, int W) {
  return ((size_t)host.n_images * H * W * sizeof(_Float16) + 255) / 256 * 256;
}

template <int TE, int NT, bool U8>
static hipError_t launch_kr_nq(int nq, dim3 grid, size_t lds, hipStream_t s, const void *I, int H, int W,
                               const DevTables *dev, const _Float16 *img, float scale, float inv, float *out,
                               float *num, float *den) {
  auto go = [&](auto k) {
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, grid, dim3(NT), lds, s, I, H, W, dev, img, scale, inv, out, num, den);
    return hipGetLastError();
  };
  if (nq <= 4) return go(kr_tile<TE, NT, 4, U8>);
  if (nq <= 8) return go(kr_tile<TE, NT, 8, U8>);
  return go(kr_tile<TE, NT, 12, U8>);
}

bf_status_t launch_reduced(const DevTables *dev, const DevTables &host, const Geometry &g, const void *I,
                           float *out, float *num, float *den, void *ws, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int te = reduced_tile(host);
  if (te == 0 || host.n_quads > 12) return BF_ERR_UNSUPPORTED;
  const int RS = te - 1 + host.tap_dy_max - host.tap_dy_min;
  const size_t lds = (size_t)(RS + 1 + 512 / 64) * kZPitch * 4;  // table and the waves' column totals
  _Float16 *img = static_cast<_Float16 *>(ws);
  const long long npx = (long long)g.H * g.W;
  profile_mark(0, 1, stream);
  hipError_t e;
  const unsigned blocks_m = (unsigned)((npx + 255) / 256);
  if (host.in_u8)
    hipLaunchKernelGGL((kr_modulate<true>), dim3(blocks_m), dim3(256), 0, s, I, g.H, g.W, dev, img);
  else
    hipLaunchKernelGGL((kr_modulate<false>), dim3(blocks_m), dim3(256), 0, s, I, g.H, g.W, dev, img);
  e = hipGetLastError();
  profile_mark(0, 0, stream);
  if (e != hipSuccess) return BF_ERR_DEVICE;
  const float scale = std::ldexp(1.0f, g.sat_shift);
  const float inv = std::ldexp(1.0f, -g.sat_shift);
  const dim3 grid(((g.W + te - 1) / te) * ((g.H + te - 1) / te));
  profile_mark(1, 1, stream);
  e = host.in_u8 ? launch_kr_nq<32, 512, true>(host.n_quads, grid, lds, s, I, g.H, g.W, dev, img, scale, inv, out, num, den)
                 : launch_kr_nq<32, 512, false>(host.n_quads, grid, lds, s, I, g.H, g.W, dev, img, scale, inv, out, num, den);
  profile_mark(1, 0, stream);
  return e == hipSuccess ? BF_OK : BF_ERR_DEVICE;
}

template <bool U8>
static hipError_t launch_reduced_group(const RBatchArgs &a, int nq, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL((kr_modulate_batch<U8>), dim3(a.mstart[a.n]), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  auto go = [&](auto k) {
    hipError_t e2 = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e2 != hipSuccess) return e2;
    hipLaunchKernelGGL(k, dim3(a.tstart[a.n]), dim3(512), lds, s, a);
    return hipGetLastError();
  };
  if (nq <= 4) return go(kr_tile_batch<32, 512, 4, U8>);
  if (nq <= 8) return go(kr_tile_batch<32, 512, 8, U8>);
  return go(kr_tile_batch<32, 512, 12, U8>);
}

// The reduced-precision requests of a batch (their geometries and FP16
// workspaces): one pair of launches per input type, at most kMaxBatch images.
bf_status_t launch_reduced_batch(const DevTables *const *dev, const DevTables *const *host, const Geometry *g,
                                 const void *const *I, float *const *out, void *const *ws, int n, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int u8 = 0; u8 < 2; ++u8) {
    RBatchArgs a{};
    size_t lds = 0;
    int nq = 0;
    auto flush = [&]() -> bool {
      if (!a.n) return true;
      const hipError_t e = u8 ? launch_reduced_group<true>(a, nq, lds, s) : launch_reduced_group<false>(a, nq, lds, s);
      a = RBatchArgs{};
      lds = 0;
      nq = 0;
      return e == hipSuccess;
    };
    for (int j = 0; j < n; ++j) {
      const DevTables &h = *host[j];
      if ((h.in_u8 != 0) != (u8 != 0)) continue;
      const int te = reduced_tile(h);
      if (te == 0 || h.n_quads > 12) return BF_ERR_UNSUPPORTED;
      const int RS = te - 1 + h.tap_dy_max - h.tap_dy_min;
      RImage &m = a.im[a.n];
      m.I = I[j];
      m.out = out[j];
      m.tab = dev[j];
      m.img = static_cast<_Float16 *>(ws[j]);
      m.scale = std::ldexp(1.0f, g[j].sat_shift);
      m.inv = std::ldexp(1.0f, -g[j].sat_shift);
      m.H = g[j].H;
      m.W = g[j].W;
      const long long npx = (long long)m.H * m.W;
      a.mstart[a.n + 1] = a.mstart[a.n] + (int)((npx + 255) / 256);
      a.tstart[a.n + 1] = a.tstart[a.n] + ((m.W + te - 1) / te) * ((m.H + te - 1) / te);
      lds = std::max(lds, (size_t)(RS + 1 + 512 / 64) * kZPitch * 4);
      nq = std::max(nq, h.n_quads);
      if (++a.n == kMaxBatch && !flush()) return BF_ERR_DEVICE;
    }
    if (!flush()) return BF_ERR_DEVICE;
  }
  return BF_OK;
}

// ---------------------------------------------------------------------------
// Batches: every image of a batch runs in one launch per kernel.  The
// per-image descriptors travel by value in the kernel arguments (nothing to
// allocate, copy or keep alive, so a batch can be captured in a graph).
// K-A: one flat grid over all images' (tile, term group) blocks.  K-B: a
// persistent grid of one block per CU with 8 work queues, one per XCD: queue
// k holds, image after image, the k-th eighth of each image's tiles in the
// XCD-aware order, so an XCD keeps working on neighbouring tiles; a block
// drains its own XCD's queue, then takes from the others, and exits when all
// eight are empty.  The queue heads live in the workspace and are zeroed by
// the K-A launch that precedes every K-B launch on the stream.  Both launches
// run the same per-image bodies as the single-image kernels, so every output
// is bitwise the one a single-image call produces.
// ---------------------------------------------------------------------------
struct BatchImage {
  const void *I;
  float *out;
  const int32_t *ws;
  const DevTables *tab;
  int ka_blocks;  // tiles * term groups
  int n_tiles;    // 64 x 64 output tiles
  int per_xcd;    // ceil(n_tiles / 8)
  ImageParams p;
};

struct BatchArgs {
  int n;
  uint32_t *heads;  // 8 queue heads per lookup launch class (kBatchQueues in all)
  int ka_start[kMaxBatch + 1];
  BatchImage img[kMaxBatch];
};

template <int G, bool U8, bool ONE>
__global__ __launch_bounds__(256) void ka_batch(BatchArgs a) {
  if (blockIdx.x == 0 && threadIdx.x < kBatchQueues) a.heads[threadIdx.x] = 0u;  // every lookup class x 8 queues
  const int b = blockIdx.x;
  int i = 0;
  while (i + 1 < a.n && b >= a.ka_start[i + 1]) ++i;
  const BatchImage &im = a.img[i];
  const int lb = b - a.ka_start[i];
  const int tiles = im.p.tiles_x * ((im.p.H + im.p.tile - 1) / im.p.tile);
  ka_body<G, U8, ONE>(im.I, im.p, im.tab, const_cast<int32_t *>(im.ws), lb % tiles, lb / tiles);
}

template <int PITCH, int NQ, int ST, bool U8>
__global__ __launch_bounds__(1024) void kb_batch(BatchArgs a) {
  __shared__ int item_sh;
  int q = blockIdx.x & 7;
  for (int exhausted = 0; exhausted < 8;) {
    __syncthreads();  // the previous tile is done with LDS and item_sh
    if (threadIdx.x == 0) item_sh = (int)atomicAdd(&a.heads[q], 1u);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(item_sh);
    int found = -1, L = 0, base = 0;
    for (int i = 0; i < a.n; ++i) {
      const int c = min(max(a.img[i].n_tiles - q * a.img[i].per_xcd, 0), a.img[i].per_xcd);
      if (item < base + c) {
        found = i;
        L = q * a.img[i].per_xcd + (item - base);
        break;
      }
      base += c;
    }
    if (found < 0) {  // queue q is empty: move on to the next XCD's queue
      q = (q + 1) & 7;
      ++exhausted;
      continue;
    }
    const BatchImage &im = a.img[found];
    kb_body<PITCH, NQ, ST, U8>(im.I, im.p, im.tab, im.ws, im.out, nullptr, nullptr, L);
  }
}

// ---------------------------------------------------------------------------
// Fused batch: one persistent launch runs a batch's table building (phase A)
// and its lookups (phase B).  Phase-A items are (image, table tile, 16 table
// units -- range terms, or tables with ONE -- one per wave), from one queue
// in image and tile order; phase-B items are 64 x 64 output tiles, from 8
// per-XCD queues as in the batched lookup.  A block takes phase-A items until
// their queue is empty, then phase-B items.  An output tile needs every table
// of its table tile: each phase-A item publishes its tables (a release at
// device scope) and then counts itself in its table tile's ready counter; a
// phase-B item waits until that counter holds the tile's item count, then
// acquires at device scope before it reads.  Every phase-A item has been
// taken before any block waits, by a block that is running, so every wait
// ends; the wait is bounded all the same (kReadySpin rounds), and one that
// runs out sets the batch's error word and goes on.
// ---------------------------------------------------------------------------
constexpr int kReadySpin = 1 << 22;
constexpr int kFusedUnits = 16;  // table units (range terms, or tables) per phase-A item: one per wave

struct FusedArgs {
  int n;
  uint32_t *ctl;                // [0] phase-A queue, [1 .. 8] phase-B queues, [9] error word
  int a_start[kMaxBatch + 1];   // phase-A items before image i
  int groups[kMaxBatch];        // phase-A items per table tile
  int db[kMaxBatch];            // 1: the double-buffered lookup body (pitch 128), 0: overlap-staged (176)
  uint32_t *ready[kMaxBatch];   // per table tile: its phase-A items done
  BatchImage img[kMaxBatch];
};

__global__ __launch_bounds__(256) void kf_reset(FusedArgs a) {
  if (threadIdx.x < 10) a.ctl[threadIdx.x] = 0u;
  for (int i = 0; i < a.n; ++i) {
    const int tiles = a.img[i].p.tiles_x * ((a.img[i].p.H + a.img[i].p.tile - 1) / a.img[i].p.tile);
    for (int t = threadIdx.x; t < tiles; t += blockDim.x) a.ready[i][t] = 0u;
  }
}

template <int NQ, bool U8, int G, bool ONE>
__global__ __launch_bounds__(1024) void kf_batch(FusedArgs a) {
  __shared__ int item_sh;
  const int n_a = a.a_start[a.n];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (;;) {
    __syncthreads();  // the previous item is done with LDS and item_sh
    if (threadIdx.x == 0) item_sh = (int)atomicAdd(&a.ctl[0], 1u);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(item_sh);
    if (item >= n_a) break;
    int i = 0;
    while (i + 1 < a.n && item >= a.a_start[i + 1]) ++i;
    const BatchImage &im = a.img[i];
    const int lb = item - a.a_start[i];
    const int tile = lb / a.groups[i], grp = lb - tile * a.groups[i];
    const int unit = grp * kFusedUnits + wave;
    if (unit < (ONE ? im.p.n_images : im.p.n_terms))
      ka_unit<G, U8, ONE, true>(im.I, im.p, im.tab, const_cast<int32_t *>(im.ws), tile, unit);
    // every wave's table stores are done (the barrier waits for them); one
    // release makes them visible to the device, then the item is counted
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(a.ready[i] + tile, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  int q = blockIdx.x & 7;
  for (int exhausted = 0; exhausted < 8;) {
    __syncthreads();
    if (threadIdx.x == 0) item_sh = (int)atomicAdd(&a.ctl[1 + q], 1u);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(item_sh);
    int found = -1, L = 0, base = 0;
    for (int i = 0; i < a.n; ++i) {
      const int c = min(max(a.img[i].n_tiles - q * a.img[i].per_xcd, 0), a.img[i].per_xcd);
      if (item < base + c) {
        found = i;
        L = q * a.img[i].per_xcd + (item - base);
        break;
      }
      base += c;
    }
    if (found < 0) {  // queue q is empty: move on to the next XCD's queue
      q = (q + 1) & 7;
      ++exhausted;
      continue;
    }
    const BatchImage &im = a.img[found];
    int y0, x0;
    kb_tile_origin(L, im.p.H, im.p.W, &y0, &x0);
    const uint32_t *rdy = a.ready[found] + (y0 / im.p.tile) * im.p.tiles_x + x0 / im.p.tile;
    const uint32_t need = (uint32_t)a.groups[found];
    // every wave waits itself, so that its acquire follows its own read of the count
    for (int k = 0;; ++k) {
      if (__hip_atomic_load(rdy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= need) break;
      if (k == kReadySpin) {
        atomicOr(&a.ctl[9], 1u);  // every lane: no branch on the lane inside the loop
        break;
      }
      __builtin_amdgcn_s_sleep(4);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (a.db[found])
      kb_body<128, NQ, kStageDouble, U8>(im.I, im.p, im.tab, im.ws, im.out, nullptr, nullptr, L);
    else
      kb_body<176, NQ, kStageOverlap, U8>(im.I, im.p, im.tab, im.ws, im.out, nullptr, nullptr, L);
  }
}

// The lattice lookup kernel over a batch: as kb_batch, for the images of one
// (pitch, M, N) class (each with its own lattice step and tile grid).
template <int PITCH, int M, int N, bool U8>
__global__ __launch_bounds__(1024) void kl_batch(BatchArgs a) {
  __shared__ int item_sh;
  int q = blockIdx.x & 7;
  for (int exhausted = 0; exhausted < 8;) {
    __syncthreads();  // the previous tile is done with LDS and item_sh
    if (threadIdx.x == 0) item_sh = (int)atomicAdd(&a.heads[q], 1u);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(item_sh);
    int found = -1, L = 0, base = 0;
    for (int i = 0; i < a.n; ++i) {
      const int c = min(max(a.img[i].n_tiles - q * a.img[i].per_xcd, 0), a.img[i].per_xcd);
      if (item < base + c) {
        found = i;
        L = q * a.img[i].per_xcd + (item - base);
        break;
      }
      base += c;
    }
    if (found < 0) {  // queue q is empty: move on to the next XCD's queue
      q = (q + 1) & 7;
      ++exhausted;
      continue;
    }
    const BatchImage &im = a.img[found];
    kl_body<PITCH, M, N, U8>(im.I, im.p, im.tab, im.ws, im.out, nullptr, nullptr, L);
  }
}

// ---------------------------------------------------------------------------
// Workspace of the allocation-free entry point: a file-scope device array
// that every GPU the library runs on holds from module load to process end.
// In host code `scratch` is only a stand-in for the symbol; its device
// address on each GPU comes from hipGetSymbolAddress, taken once per device
// with that device current and kept, and only that address is handed to
// kernels.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

bf_status_t scratch_workspace(void **ptr) {
  static std::mutex mu;
  static std::vector<void *> per_device;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return BF_ERR_DEVICE;
  std::lock_guard<std::mutex> lk(mu);
  if ((size_t)dev >= per_device.size()) per_device.resize((size_t)dev + 1, nullptr);
  if (!per_device[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BF_ERR_DEVICE;
    per_device[dev] = p;
  }
  *ptr = per_device[dev];
  return BF_OK;
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <bool U8, bool ONE>
static hipError_t launch_ka1(int G, dim3 grid, dim3 block, hipStream_t s, const void *I,
                             ImageParams p, const DevTables *tab, int32_t *ws) {
  switch (G) {
    case 1: hipLaunchKernelGGL((ka_sat<1, U8, ONE>), grid, block, 0, s, I, p, tab, ws); break;
    case 2: hipLaunchKernelGGL((ka_sat<2, U8, ONE>), grid, block, 0, s, I, p, tab, ws); break;
    case 3: hipLaunchKernelGGL((ka_sat<3, U8, ONE>), grid, block, 0, s, I, p, tab, ws); break;
    case 4: hipLaunchKernelGGL((ka_sat<4, U8, ONE>), grid, block, 0, s, I, p, tab, ws); break;
    case 5: hipLaunchKernelGGL((ka_sat<5, U8, ONE>), grid, block, 0, s, I, p, tab, ws); break;
    case 6: hipLaunchKernelGGL((ka_sat<6, U8, ONE>), grid, block, 0, s, I, p, tab, ws); break;
    case 7: hipLaunchKernelGGL((ka_sat<7, U8, ONE>), grid, block, 0, s, I, p, tab, ws); break;
    default: hipLaunchKernelGGL((ka_sat<8, U8, ONE>), grid, block, 0, s, I, p, tab, ws); break;
  }
  return hipGetLastError();
}

// the pair form, for table rows of up to 4 chunks
template <bool U8>
static hipError_t launch_ka_pair(int G, dim3 grid, dim3 block, hipStream_t s, const void *I, ImageParams p,
                                 const DevTables *tab, int32_t *ws) {
  switch (G) {
    case 1: hipLaunchKernelGGL((ka_sat<1, U8, false, true>), grid, block, 0, s, I, p, tab, ws); break;
    case 2: hipLaunchKernelGGL((ka_sat<2, U8, false, true>), grid, block, 0, s, I, p, tab, ws); break;
    case 3: hipLaunchKernelGGL((ka_sat<3, U8, false, true>), grid, block, 0, s, I, p, tab, ws); break;
    default: hipLaunchKernelGGL((ka_sat<4, U8, false, true>), grid, block, 0, s, I, p, tab, ws); break;
  }
  return hipGetLastError();
}

// mode: 0 a range term per wave, 1 a table, 2 a cosine or sine pair
template <bool U8>
static hipError_t launch_ka(int G, int mode, dim3 grid, dim3 block, hipStream_t s, const void *I,
                            ImageParams p, const DevTables *tab, int32_t *ws) {
  if (mode == 2) return launch_ka_pair<U8>(G, grid, block, s, I, p, tab, ws);
  return mode == 1 ? launch_ka1<U8, true>(G, grid, block, s, I, p, tab, ws)
                   : launch_ka1<U8, false>(G, grid, block, s, I, p, tab, ws);
}

template <bool U8>
static hipError_t launch_kb(dim3 grid, dim3 block, hipStream_t s, const void *I, ImageParams p,
                            const DevTables *tab, const int32_t *ws, float *out, float *num,
                            float *den) {
  hipLaunchKernelGGL((kb_lookup<U8>), grid, block, 0, s, I, p, tab, ws, out, num, den);
  return hipGetLastError();
}

// Staged-region row pitches: 128 double-buffered (two regions of up to 128 x
// 128 take at most 128 KB), wider regions single-buffered.
static const int kLdsPitches[] = {128, 160, 176, 192};

int lds_pitch_for(int width) {
  for (int pch : kLdsPitches)
    if (width <= pch) return pch;
  return 0;
}

static size_t kb_region_bytes(const DevTables &h) {
  return (size_t)(64 + h.tap_dy_max - h.tap_dy_min) * h.lds_pitch * sizeof(int32_t);
}
bool kb_double_buffered(const DevTables &h) {
  return h.lds_pitch == 128 && 2 * kb_region_bytes(h) <= 160 * 1024;
}
// overlap staging at pitch 160 and 176 (at 192 the overlap would take too
// many registers), for regions it can hold
bool kb_overlap_staged(const DevTables &h, int pitch) {
  return (pitch == 160 || pitch == 176) && 64 + h.tap_dy_max - h.tap_dy_min <= kOverlapMaxRows(pitch);
}

template <int PITCH, int NQ, int ST, bool U8>
static hipError_t launch_kb_tile(dim3 grid, size_t lds, hipStream_t s, const void *I,
                                 ImageParams p, const DevTables *tab, const int32_t *ws, float *out,
                                 float *num, float *den) {
  auto k = kb_tile<PITCH, NQ, ST, U8>;
  hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, grid, dim3(1024), lds, s, I, p, tab, ws, out, num, den);
  return hipGetLastError();
}

template <int PITCH, int ST, bool U8>
static hipError_t launch_kb_tile_nq(int nq, dim3 grid, size_t lds, hipStream_t s, const void *I,
                                    ImageParams p, const DevTables *tab, const int32_t *ws,
                                    float *out, float *num, float *den) {
  if (nq <= 4) return launch_kb_tile<PITCH, 4, ST, U8>(grid, lds, s, I, p, tab, ws, out, num, den);
  if (nq <= 8) return launch_kb_tile<PITCH, 8, ST, U8>(grid, lds, s, I, p, tab, ws, out, num, den);
  return launch_kb_tile<PITCH, 12, ST, U8>(grid, lds, s, I, p, tab, ws, out, num, den);
}

template <int ST, bool U8>
static hipError_t launch_kb_tile_pitch(int pitch, int nq, dim3 grid, size_t lds, hipStream_t s,
                                       const void *I, ImageParams p, const DevTables *tab,
                                       const int32_t *ws, float *out, float *num, float *den) {
  switch (pitch) {
    case 128: return launch_kb_tile_nq<128, ST, U8>(nq, grid, lds, s, I, p, tab, ws, out, num, den);
    case 160: return launch_kb_tile_nq<160, ST, U8>(nq, grid, lds, s, I, p, tab, ws, out, num, den);
    case 176: return launch_kb_tile_nq<176, ST, U8>(nq, grid, lds, s, I, p, tab, ws, out, num, den);
    default: return launch_kb_tile_nq<192, ST, U8>(nq, grid, lds, s, I, p, tab, ws, out, num, den);
  }
}

template <bool U8>
static hipError_t launch_kb_tile_any(const DevTables &h, bool single, dim3 grid, hipStream_t s,
                                     const void *I, ImageParams p, const DevTables *tab,
                                     const int32_t *ws, float *out, float *num, float *den) {
  const size_t lds = kb_region_bytes(h);
  const int nq = h.n_quads;
  if (!single && kb_double_buffered(h))
    return launch_kb_tile_nq<128, kStageDouble, U8>(nq, grid, 2 * lds, s, I, p, tab, ws, out, num, den);
  if (kb_overlap_staged(h, h.lds_pitch)) {
    const size_t lo = lds + (size_t)kOverlapBase(h.lds_pitch) * h.lds_pitch * sizeof(int32_t);
    return h.lds_pitch == 160
               ? launch_kb_tile_nq<160, kStageOverlap, U8>(nq, grid, lo, s, I, p, tab, ws, out, num, den)
               : launch_kb_tile_nq<176, kStageOverlap, U8>(nq, grid, lo, s, I, p, tab, ws, out, num, den);
  }
  return launch_kb_tile_pitch<kStageSingle, U8>(h.lds_pitch, nq, grid, lds, s, I, p, tab, ws, out, num, den);
}

void choose_tiling(int H, int W, int radius, int n_terms, int fixed_tile, double gmax, int row_unit, int *tile,
                   int *sat_shift) {
  int t = fixed_tile;
  if (!t) {
    // table tiles that hold whole lattice tiles (multiples of 64 and of
    // row_unit, up to 576), else the general ones
    std::vector<int> cands;
    if (row_unit > 0) {
      const int l = std::lcm(64, row_unit);
      for (int c = (576 / l) * l; c >= l; c -= l) cands.push_back(c);
    }
    if (cands.empty()) cands = {512, 256, 128, 64};
    t = cands.back();
    for (int c : cands) {
      if (c + 2 * radius + 1 > 768) continue;
      const long long waves = (long long)((H + c - 1) / c) * ((W + c - 1) / c) * n_terms;
      t = c;
      if (waves >= 2048) break;
    }
  }
  const double E = 2.0 * radius + 1.0;
  const double lim = 2147483647.0 / (E * E);  // bound of |round(v 2^q)| per entry
  int q = 0;
  while (q < 24 && gmax * std::ldexp(1.0, q + 1) * (1.0 + std::ldexp(1.0, -20)) + 1.0 <= lim) ++q;
  *tile = t;
  *sat_shift = q;
}

Geometry make_geometry(int H, int W, int tile, int radius, int n_images, int sat_shift) {
  Geometry g;
  g.sat_shift = sat_shift;
  g.H = H;
  g.W = W;
  g.tile = tile;
  g.radius = radius;
  g.tiles_y = (H + tile - 1) / tile;
  g.tiles_x = (W + tile - 1) / tile;
  g.n_images = n_images;
  g.E_max = tile + 2 * radius + 1;
  g.pitch = (g.E_max + 63) / 64 * 64;
  g.table_elems = (size_t)g.E_max * g.pitch;
  g.ready_off = (size_t)g.tiles_y * g.tiles_x * n_images * g.table_elems * sizeof(int32_t);
  // the fused batch launch's ready counters, one per table tile (none without tables)
  g.bytes = g.ready_off + (n_images ? ((size_t)g.tiles_y * g.tiles_x * sizeof(uint32_t) + 255) / 256 * 256 : 0);
  return g;
}

static ImageParams image_params(const DevTables &host, const Geometry &g) {
  ImageParams p;
  p.H = g.H;
  p.W = g.W;
  p.tile = g.tile;
  p.radius = g.radius;
  p.tiles_x = g.tiles_x;
  p.n_images = g.n_images;
  p.pitch = g.pitch;
  p.n_terms = host.n_terms;
  p.table_elems = (long long)g.table_elems;
  p.sat_scale = std::ldexp(1.0f, g.sat_shift);
  p.inv_sat_scale = std::ldexp(1.0f, -g.sat_shift);
  return p;
}

// 256-column chunks of one K-A wave row (the table row of this image)
static int ka_chunks(const Geometry &g) {
  const int Ew = std::min(g.tile + 2 * g.radius + 1, g.W + 1);
  return (Ew + 255) / 256;
}

bool kb_tile_eligible(const DevTables &h) {
  return h.lds_pitch > 0 && kb_region_bytes(h) <= 160 * 1024 && h.n_quads <= 12;
}

int lookup_kernel_kind(const DevTables &h) { return kb_tile_eligible(h) || lattice_eligible(h) ? 1 : 0; }

bool lattice_eligible(const DevTables &h) {
  return h.lat && h.lat_pitch > 0 && lattice_lds_bytes(h) <= 160 * 1024;
}

int lookup_kernel_for(const DevTables &h, int kb_single) {
  const bool tile = kb_tile_eligible(h), lat = lattice_eligible(h);
  const bool db = tile && kb_double_buffered(h);
  if (kb_single == 2 && lat) return 3;
  if (kb_single == 1 && tile) return 2;
  if (db) return 1;
  // without double buffering, the lattice kernel's fewer table reads pay for
  // its staging once a pixel has more than 8 boxes
  if (lat && h.n_quads > 8) return 3;
  if (tile) return 2;
  return lat ? 3 : 0;
}

int lattice_rows(const DevTables &h) { return h.lat_s * kLatU * h.lat_g; }

template <int PITCH, int M, int N, bool U8, uint32_t MASK = 0xFFFFu>
static hipError_t launch_kl1(int n_tiles, size_t lds, hipStream_t s, const void *I, ImageParams p,
                             const DevTables *tab, const int32_t *ws, float *out, float *num, float *den, bool tab12 = false) {
  auto k = kl_tile<PITCH, M, N, U8, MASK>;
  auto k12 = kl_tile<PITCH, M, N, U8, MASK, 12>;
  // twelve-wave blocks where twelve waves compute (no wave that only copies)
  const bool w12 = MASK != 0xFFFFu && tab12;
  hipError_t e = hipFuncSetAttribute(w12 ? (const void *)k12 : (const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (w12) hipLaunchKernelGGL(k12, dim3(8 * ((n_tiles + 7) / 8)), dim3(768), lds, s, I, p, tab, ws, out, num, den, n_tiles);
  else hipLaunchKernelGGL(k, dim3(8 * ((n_tiles + 7) / 8)), dim3(1024), lds, s, I, p, tab, ws, out, num, den, n_tiles);
  return hipGetLastError();
}

template <int PITCH, bool U8>
static hipError_t launch_kl_mn(const DevTables &h, int n_tiles, size_t lds, hipStream_t s, const void *I,
                               ImageParams p, const DevTables *tab, const int32_t *ws, float *out, float *num,
                               float *den) {
  const bool n4 = h.lat_n > 2;
  switch (h.lat_m) {
    case 2: return n4 ? launch_kl1<PITCH, 2, 4, U8>(n_tiles, lds, s, I, p, tab, ws, out, num, den)
                      : launch_kl1<PITCH, 2, 2, U8>(n_tiles, lds, s, I, p, tab, ws, out, num, den);
    case 3: return n4 ? launch_kl1<PITCH, 3, 4, U8>(n_tiles, lds, s, I, p, tab, ws, out, num, den)
                      : launch_kl1<PITCH, 3, 2, U8>(n_tiles, lds, s, I, p, tab, ws, out, num, den);
    default:
      // the boxes of the N_s = 8 Gaussian expansion's level groups: an
      // instantiation that skips the 4 empty ones of the 16
      if (n4 && h.lat_mask == (int)kLatMaskNs8)
        return launch_kl1<PITCH, 4, 4, U8, kLatMaskNs8>(n_tiles, lds, s, I, p, tab, ws, out, num, den, h.lat_s * h.lat_g == 12);
      return n4 ? launch_kl1<PITCH, 4, 4, U8>(n_tiles, lds, s, I, p, tab, ws, out, num, den)
                : launch_kl1<PITCH, 4, 2, U8>(n_tiles, lds, s, I, p, tab, ws, out, num, den);
  }
}

template <bool U8>
static hipError_t launch_kl(const DevTables &h, const Geometry &g, hipStream_t s, const void *I, ImageParams p,
                            const DevTables *tab, const int32_t *ws, float *out, float *num, float *den) {
  const LatGrid lg = lat_grid(g.H, g.W, g.tile, h.lat_s, h.lat_g);
  const int n_tiles = lg.nty * lg.ntx;
  const size_t lds = lattice_lds_bytes(h);
  return h.lat_pitch == 128 ? launch_kl_mn<128, U8>(h, n_tiles, lds, s, I, p, tab, ws, out, num, den)
                            : launch_kl_mn<192, U8>(h, n_tiles, lds, s, I, p, tab, ws, out, num, den);
}

bf_status_t launch_tables(const DevTables *dev, const DevTables &host, const Geometry &g,
                          const void *I, int32_t *ws, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const ImageParams p = image_params(host, g);
  const int G = ka_chunks(g);
  if (G > kMaxChunks) return BF_ERR_UNSUPPORTED;
  // a pair per wave only where its instantiations go (rows of up to 4 chunks)
  const int mode = g.ka_one == 2 && G > 4 ? 0 : g.ka_one;
  const int units = mode == 1 ? host.n_images : mode == 2 ? 2 * host.n_terms : host.n_terms;
  dim3 ga(g.tiles_y * g.tiles_x, (units + 3) / 4), ba(256);
  profile_mark(0, 1, stream);
  hipError_t e = host.in_u8 ? launch_ka<true>(G, mode, ga, ba, s, I, p, dev, ws)
                            : launch_ka<false>(G, mode, ga, ba, s, I, p, dev, ws);
  profile_mark(0, 0, stream);
  return e == hipSuccess ? BF_OK : BF_ERR_DEVICE;
}

bf_status_t launch_lookup(const DevTables *dev, const DevTables &host, const Geometry &g,
                          const void *I, float *out, float *num, float *den, const int32_t *ws,
                          void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const ImageParams p = image_params(host, g);
  hipError_t e;
  // LDS tile kernel when the staged region fits and the quadruplets' corner
  // addresses fit in registers, else the per-pixel kernel
  profile_mark(1, 1, stream);
  const int kind = lookup_kernel_for(host, g.kb_single);
  if (kind == 3) {
    e = host.in_u8 ? launch_kl<true>(host, g, s, I, p, dev, ws, out, num, den)
                   : launch_kl<false>(host, g, s, I, p, dev, ws, out, num, den);
  } else if (kind != 0) {
    const int n_tiles = ((g.W + 63) / 64) * ((g.H + 63) / 64);
    dim3 gt(8 * ((n_tiles + 7) / 8));
    const bool single = kind == 2;
    e = host.in_u8 ? launch_kb_tile_any<true>(host, single, gt, s, I, p, dev, ws, out, num, den)
                   : launch_kb_tile_any<false>(host, single, gt, s, I, p, dev, ws, out, num, den);
  } else {
    dim3 gb((g.W + 63) / 64, (g.H + 3) / 4), bb(256);
    e = host.in_u8 ? launch_kb<true>(gb, bb, s, I, p, dev, ws, out, num, den)
                   : launch_kb<false>(gb, bb, s, I, p, dev, ws, out, num, den);
  }
  profile_mark(1, 0, stream);
  return e == hipSuccess ? BF_OK : BF_ERR_DEVICE;
}

bf_status_t launch_filter(const DevTables *dev, const DevTables &host, const Geometry &g,
                          const void *I, float *out, float *num, float *den, int32_t *ws,
                          void *stream) {
  if (host.direct) return launch_direct(host, I, out, num, den, g.H, g.W, stream);
  if (host.range_box) return launch_rangebox(dev, host, I, out, num, den, g.H, g.W, stream);
  if (host.reduced) return launch_reduced(dev, host, g, I, out, num, den, ws, stream);
  bf_status_t st = launch_tables(dev, host, g, I, ws, stream);
  if (st != BF_OK) return st;
  return launch_lookup(dev, host, g, I, out, num, den, ws, stream);
}

template <bool U8, bool ONE>
static hipError_t launch_ka_batch1(int G, int blocks, hipStream_t s, const BatchArgs &a) {
  dim3 grid(blocks), block(256);
  switch (G) {
    case 1: hipLaunchKernelGGL((ka_batch<1, U8, ONE>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((ka_batch<2, U8, ONE>), grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL((ka_batch<3, U8, ONE>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((ka_batch<4, U8, ONE>), grid, block, 0, s, a); break;
    case 5: hipLaunchKernelGGL((ka_batch<5, U8, ONE>), grid, block, 0, s, a); break;
    case 6: hipLaunchKernelGGL((ka_batch<6, U8, ONE>), grid, block, 0, s, a); break;
    case 7: hipLaunchKernelGGL((ka_batch<7, U8, ONE>), grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL((ka_batch<8, U8, ONE>), grid, block, 0, s, a); break;
  }
  return hipGetLastError();
}

template <bool U8>
static hipError_t launch_ka_batch(int G, bool one, int blocks, hipStream_t s, const BatchArgs &a) {
  return one ? launch_ka_batch1<U8, true>(G, blocks, s, a) : launch_ka_batch1<U8, false>(G, blocks, s, a);
}

template <int PITCH, int NQ, int ST, bool U8>
static hipError_t launch_kb_batch1(int blocks, size_t lds, hipStream_t s, const BatchArgs &a) {
  auto k = kb_batch<PITCH, NQ, ST, U8>;
  hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(1024), lds, s, a);
  return hipGetLastError();
}

template <int PITCH, int M, int N, bool U8>
static hipError_t launch_kl_batch1(int blocks, size_t lds, hipStream_t s, const BatchArgs &a) {
  auto k = kl_batch<PITCH, M, N, U8>;
  hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(1024), lds, s, a);
  return hipGetLastError();
}

// the lattice class index (pitch, M, N) of a plan: 0 .. kLatClasses - 1
static int lattice_class(const DevTables &h) {
  return (h.lat_pitch == 128 ? 0 : 6) + (h.lat_m - 2) * 2 + (h.lat_n > 2 ? 1 : 0);
}

template <int PITCH, bool U8>
static hipError_t launch_kl_batch_mn(int mn, int blocks, size_t lds, hipStream_t s, const BatchArgs &a) {
  switch (mn) {
    case 0: return launch_kl_batch1<PITCH, 2, 2, U8>(blocks, lds, s, a);
    case 1: return launch_kl_batch1<PITCH, 2, 4, U8>(blocks, lds, s, a);
    case 2: return launch_kl_batch1<PITCH, 3, 2, U8>(blocks, lds, s, a);
    case 3: return launch_kl_batch1<PITCH, 3, 4, U8>(blocks, lds, s, a);
    case 4: return launch_kl_batch1<PITCH, 4, 2, U8>(blocks, lds, s, a);
    default: return launch_kl_batch1<PITCH, 4, 4, U8>(blocks, lds, s, a);
  }
}

template <bool U8>
static hipError_t launch_kl_batch(int cls, int blocks, size_t lds, hipStream_t s, const BatchArgs &a) {
  return cls < 6 ? launch_kl_batch_mn<128, U8>(cls % 6, blocks, lds, s, a)
                 : launch_kl_batch_mn<192, U8>(cls % 6, blocks, lds, s, a);
}

template <int PITCH, int ST, bool U8>
static hipError_t launch_kb_batch_nq(int nq, int blocks, size_t lds, hipStream_t s, const BatchArgs &a) {
  if (nq <= 4) return launch_kb_batch1<PITCH, 4, ST, U8>(blocks, lds, s, a);
  if (nq <= 8) return launch_kb_batch1<PITCH, 8, ST, U8>(blocks, lds, s, a);
  return launch_kb_batch1<PITCH, 12, ST, U8>(blocks, lds, s, a);
}

template <int ST, bool U8>
static hipError_t launch_kb_batch_pitch(int pitch, int nq, int blocks, size_t lds, hipStream_t s,
                                        const BatchArgs &a) {
  switch (pitch) {
    case 128: return launch_kb_batch_nq<128, ST, U8>(nq, blocks, lds, s, a);
    case 160: return launch_kb_batch_nq<160, ST, U8>(nq, blocks, lds, s, a);
    case 176: return launch_kb_batch_nq<176, ST, U8>(nq, blocks, lds, s, a);
    default: return launch_kb_batch_nq<192, ST, U8>(nq, blocks, lds, s, a);
  }
}

template <bool U8>
static hipError_t launch_kb_batch(int pitch, int st, int nq, int blocks, size_t lds, hipStream_t s,
                                  const BatchArgs &a) {
  if (st == kStageDouble) return launch_kb_batch_nq<128, kStageDouble, U8>(nq, blocks, lds, s, a);
  if (st == kStageOverlap) {  // at most 8 quadruplets (launch_batch_chunk)
    if (pitch == 160)
      return nq <= 4 ? launch_kb_batch1<160, 4, kStageOverlap, U8>(blocks, lds, s, a)
                     : launch_kb_batch1<160, 8, kStageOverlap, U8>(blocks, lds, s, a);
    return nq <= 4 ? launch_kb_batch1<176, 4, kStageOverlap, U8>(blocks, lds, s, a)
                   : launch_kb_batch1<176, 8, kStageOverlap, U8>(blocks, lds, s, a);
  }
  return launch_kb_batch_pitch<kStageSingle, U8>(pitch, nq, blocks, lds, s, a);
}

template <int NQ, int G, bool U8, bool ONE>
static hipError_t launch_kf1(int blocks, size_t lds, hipStream_t s, const FusedArgs &a) {
  auto k = kf_batch<NQ, U8, G, ONE>;
  hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(1024), lds, s, a);
  return hipGetLastError();
}

// one range term per table wave (ONE = false) for table rows of at most
// 2 chunks, else one table per wave (fewer registers)
template <int NQ, bool U8>
static hipError_t launch_kf_g(int G, bool one, int blocks, size_t lds, hipStream_t s, const FusedArgs &a) {
  if (!one) return G == 1 ? launch_kf1<NQ, 1, U8, false>(blocks, lds, s, a) : launch_kf1<NQ, 2, U8, false>(blocks, lds, s, a);
  switch (G) {
    case 1: return launch_kf1<NQ, 1, U8, true>(blocks, lds, s, a);
    case 2: return launch_kf1<NQ, 2, U8, true>(blocks, lds, s, a);
    case 3: return launch_kf1<NQ, 3, U8, true>(blocks, lds, s, a);
    default: return launch_kf1<NQ, 4, U8, true>(blocks, lds, s, a);
  }
}

// the counters and queues first (a fill kernel, so that the pair can be
// captured in a graph), then the fused launch
template <bool U8>
static hipError_t launch_kf(int nq, int G, bool one, int blocks, size_t lds, hipStream_t s, const FusedArgs &a) {
  hipLaunchKernelGGL(kf_reset, dim3(1), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return nq <= 4 ? launch_kf_g<4, U8>(G, one, blocks, lds, s, a) : launch_kf_g<8, U8>(G, one, blocks, lds, s, a);
}

// The fused launch takes a group whose every image is looked up by the LDS
// tile kernel -- double-buffered at pitch 128, or overlap-staged at pitch 176
// (regions up to kOverlapMaxRows(176) rows) -- with at most 8 quadruplets and
// table rows of at most 4 chunks; *lds is then the launch's LDS.
static std::atomic<int> g_fused_batch{0};  // bf_batch_set_fused

void set_fused_batch(int on) { g_fused_batch.store(on); }

static bool fused_eligible(const BatchItem *items, const int *idx, int n, const int *kind, int *nq, int *G,
                           size_t *lds) {
  if (!g_fused_batch.load()) return false;
  *nq = 0;
  *G = 1;
  *lds = 0;
  for (int j = 0; j < n; ++j) {
    const BatchItem &it = items[idx[j]];
    const DevTables &h = *it.host;
    const int rh = 64 + h.tap_dy_max - h.tap_dy_min, rw = 64 + h.tap_dx_max - h.tap_dx_min;
    if (kind[j] == 1)
      *lds = std::max(*lds, (size_t)2 * rh * 128 * sizeof(int32_t));
    else if (kind[j] == 2 && rw <= 176 && rh <= kOverlapMaxRows(176))
      *lds = std::max(*lds, (size_t)(kOverlapBase(176) + rh) * 176 * sizeof(int32_t));
    else
      return false;
    *nq = std::max(*nq, h.n_quads);
    *G = std::max(*G, ka_chunks(it.g));
  }
  if (items[idx[0]].host->in_u8) *lds = std::max(*lds, (size_t)kFusedUnits * 256 * sizeof(int4));  // a lookup table per wave
  return *nq <= 8 && *G <= 4;
}

// One chunk of at most kMaxBatch images of one input type.
static bf_status_t launch_batch_chunk(const BatchItem *items, const int *idx, int n, uint32_t *heads,
                                      hipStream_t s) {
  const bool u8 = items[idx[0]].host->in_u8 != 0;
  int dev = 0, n_cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) n_cu = v;
  }
  // each image's lookup kernel, as its single-image call would choose it;
  // 4: the lattice kernel as the untuned default, launched per image as a
  // single call launches it (its persistent form, for images tuned to the
  // lattice kernel, spills registers at four columns of boxes)
  int kind[kMaxBatch];
  for (int j = 0; j < n; ++j) {
    const BatchItem &it = items[idx[j]];
    kind[j] = lookup_kernel_for(*it.host, it.g.kb_single);
    if (kind[j] == 3 && it.g.kb_single != 2) kind[j] = 4;
  }
  {
    int nq, G;
    size_t lds;
    if (fused_eligible(items, idx, n, kind, &nq, &G, &lds)) {
      FusedArgs f{};
      f.n = n;
      f.ctl = heads;
      // a range term per table wave as the images were tuned, where the rows allow
      bool one = G > 2;
      for (int j = 0; j < n; ++j) one = one || items[idx[j]].g.ka_one != 0;
      int a_items = 0, b_tiles = 0;
      for (int j = 0; j < n; ++j) {
        const BatchItem &it = items[idx[j]];
        BatchImage &im = f.img[j];
        im.I = it.I;
        im.out = it.out;
        im.ws = it.ws;
        im.tab = it.dev;
        im.p = image_params(*it.host, it.g);
        im.n_tiles = ((it.g.W + 63) / 64) * ((it.g.H + 63) / 64);
        im.per_xcd = (im.n_tiles + 7) / 8;
        f.groups[j] = ((one ? it.host->n_images : it.host->n_terms) + kFusedUnits - 1) / kFusedUnits;
        f.db[j] = kind[j] == 1;
        f.ready[j] = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(it.ws) + it.g.ready_off);
        f.a_start[j] = a_items;
        a_items += it.g.tiles_y * it.g.tiles_x * f.groups[j];
        b_tiles += im.n_tiles;
      }
      f.a_start[n] = a_items;
      const int blocks = std::min(8 * ((std::max(a_items, b_tiles) + 7) / 8), 8 * ((n_cu + 7) / 8));
      profile_mark(1, 1, s);
      hipError_t e =
          u8 ? launch_kf<true>(nq, G, one, blocks, lds, s, f) : launch_kf<false>(nq, G, one, blocks, lds, s, f);
      profile_mark(1, 0, s);
      return e == hipSuccess ? BF_OK : BF_ERR_DEVICE;
    }
  }
  BatchArgs ka{};
  ka.n = n;
  ka.heads = heads;
  // one table per K-A wave when every image of the group was tuned that way
  bool one = true;
  for (int j = 0; j < n; ++j) one = one && items[idx[j]].g.ka_one != 0;
  int G = 1, blocks = 0;
  for (int j = 0; j < n; ++j) {
    const BatchItem &it = items[idx[j]];
    BatchImage &im = ka.img[j];
    im.I = it.I;
    im.out = it.out;
    im.ws = it.ws;
    im.tab = it.dev;
    im.p = image_params(*it.host, it.g);
    im.ka_blocks = it.g.tiles_y * it.g.tiles_x * (((one ? it.host->n_images : it.host->n_terms) + 3) / 4);
    im.n_tiles = ((it.g.W + 63) / 64) * ((it.g.H + 63) / 64);
    im.per_xcd = (im.n_tiles + 7) / 8;
    ka.ka_start[j] = blocks;
    blocks += im.ka_blocks;
    G = std::max(G, ka_chunks(it.g));
  }
  ka.ka_start[n] = blocks;
  if (G > kMaxChunks) return BF_ERR_UNSUPPORTED;
  profile_mark(0, 1, s);
  hipError_t e = u8 ? launch_ka_batch<true>(G, one, blocks, s, ka) : launch_ka_batch<false>(G, one, blocks, s, ka);
  profile_mark(0, 0, s);
  if (e != hipSuccess) return BF_ERR_DEVICE;

  // K-B: images the LDS tile kernel takes run in persistent launches, one
  // per buffering class -- double-buffered at pitch 128, and single-buffered
  // at the widest pitch of the rest -- each at the largest quadruplet count
  // of its class, with its own 8 queue heads; the others run the per-pixel
  // kernel one by one.
  profile_mark(1, 1, s);
  for (int cls = 0; cls < 2; ++cls) {
    BatchArgs kb{};
    kb.heads = heads + 8 * cls;
    int pitch = 0, nq = 0, tiles = 0, rh = 0;
    for (int j = 0; j < n; ++j) {
      const BatchItem &it = items[idx[j]];
      const DevTables &h = *it.host;
      if (kind[j] != 1 + cls) continue;
      kb.img[kb.n++] = ka.img[j];
      pitch = std::max(pitch, h.lds_pitch);
      nq = std::max(nq, h.n_quads);
      rh = std::max(rh, 64 + h.tap_dy_max - h.tap_dy_min);
      tiles += ka.img[j].n_tiles;
    }
    if (kb.n == 0) continue;
    const bool db = cls == 0;
    // overlap staging when every image's region is no taller than the class pitch
    const int st = db ? kStageDouble
                   : (pitch == 160 || pitch == 176) && rh <= kOverlapMaxRows(pitch) && nq <= 8 ? kStageOverlap
                                                                                             : kStageSingle;
    const size_t lds = (size_t)(rh * (db ? 2 : 1) + (st == kStageOverlap ? kOverlapBase(pitch) : 0)) * pitch *
                       sizeof(int32_t);
    const int grid = std::min(8 * ((tiles + 7) / 8), 8 * ((n_cu + 7) / 8));
    e = u8 ? launch_kb_batch<true>(pitch, st, nq, grid, lds, s, kb)
           : launch_kb_batch<false>(pitch, st, nq, grid, lds, s, kb);
    if (e != hipSuccess) {
      profile_mark(1, 0, s);
      return BF_ERR_DEVICE;
    }
  }
  // lattice kernels: one persistent launch per (pitch, M, N) class, queue
  // heads 16 + 8 class onwards
  for (int cls = 0; cls < kLatClasses; ++cls) {
    BatchArgs kb{};
    kb.heads = heads + 16 + 8 * cls;
    int tiles = 0;
    size_t lds = 0;
    for (int j = 0; j < n; ++j) {
      const BatchItem &it = items[idx[j]];
      const DevTables &h = *it.host;
      if (kind[j] != 3 || lattice_class(h) != cls) continue;
      BatchImage im = ka.img[j];
      const LatGrid lg = lat_grid(it.g.H, it.g.W, it.g.tile, h.lat_s, h.lat_g);
      im.n_tiles = lg.nty * lg.ntx;
      im.per_xcd = (im.n_tiles + 7) / 8;
      kb.img[kb.n++] = im;
      lds = std::max(lds, lattice_lds_bytes(h));
      tiles += im.n_tiles;
    }
    if (kb.n == 0) continue;
    const int grid = std::min(8 * ((tiles + 7) / 8), 8 * ((n_cu + 7) / 8));
    e = u8 ? launch_kl_batch<true>(cls, grid, lds, s, kb) : launch_kl_batch<false>(cls, grid, lds, s, kb);
    if (e != hipSuccess) {
      profile_mark(1, 0, s);
      return BF_ERR_DEVICE;
    }
  }
  for (int j = 0; j < n; ++j) {
    const BatchItem &it = items[idx[j]];
    if (kind[j] != 0 && kind[j] != 4) continue;
    const BatchImage &im = ka.img[j];
    if (kind[j] == 4) {
      e = u8 ? launch_kl<true>(*it.host, it.g, s, it.I, im.p, it.dev, it.ws, it.out, nullptr, nullptr)
             : launch_kl<false>(*it.host, it.g, s, it.I, im.p, it.dev, it.ws, it.out, nullptr, nullptr);
    } else {
      dim3 gb((it.g.W + 63) / 64, (it.g.H + 3) / 4), bb(256);
      e = u8 ? launch_kb<true>(gb, bb, s, it.I, im.p, it.dev, it.ws, it.out, nullptr, nullptr)
             : launch_kb<false>(gb, bb, s, it.I, im.p, it.dev, it.ws, it.out, nullptr, nullptr);
    }
    if (e != hipSuccess) break;
  }
  profile_mark(1, 0, s);
  return e == hipSuccess ? BF_OK : BF_ERR_DEVICE;
}

bf_status_t launch_batch(const BatchItem *items_all, int n_all, uint32_t *heads, void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  // requests without term tables: direct summation in one launch per input
  // type and range kernel kind, the range-box regime in one launch per output
  // tile size; reduced-precision requests in one pair of launches per input
  // type
  std::vector<BatchItem> kept;
  kept.reserve(n_all);
  std::vector<const DevTables *> dh, zd, zh, rd, rh;
  std::vector<const void *> di, zi, ri;
  std::vector<float *> dout, zout, rout;
  std::vector<void *> rws;
  std::vector<Geometry> rg;
  std::vector<int> dH, dW, zH, zW;
  for (int i = 0; i < n_all; ++i) {
    const BatchItem &it = items_all[i];
    if (it.host->direct) {
      dh.push_back(it.host);
      di.push_back(it.I);
      dout.push_back(it.out);
      dH.push_back(it.g.H);
      dW.push_back(it.g.W);
    } else if (it.host->range_box) {
      zd.push_back(it.dev);
      zh.push_back(it.host);
      zi.push_back(it.I);
      zout.push_back(it.out);
      zH.push_back(it.g.H);
      zW.push_back(it.g.W);
    } else if (it.host->reduced) {
      rd.push_back(it.dev);
      rh.push_back(it.host);
      rg.push_back(it.g);
      ri.push_back(it.I);
      rout.push_back(it.out);
      rws.push_back(it.ws);
    } else {
      kept.push_back(it);
    }
  }
  if (!dh.empty()) {
    bf_status_t st = launch_direct_batch(dh.data(), di.data(), dout.data(), dH.data(), dW.data(), (int)dh.size(),
                                         stream);
    if (st != BF_OK) return st;
  }
  if (!zd.empty()) {
    bf_status_t st = launch_rangebox_batch(zd.data(), zh.data(), zi.data(), zout.data(), zH.data(), zW.data(),
                                           (int)zd.size(), stream);
    if (st != BF_OK) return st;
  }
  if (!rd.empty()) {
    bf_status_t st = launch_reduced_batch(rd.data(), rh.data(), rg.data(), ri.data(), rout.data(), rws.data(),
                                          (int)rd.size(), stream);
    if (st != BF_OK) return st;
  }
  const BatchItem *items = kept.data();
  const int n = (int)kept.size();
  // by input type, costliest first (largest tile count x tables x quadruplets)
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  auto cost = [&](int i) {
    const BatchItem &it = items[i];
    return (double)((it.g.W + 63) / 64) * ((it.g.H + 63) / 64) * it.host->n_images * std::max(1, it.host->n_quads);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (items[a].host->in_u8 != items[b].host->in_u8) return items[a].host->in_u8 < items[b].host->in_u8;
    return cost(a) > cost(b);
  });
  for (int j0 = 0; j0 < n;) {
    int j1 = j0;
    while (j1 < n && j1 - j0 < kMaxBatch && items[order[j1]].host->in_u8 == items[order[j0]].host->in_u8) ++j1;
    bf_status_t st = launch_batch_chunk(items, order.data() + j0, j1 - j0, heads, s);
    if (st != BF_OK) return st;
    j0 = j1;
  }
  return BF_OK;
}

}  // namespace bf
