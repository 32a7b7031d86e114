// gfx950 kernels of the N-term bilateral filter.
//
// K-A (ka_sat): for one output tile and one range term k, modulate the image
//   (C = cos(omega_k I), S = sin(omega_k I); term values C*I, S*I, C, S, or I
//   alone for k = 0 -- the shift identity of Eq. 1D_N_terms) and build the
//   summed-area table of each term image over the tile plus an r-pixel halo
//   (recurrences of Eq. sum_sat_recurrence_2D: prefix along the row, then
//   accumulation down the columns).  Values are stored as round(v * 2^q) in
//   int32, so every prefix sum and every box difference is exact; q is chosen
//   per plan so that no tile table can overflow.
// K-B (kb_lookup): per output pixel, read the table at the taps of the
//   spatial expansion (four-reference box sums of Eq. sum_sat_sum_region_2D,
//   merged at shared corners), accumulate the numerator and denominator of
//   Eq. BF over the range terms and normalise.
//
// Layout in HBM: one workspace of int32 tables, [tile][image][row][pitch],
// each table (tile + 2r + 1) x pitch with pitch a multiple of 64 elements.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "bf_internal.h"

namespace bf {

// Per-launch scalars of one image.
struct ImageParams {
  int H, W, tile, radius, tiles_x, n_images, pitch, n_terms;
  long long table_elems;
  float sat_scale;       // 2^q
  double inv_sat_scale;  // 2^-q
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
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  int x = v;
  x += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);   // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);   // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, v, 0x113, 0xf, 0xf, true);   // row_shr:3
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xe, false);  // row_shr:4, lanes 4..15 of a row
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xc, false);  // row_shr:8, lanes 8..15 of a row
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
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

template <int G, bool U8>
__global__ __launch_bounds__(256) void ka_sat(const void *__restrict__ I, ImageParams p,
                                             const DevTables *__restrict__ tab,
                                             int32_t *__restrict__ ws) {
  // the wave index is uniform; saying so keeps per-term loads scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int term = blockIdx.y * 4 + wave;
  if (term >= p.n_terms) return;
  const int tile_id = blockIdx.x;
  const int ty = tile_id / p.tiles_x, tx = tile_id - ty * p.tiles_x;
  const int y0 = ty * p.tile, x0 = tx * p.tile;
  const int y1 = min(p.H, y0 + p.tile), x1 = min(p.W, x0 + p.tile);
  const int oy = max(y0 - p.radius, 0), ox = max(x0 - p.radius, 0);
  const int Eh = min(y1 + p.radius, p.H) - oy + 1;
  const int Ew = min(x1 + p.radius, p.W) - ox + 1;
  const bool k0 = tab->k_is_zero[term] != 0;
  const int nimg = k0 ? 1 : 4;
  const float f_hi = tab->f_hi[term], f_lo = tab->f_lo[term];
  const float scale = p.sat_scale;
  int32_t *base = ws + ((long long)tile_id * p.n_images + tab->slot[term]) * p.table_elems;
  const long long te = p.table_elems;

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

  int acc[4][G][4];
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

    int carry[4] = {0, 0, 0, 0};
    int32_t *row = base + (long long)i * p.pitch;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      int v[4][4];  // [image][column]
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float px = cur[g][c];
        const float xs = (U8 ? px * (1.0f / 255.0f) : px) * scale;  // I * 2^q
        if (k0) {
          v[0][c] = __float2int_rn(xs);
          v[1][c] = v[2][c] = v[3][c] = 0;
        } else {
          const float fr = phase_rev(f_hi, f_lo, px);
          const float C = __builtin_amdgcn_cosf(fr), S = __builtin_amdgcn_sinf(fr);
          v[0][c] = __float2int_rn(C * xs);
          v[1][c] = __float2int_rn(S * xs);
          v[2][c] = __float2int_rn(C * scale);
          v[3][c] = __float2int_rn(S * scale);
        }
      }
      const int j0 = 4 * lane + 256 * g;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (m >= nimg) break;
        v[m][1] += v[m][0];
        v[m][2] += v[m][1];
        v[m][3] += v[m][2];
        const int incl = wave_inclusive_scan(v[m][3]);
        const int excl = incl - v[m][3] + carry[m];
        carry[m] += __builtin_amdgcn_readlane(incl, 63);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[m][g][c] += v[m][c] + excl;
        if (j0 < p.pitch)
          *reinterpret_cast<int4 *>(row + m * te + j0) =
              make_int4(acc[m][g][0], acc[m][g][1], acc[m][g][2], acc[m][g][3]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// K-B: taps, accumulation over range terms, normalisation.
// Block 64 x 4 pixels, never straddling a tile (tile % 64 == 0).  Table reads
// are raw buffer loads: the per-thread byte offset stays in a VGPR and the
// per-tap / per-image offset is a uniform scalar, so addressing costs no
// vector instructions; loads out of the tile's table range return 0.  Blocks
// whose taps all fall inside the image take the unclamped path; border
// blocks clamp every tap to [0, H] x [0, W].
// ---------------------------------------------------------------------------
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  // raw buffer (stride 0), word 3 = 0x00020000 on gfx9-family targets
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ int load_i32(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return (int)__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
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
  const bool interior = by0 + tab->tap_dy_min >= 0 && by0 + 3 + tab->tap_dy_max <= p.H &&
                        bx0 + tab->tap_dx_min >= 0 && bx0 + 63 + tab->tap_dx_max <= p.W;
  const uint32_t te4 = (uint32_t)p.table_elems * 4u;
  const __amdgpu_buffer_rsrc_t rsrc =
      make_rsrc(ws + (long long)tile_id * p.n_images * p.table_elems, te4 * (uint32_t)p.n_images);
  const int n4 = tab->n_taps4;
  const int yr = y - oy, xr = x - ox;
  // interior: the thread's offset at tap (dy_min, dx_min); each tap adds the
  // uniform, non-negative (dy - dy_min) * pitch + dx - dx_min
  const int dy0 = tab->tap_dy_min, dx0 = tab->tap_dx_min;
  const uint32_t voff0 = (uint32_t)((yr + dy0) * p.pitch + xr + dx0) * 4u;
  auto tap_soff = [&](int i) {
    return (uint32_t)((tab->tap_dy[i] - dy0) * p.pitch + (tab->tap_dx[i] - dx0)) * 4u;
  };

  float px, xv;
  load_pixel<U8>(I, (long long)y * p.W + x, &px, &xv);
  const double inv = p.inv_sat_scale;
  double num = 0.0, den = 0.0;
  for (int t = 0; t < p.n_terms; ++t) {
    const uint32_t sb = (uint32_t)tab->slot[t] * te4;
    const double a = tab->a[t];
    if (tab->k_is_zero[t]) {
      // numerator a_0 (K * I); denominator a_0 (K * 1) from the clamped corner
      // coordinates (the table of ones is (Y - oy)(X - ox))
      double c0 = 0.0, d0 = 0.0;
      for (int i = 0; i < n4; ++i) {
        const int Y = min(max(y + tab->tap_dy[i], 0), p.H) - oy;
        const int X = min(max(x + tab->tap_dx[i], 0), p.W) - ox;
        const double w = tab->tap_w[i];
        const int v = interior ? load_i32(rsrc, voff0, sb + tap_soff(i))
                               : load_i32(rsrc, (uint32_t)(Y * p.pitch + X) * 4u, sb);
        c0 = __builtin_fma(w, (double)v, c0);
        d0 = __builtin_fma(w, (double)(Y * X), d0);
      }
      num = __builtin_fma(a, c0 * inv, num);
      den = __builtin_fma(a, d0, den);
      continue;
    }
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (interior) {
      for (int i = 0; i < n4; i += 4) {
        int v[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t so = sb + tap_soff(i + j);
#pragma unroll
          for (int m = 0; m < 4; ++m) v[j][m] = load_i32(rsrc, voff0, so + (uint32_t)m * te4);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double w = tab->tap_w[i + j];
          s0 = __builtin_fma(w, (double)v[j][0], s0);
          s1 = __builtin_fma(w, (double)v[j][1], s1);
          s2 = __builtin_fma(w, (double)v[j][2], s2);
          s3 = __builtin_fma(w, (double)v[j][3], s3);
        }
      }
    } else {
      for (int i = 0; i < n4; i += 4) {
        int v[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int Y = min(max(y + tab->tap_dy[i + j], 0), p.H) - oy;
          const int X = min(max(x + tab->tap_dx[i + j], 0), p.W) - ox;
          const uint32_t vo = (uint32_t)(Y * p.pitch + X) * 4u;
#pragma unroll
          for (int m = 0; m < 4; ++m) v[j][m] = load_i32(rsrc, vo, sb + (uint32_t)m * te4);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double w = tab->tap_w[i + j];
          s0 = __builtin_fma(w, (double)v[j][0], s0);
          s1 = __builtin_fma(w, (double)v[j][1], s1);
          s2 = __builtin_fma(w, (double)v[j][2], s2);
          s3 = __builtin_fma(w, (double)v[j][3], s3);
        }
      }
    }
    const float fr = phase_rev(tab->f_hi[t], tab->f_lo[t], px);
    const double C = (double)__builtin_amdgcn_cosf(fr), S = (double)__builtin_amdgcn_sinf(fr);
    num = __builtin_fma(a * inv, C * s0 + S * s1, num);
    den = __builtin_fma(a * inv, C * s2 + S * s3, den);
  }
  const long long idx = (long long)y * p.W + x;
  out[idx] = den > tab->den_floor ? (float)(num / den) : xv;
  if (num_out) num_out[idx] = (float)num;
  if (den_out) den_out[idx] = (float)den;
}

// ---------------------------------------------------------------------------
// K-B (LDS tile form): one block per 64 x 64 output tile; tables are the
// outer loop.  For each table the block copies the region its taps read --
// (64 + dy span) rows x (64 + dx span) columns, border clamp applied through
// the per-lane source columns -- from the workspace straight into LDS with
// buffer-to-LDS loads (no registers, no vector instructions), then every
// pixel reads its taps from LDS.  Symmetric quadruplets of taps are one box
// sum differenced exactly in int32 and one FP64 FMA.  Each thread owns the
// pixels (wave + 16 i, lane), i < 4, of the tile: one precomputed LDS address
// per quadruplet corner serves all four through instruction offsets.  When
// two regions fit in LDS they are double-buffered with their rows
// interleaved (row r of buffer b at (2r + b) * PITCH), so the second buffer
// is an instruction offset too and each table costs one barrier; the copy of
// table m + 1 runs while table m is read.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void_t;

__device__ __forceinline__ int lds_ld(const int *lds, uint32_t byte_addr) {
  return *reinterpret_cast<const int *>(reinterpret_cast<const char *>(lds) + byte_addr);
}

template <int PITCH, int NQ, bool DB, bool U8>
__global__ __launch_bounds__(1024) void kb_tile(const void *__restrict__ I, ImageParams p,
                                               const DevTables *__restrict__ tab,
                                               const int32_t *__restrict__ ws,
                                               float *__restrict__ out, float *__restrict__ num_out,
                                               float *__restrict__ den_out) {
  constexpr int NW = 16;                          // waves
  constexpr int PX = 64 / NW;                     // rows of the tile per thread
  constexpr int RS = DB ? 2 * PITCH : PITCH;      // LDS row stride (int32 elements)
  constexpr int CC = (PITCH + 63) / 64;           // 64-column chunks of a staged row
  constexpr uint32_t PSTEP = NW * RS * 4;         // bytes between a thread's pixels
  constexpr uint32_t BSTEP = PITCH * 4;           // bytes from buffer 0 to buffer 1
  extern __shared__ int lds[];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // XCD-aware order: blocks are dispatched round-robin over the 8 XCDs, so
  // XCD k (blockIdx % 8) takes the k-th contiguous eighth of the tiles, walked
  // in patches of 8 x 4 tiles; the tiles one XCD runs at the same time are
  // neighbours whose staged halos overlap in that XCD's L2.
  const int ntx = (p.W + 63) / 64, nty = (p.H + 63) / 64;
  const int n_tiles = ntx * nty;
  const int per_xcd = (n_tiles + 7) / 8;
  const int L = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (L >= n_tiles) return;
  // patch rows of PH tile rows (the last may be shorter); within one, patches
  // of PW tile columns (the last may be narrower); tiles row-major in a patch
  constexpr int PW = 8, PH = 4;
  const int pr = L / (PH * ntx);
  const int rem = L - pr * PH * ntx;
  const int ph = min(PH, nty - pr * PH);
  const int pc = rem / (PW * ph);
  const int in = rem - pc * PW * ph;
  const int pw = min(PW, ntx - pc * PW);
  const int bx = pc * PW + in % pw, by = pr * PH + in / pw;
  const int x0 = bx * 64, y0 = by * 64;
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

  // staging: wave w copies region rows w, w + NW, ...; lane l columns l,
  // l + 64, ...  The clamped source column is fixed per lane (vector offset),
  // the table and row part is wave-uniform (scalar offset), the LDS target is
  // the wave-uniform row start plus 4 bytes per lane.
  uint32_t xoff4[CC];
#pragma unroll
  for (int c = 0; c < CC; ++c) xoff4[c] = (uint32_t)(min(max(x0 + dx0 + lane + 64 * c, 0), p.W) - ox) * 4u;
  const uint32_t gp4 = (uint32_t)p.pitch * 4u;
  auto stage = [&](int m, int buf) {
    const uint32_t sm = (uint32_t)m * te4;
    for (int r = wave; r < RH; r += NW) {
      const int Y = min(max(y0 + dy0 + r, 0), p.H) - oy;
      const uint32_t soff = sm + (uint32_t)Y * gp4;
      int *dst = lds + r * RS + buf * PITCH;
#pragma unroll
      for (int c = 0; c < CC; ++c)
        if (lane + 64 * c < RW)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void_t *)(dst + 64 * c), 4, xoff4[c], soff, 0, 0);
    }
  };

  // LDS byte address of each quadruplet corner for this thread's pixel 0 in
  // buffer 0: region row r holds image row y0 + dy0 + r, so tap (dy, dx) of
  // the pixel in tile row wave, column lane is at element
  // (wave + dy - dy0) * RS + lane + dx - dx0.  Padding quadruplets read one
  // valid element four times with weight 0.
  const uint32_t lb = (uint32_t)(wave * RS + lane) * 4u;
  const int nq = tab->n_quads;
  uint32_t qa[NQ][4];
  double qw[NQ];
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
      qw[q] = 0.0;
    }
  }

  float pxv[PX];
  double num[PX], den[PX];
#pragma unroll
  for (int i = 0; i < PX; ++i) {
    const int y = y0 + wave + NW * i;
    pxv[i] = 0.0f;
    if (xin && y < p.H) {
      float px, v;
      load_pixel<U8>(I, (long long)y * p.W + x, &px, &v);
      pxv[i] = px;
    }
    num[i] = 0.0;
    den[i] = 0.0;
  }
  const double inv = p.inv_sat_scale;
  float cs[PX], sn[PX];

  // one table: box sums of every quadruplet (and lone taps), then the fold of
  // Eq. 1D_N_terms into the numerator / denominator
  auto body = [&](int m, auto BUF) {
    constexpr uint32_t bo = decltype(BUF)::value * BSTEP;
    const int t = tab->slot_term[m], part = tab->slot_part[m];
    if (part == 0) {
#pragma unroll
      for (int i = 0; i < PX; ++i) {
        const float fr = phase_rev(tab->f_hi[t], tab->f_lo[t], pxv[i]);
        cs[i] = __builtin_amdgcn_cosf(fr);
        sn[i] = __builtin_amdgcn_sinf(fr);
      }
    }
    double s[PX];
#pragma unroll
    for (int i = 0; i < PX; ++i) s[i] = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
#pragma unroll
      for (int i = 0; i < PX; ++i) {
        const uint32_t o = i * PSTEP + bo;
        const int box = (lds_ld(lds, qa[q][0] + o) - lds_ld(lds, qa[q][1] + o)) -
                        (lds_ld(lds, qa[q][2] + o) - lds_ld(lds, qa[q][3] + o));
        s[i] = __builtin_fma(qw[q], (double)box, s[i]);
      }
    }
    for (int q = 0; q < tab->n_single; ++q) {
      const uint32_t a =
          lb + (uint32_t)((tab->single_dy[q] - dy0) * RS + tab->single_dx[q] - dx0) * 4u + bo;
      const double w = tab->single_w[q];
#pragma unroll
      for (int i = 0; i < PX; ++i) s[i] = __builtin_fma(w, (double)lds_ld(lds, a + i * PSTEP), s[i]);
    }
    const double ai = tab->a[t] * inv;
#pragma unroll
    for (int i = 0; i < PX; ++i) {
      if (part == 4) {
        num[i] = __builtin_fma(ai, s[i], num[i]);
      } else if (part == 0) {
        num[i] = __builtin_fma(ai * cs[i], s[i], num[i]);
      } else if (part == 1) {
        num[i] = __builtin_fma(ai * sn[i], s[i], num[i]);
      } else if (part == 2) {
        den[i] = __builtin_fma(ai * cs[i], s[i], den[i]);
      } else {
        den[i] = __builtin_fma(ai * sn[i], s[i], den[i]);
      }
    }
    if (part == 4) {
      // denominator of the k = 0 term: a_0 (K * 1) from the clamped corners
      // (the table of ones is (Y - oy)(X - ox))
#pragma unroll
      for (int i = 0; i < PX; ++i) {
        const int y = y0 + wave + NW * i;
        double d0 = 0.0;
        for (int q = 0; q < tab->n_taps4; ++q) {
          const int Y = min(max(y + tab->tap_dy[q], 0), p.H) - oy;
          const int X = min(max(x + tab->tap_dx[q], 0), p.W) - ox;
          d0 = __builtin_fma(tab->tap_w[q], (double)(Y * X), d0);
        }
        den[i] = __builtin_fma(tab->a[t], d0, den[i]);
      }
    }
  };

  const int n = p.n_images;
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
    const int y = y0 + wave + NW * i;
    if (!xin || y >= p.H) continue;
    const long long idx = (long long)y * p.W + x;
    const float xv = U8 ? pxv[i] * (1.0f / 255.0f) : pxv[i];
    out[idx] = den[i] > tab->den_floor ? (float)(num[i] / den[i]) : xv;
    if (num_out) num_out[idx] = (float)num[i];
    if (den_out) den_out[idx] = (float)den[i];
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <bool U8>
static hipError_t launch_ka(int G, dim3 grid, dim3 block, hipStream_t s, const void *I,
                            ImageParams p, const DevTables *tab, int32_t *ws) {
  switch (G) {
    case 1: hipLaunchKernelGGL((ka_sat<1, U8>), grid, block, 0, s, I, p, tab, ws); break;
    case 2: hipLaunchKernelGGL((ka_sat<2, U8>), grid, block, 0, s, I, p, tab, ws); break;
    case 3: hipLaunchKernelGGL((ka_sat<3, U8>), grid, block, 0, s, I, p, tab, ws); break;
    case 4: hipLaunchKernelGGL((ka_sat<4, U8>), grid, block, 0, s, I, p, tab, ws); break;
    case 5: hipLaunchKernelGGL((ka_sat<5, U8>), grid, block, 0, s, I, p, tab, ws); break;
    case 6: hipLaunchKernelGGL((ka_sat<6, U8>), grid, block, 0, s, I, p, tab, ws); break;
    case 7: hipLaunchKernelGGL((ka_sat<7, U8>), grid, block, 0, s, I, p, tab, ws); break;
    default: hipLaunchKernelGGL((ka_sat<8, U8>), grid, block, 0, s, I, p, tab, ws); break;
  }
  return hipGetLastError();
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
static bool kb_double_buffered(const DevTables &h) {
  return h.lds_pitch == 128 && 2 * kb_region_bytes(h) <= 160 * 1024;
}

template <int PITCH, int NQ, bool DB, bool U8>
static hipError_t launch_kb_tile(dim3 grid, size_t lds, hipStream_t s, const void *I,
                                 ImageParams p, const DevTables *tab, const int32_t *ws, float *out,
                                 float *num, float *den) {
  auto k = kb_tile<PITCH, NQ, DB, U8>;
  hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, grid, dim3(1024), lds, s, I, p, tab, ws, out, num, den);
  return hipGetLastError();
}

template <int PITCH, bool DB, bool U8>
static hipError_t launch_kb_tile_nq(int nq, dim3 grid, size_t lds, hipStream_t s, const void *I,
                                    ImageParams p, const DevTables *tab, const int32_t *ws,
                                    float *out, float *num, float *den) {
  if (nq <= 4) return launch_kb_tile<PITCH, 4, DB, U8>(grid, lds, s, I, p, tab, ws, out, num, den);
  if (nq <= 8) return launch_kb_tile<PITCH, 8, DB, U8>(grid, lds, s, I, p, tab, ws, out, num, den);
  return launch_kb_tile<PITCH, 12, DB, U8>(grid, lds, s, I, p, tab, ws, out, num, den);
}

template <bool U8>
static hipError_t launch_kb_tile_any(const DevTables &h, dim3 grid, hipStream_t s, const void *I,
                                     ImageParams p, const DevTables *tab, const int32_t *ws,
                                     float *out, float *num, float *den) {
  const size_t lds = kb_region_bytes(h);
  const int nq = h.n_quads;
  if (kb_double_buffered(h))
    return launch_kb_tile_nq<128, true, U8>(nq, grid, 2 * lds, s, I, p, tab, ws, out, num, den);
  switch (h.lds_pitch) {
    case 128: return launch_kb_tile_nq<128, false, U8>(nq, grid, lds, s, I, p, tab, ws, out, num, den);
    case 160: return launch_kb_tile_nq<160, false, U8>(nq, grid, lds, s, I, p, tab, ws, out, num, den);
    case 176: return launch_kb_tile_nq<176, false, U8>(nq, grid, lds, s, I, p, tab, ws, out, num, den);
    default: return launch_kb_tile_nq<192, false, U8>(nq, grid, lds, s, I, p, tab, ws, out, num, den);
  }
}

void choose_tiling(int H, int W, int radius, int n_terms, int fixed_tile, double gmax, int *tile,
                   int *sat_shift) {
  int t = fixed_tile;
  if (!t) {
    t = 64;
    for (int c : {512, 256, 128, 64}) {
      if (c + 2 * radius + 1 > 768) continue;
      const long long waves = (long long)((H + c - 1) / c) * ((W + c - 1) / c) * n_terms;
      t = c;
      if (waves >= 2048) break;
    }
  }
  const double E = t + 2.0 * radius;
  int q = (int)std::floor(std::log2(2147483647.0 / (E * E * gmax)));
  *tile = t;
  *sat_shift = std::max(0, std::min(24, q));
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
  g.bytes = (size_t)g.tiles_y * g.tiles_x * n_images * g.table_elems * sizeof(int32_t);
  return g;
}

bf_status_t launch_filter(const DevTables *dev, const DevTables &host, const Geometry &g,
                          const void *I, float *out, float *num, float *den, int32_t *ws,
                          void *stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
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
  p.inv_sat_scale = std::ldexp(1.0, -g.sat_shift);
  const int Ew = std::min(g.tile + 2 * g.radius + 1, g.W + 1);
  const int G = (Ew + 255) / 256;
  if (G > kMaxChunks) return BF_ERR_UNSUPPORTED;
  dim3 ga(g.tiles_y * g.tiles_x, (host.n_terms + 3) / 4), ba(256);
  profile_mark(0, 1, stream);
  hipError_t e = host.in_u8 ? launch_ka<true>(G, ga, ba, s, I, p, dev, ws)
                            : launch_ka<false>(G, ga, ba, s, I, p, dev, ws);
  profile_mark(0, 0, stream);
  if (e != hipSuccess) return BF_ERR_DEVICE;
  // LDS tile kernel when the staged region fits and the quadruplets' corner
  // addresses fit in registers, else the per-pixel kernel
  profile_mark(1, 1, stream);
  if (host.lds_pitch > 0 && kb_region_bytes(host) <= 160 * 1024 && host.n_quads <= 12) {
    const int n_tiles = ((g.W + 63) / 64) * ((g.H + 63) / 64);
    dim3 gt(8 * ((n_tiles + 7) / 8));
    e = host.in_u8 ? launch_kb_tile_any<true>(host, gt, s, I, p, dev, ws, out, num, den)
                   : launch_kb_tile_any<false>(host, gt, s, I, p, dev, ws, out, num, den);
  } else {
    dim3 gb((g.W + 63) / 64, (g.H + 3) / 4), bb(256);
    e = host.in_u8 ? launch_kb<true>(gb, bb, s, I, p, dev, ws, out, num, den)
                   : launch_kb<false>(gb, bb, s, I, p, dev, ws, out, num, den);
  }
  profile_mark(1, 0, stream);
  return e == hipSuccess ? BF_OK : BF_ERR_DEVICE;
}

}  // namespace bf
