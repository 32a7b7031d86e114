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

#include "bf_internal.h"

namespace bf {

// Per-launch scalars of one image.
struct ImageParams {
  int H, W, tile, radius, tiles_x, n_images, pitch, n_terms;
  long long table_elems;
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

__device__ __forceinline__ int quantize(float v, float gmax, float scale) {
  v = fminf(fmaxf(v, -gmax), gmax);
  return __float2int_rn(v * scale);
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_inclusive_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

// ---------------------------------------------------------------------------
// K-A: tile-relative int32 summed-area tables of the term images of one k.
// Block: one tile x one term; thread t owns table columns [t*CPT, t*CPT+CPT).
// ---------------------------------------------------------------------------
template <int CPT, bool U8>
__global__ __launch_bounds__(512) void ka_sat(const void *__restrict__ I, ImageParams p,
                                             const DevTables *__restrict__ tab,
                                             int32_t *__restrict__ ws) {
  __shared__ int wave_tot[2][8][4];
  const int tile_id = blockIdx.x;
  const int term = blockIdx.y;
  const int ty = tile_id / p.tiles_x, tx = tile_id - ty * p.tiles_x;
  const int y0 = ty * p.tile, x0 = tx * p.tile;
  const int y1 = min(p.H, y0 + p.tile), x1 = min(p.W, x0 + p.tile);
  const int oy = max(y0 - p.radius, 0), ox = max(x0 - p.radius, 0);
  const int Eh = min(y1 + p.radius, p.H) - oy + 1;
  const int Ew = min(x1 + p.radius, p.W) - ox + 1;
  const bool k0 = tab->k_is_zero[term] != 0;
  const int nimg = k0 ? 1 : 4;
  int32_t *base = ws + ((long long)tile_id * p.n_images + tab->slot[term]) * p.table_elems;
  const float f_hi = tab->f_hi[term], f_lo = tab->f_lo[term];
  const float gmax = tab->gmax, scale = tab->sat_scale;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nwaves = blockDim.x >> 6;
  const int c0 = threadIdx.x * CPT;

  int acc[4][CPT];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int c = 0; c < CPT; ++c) acc[m][c] = 0;

  // row 0 of every table is zero
  for (int m = 0; m < nimg; ++m)
#pragma unroll
    for (int c = 0; c < CPT; ++c)
      if (c0 + c < Ew) base[(long long)m * p.table_elems + c0 + c] = 0;

  for (int i = 1; i < Eh; ++i) {
    const int yy = oy + i - 1;
    int v[4][CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int j = c0 + c;
      if (j >= 1 && j < Ew) {
        float px, x;
        load_pixel<U8>(I, (long long)yy * p.W + (ox + j - 1), &px, &x);
        if (k0) {
          v[0][c] = quantize(x, gmax, scale);
          v[1][c] = v[2][c] = v[3][c] = 0;
        } else {
          const float fr = phase_rev(f_hi, f_lo, px);
          const float C = __builtin_amdgcn_cosf(fr), S = __builtin_amdgcn_sinf(fr);
          v[0][c] = quantize(C * x, gmax, scale);
          v[1][c] = quantize(S * x, gmax, scale);
          v[2][c] = quantize(C, gmax, scale);
          v[3][c] = quantize(S, gmax, scale);
        }
      } else {
        v[0][c] = v[1][c] = v[2][c] = v[3][c] = 0;
      }
    }
    // in-thread inclusive prefix, wave scan of thread totals, cross-wave carry
    int tot[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
      for (int c = 1; c < CPT; ++c) v[m][c] += v[m][c - 1];
      const int incl = wave_inclusive_scan(v[m][CPT - 1]);
      tot[m] = incl - v[m][CPT - 1];  // exclusive within the wave
      if (lane == 63) wave_tot[i & 1][wave][m] = incl;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      int carry = 0;
      for (int w = 0; w < wave; ++w) carry += wave_tot[i & 1][w][m];
      tot[m] += carry;
    }
    (void)nwaves;
    int32_t *row = base + (long long)i * p.pitch;
    for (int m = 0; m < nimg; ++m) {
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        acc[m][c] += v[m][c] + tot[m];
        if (c0 + c < Ew) row[(long long)m * p.table_elems + c0 + c] = acc[m][c];
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
  // interior: element offset of the tap with the smallest dy * pitch + dx
  const uint32_t voff0 = (uint32_t)(yr * p.pitch + xr + tab->tap_d_min) * 4u;

  float px, xv;
  load_pixel<U8>(I, (long long)y * p.W + x, &px, &xv);
  const double inv = tab->inv_sat_scale;
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
        const int v = interior ? load_i32(rsrc, voff0, sb + (uint32_t)tab->tap_boff[i])
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
          const uint32_t so = sb + (uint32_t)tab->tap_boff[i + j];
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
// Host launchers
// ---------------------------------------------------------------------------
template <bool U8>
static hipError_t launch_ka(int cpt, dim3 grid, dim3 block, hipStream_t s, const void *I,
                            ImageParams p, const DevTables *tab, int32_t *ws) {
  switch (cpt) {
    case 1: hipLaunchKernelGGL((ka_sat<1, U8>), grid, block, 0, s, I, p, tab, ws); break;
    case 2: hipLaunchKernelGGL((ka_sat<2, U8>), grid, block, 0, s, I, p, tab, ws); break;
    case 4: hipLaunchKernelGGL((ka_sat<4, U8>), grid, block, 0, s, I, p, tab, ws); break;
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

Geometry make_geometry(int H, int W, int tile, int radius, int n_images) {
  Geometry g;
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
  const int Ew = std::min(g.tile + 2 * g.radius + 1, g.W + 1);
  int cpt = 1;
  while (cpt < 8 && (Ew + cpt - 1) / cpt > 512) cpt *= 2;
  int threads = (Ew + cpt - 1) / cpt;
  threads = (threads + 63) / 64 * 64;
  if (threads > 512) return BF_ERR_UNSUPPORTED;
  dim3 ga(g.tiles_y * g.tiles_x, host.n_terms), ba(threads);
  profile_mark(0, 1, stream);
  hipError_t e = host.in_u8 ? launch_ka<true>(cpt, ga, ba, s, I, p, dev, ws)
                            : launch_ka<false>(cpt, ga, ba, s, I, p, dev, ws);
  profile_mark(0, 0, stream);
  if (e != hipSuccess) return BF_ERR_DEVICE;
  dim3 gb((g.W + 63) / 64, (g.H + 3) / 4), bb(256);
  profile_mark(1, 1, stream);
  e = host.in_u8 ? launch_kb<true>(gb, bb, s, I, p, dev, ws, out, num, den)
                 : launch_kb<false>(gb, bb, s, I, p, dev, ws, out, num, den);
  profile_mark(1, 0, stream);
  return e == hipSuccess ? BF_OK : BF_ERR_DEVICE;
}

}  // namespace bf
