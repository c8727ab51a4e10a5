// Matrix-core evaluation of the operators (SL1M_PREC_MFMA_F16 / _BF16, delta
// pixels) for gfx950.
//
// With R right-hand sides (the paper's independent polarisations through one
// matrix, Section "Defining the direct solution") the forward is the product
// of the N_v x N_p matrix M with the N_p x R images and the adjoint
// Re(M^H r) that of the N_p x N_v matrix with the N_v x R residuals.  Both
// run on v_mfma_f32_4x4x4_16b: 16 blocks of D(4x4) += A(4x4) B(4x4), lane
// L = i + 4b holding row i of A of block b (four K values) and lane
// L = j + 4b column j of B and of D (D's four rows in its four registers).
// Here every block shares the same four K indices (pixels in the forward,
// visibilities in the adjoint) and the same B (the four sides of those four
// K values), so
//   * A row i of block b is the lane's own visibility (forward) or pixel
//     (adjoint): each lane forms its four entries of M from the FP64 phase
//     u l + v m + w (n - 1) exactly as the FP32 kernels do (FMAs from kMagic,
//     low mantissa bits into 1.0f, v_sin/v_cos in turns), the K index being
//     wavefront-uniform so that its coordinates are scalar loads;
//   * cos and sin of the entries are two A operands against one B
//     (forward: V_re = sum c x, V_im = -sum s x; adjoint: g = sum c r_re +
//     s (-r_im), the two products chained into one accumulator);
//   * D(b, i, j) of lane j + 4b is side j at visibility / pixel 4b + i.
// B is the per-call packed image or residual (power-of-two scaled into the
// operand range, rounded once), eight 4-value steps per lane loaded ahead of
// the 32-index block that uses them.  Partial rows and their reduction are
// those of the direct kernels: forward [side][chunk][n_vis] complex (pixel
// amplitudes inside), adjoint [side][chunk][n_pix] (amplitudes applied by
// the reduction).
#include "sl1m_grid.h"

namespace sl1m {

namespace {

using namespace dev;

constexpr int kMfmaRedBlocks = 256;  // blocks of the max-magnitude pass

typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// operand type: storage as 16-bit words, conversion, the MFMA
template <int PREC>
struct MOp;

template <>
struct MOp<SL1M_PREC_MFMA_F16> {
  typedef h4_t vec;
  static __device__ __forceinline__ f4_t mma(vec a, vec b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_4x4x4f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ uint16_t bits(float x) {
    return __builtin_bit_cast(uint16_t, static_cast<_Float16>(x));
  }
};

template <>
struct MOp<SL1M_PREC_MFMA_BF16> {
  typedef s4_t vec;
  static __device__ __forceinline__ f4_t mma(vec a, vec b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ uint16_t bits(float x) {
    return __builtin_bit_cast(uint16_t, static_cast<__bf16>(x));
  }
};

template <typename V>
__device__ __forceinline__ V as_vec(uint2 w) {
  return __builtin_bit_cast(V, w);
}

// Four float32 values to one operand (two v_cvt_pk per four values).
typedef __bf16 b4_t __attribute__((ext_vector_type(4)));
template <int PREC>
__device__ __forceinline__ typename MOp<PREC>::vec pack4(f4_t v) {
  if constexpr (PREC == SL1M_PREC_MFMA_F16)
    return __builtin_convertvector(v, h4_t);
  else
    return __builtin_bit_cast(s4_t, __builtin_convertvector(v, b4_t));
}

// Power of two s with max * s in [2^13, 2^14) (1 for a zero or non-finite
// maximum): operands stay inside float16's range with 2 bits of headroom for
// the rounding of the largest one.
__device__ __forceinline__ float op_scale(float mx) {
  if (!(mx > 0.0f) || !isfinite(mx)) return 1.0f;
  int ex;
  frexpf(mx, &ex);  // mx = f 2^ex, f in [0.5, 1)
  int e = 14 - ex;
  e = e < -120 ? -120 : (e > 120 ? 120 : e);
  return ldexpf(1.0f, e);
}

// Wavefront maximum through cross-lane shuffles, then the block's in LDS.
__device__ __forceinline__ float block_max(float v) {
  __shared__ float wm[kBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = v;
  __syncthreads();
  float m = wm[0];
#pragma unroll
  for (int w = 1; w < kBlock / 64; ++w) m = fmaxf(m, wm[w]);
  __syncthreads();
  return m;
}

// Block maxima of |x[r][j] scale[j]| (scale may be null: |x[i]|) over n values.
__global__ __launch_bounds__(kBlock) void k_mfma_absmax(const float* __restrict__ x, int64_t n,
                                                        const float* __restrict__ scale,
                                                        int64_t n_scale, float* __restrict__ out) {
  float m = 0.0f;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kBlock) {
    const float v = scale ? x[i] * scale[i % n_scale] : x[i];
    // a NaN counts as infinite (fmaxf would drop it): the scale falls back to 1
    m = fmaxf(m, v != v ? __builtin_inff() : fabsf(v));
  }
  m = block_max(m);
  if (threadIdx.x == 0) out[blockIdx.x] = m;
}

// The maximum of the kMfmaRedBlocks block maxima (every block of the packing
// kernels recomputes it; block 0 stores the inverse scale for the operator).
__device__ __forceinline__ float max_of_blocks(const float* __restrict__ bm) {
  static_assert(kMfmaRedBlocks == kBlock, "one block maximum per thread");
  const float v = bm[threadIdx.x];
  return block_max(v != v ? __builtin_inff() : v);
}

// Images: out[((g np4 + s) 4 + j) 4 + e] = x[4g + j][4s + e] scale[4s + e] c,
// zero past n_pix or nr.  One thread per (g, s, j).
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_mfma_pack_x(const float* __restrict__ x,
                                                        const float* __restrict__ scale,
                                                        int64_t n_pix, int nr, int64_t np4,
                                                        int ng, const float* __restrict__ bm,
                                                        float* __restrict__ inv_out,
                                                        uint16_t* __restrict__ out) {
  const float c = op_scale(max_of_blocks(bm));
  if (blockIdx.x == 0 && threadIdx.x == 0) *inv_out = 1.0f / c;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= static_cast<int64_t>(ng) * np4 * 4) return;
  const int j = static_cast<int>(t & 3);
  const int64_t s = (t >> 2) % np4;
  const int g = static_cast<int>((t >> 2) / np4);
  const int r = 4 * g + j;
  uint16_t w[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t px = 4 * s + e;
    const float v = (r < nr && px < n_pix) ? x[r * n_pix + px] * scale[px] * c : 0.0f;
    w[e] = MOp<PREC>::bits(v);
  }
  uint2 o;
  o.x = static_cast<uint32_t>(w[0]) | (static_cast<uint32_t>(w[1]) << 16);
  o.y = static_cast<uint32_t>(w[2]) | (static_cast<uint32_t>(w[3]) << 16);
  reinterpret_cast<uint2*>(out)[t] = o;
}

// Residual records rres[k][nr] (complex): out[(((g nv4 + s) 4 + j) 2 + h) 4 + e]
// = (h ? -Im : Re) rres[4s + e][4g + j] c, zero past n_vis or nr.
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_mfma_pack_r(const float2* __restrict__ rres,
                                                        int64_t n_vis, int nr, int64_t nv4,
                                                        int ng, const float* __restrict__ bm,
                                                        float* __restrict__ inv_out,
                                                        uint16_t* __restrict__ out) {
  const float c = op_scale(max_of_blocks(bm));
  if (blockIdx.x == 0 && threadIdx.x == 0) *inv_out = 1.0f / c;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= static_cast<int64_t>(ng) * nv4 * 4) return;
  const int j = static_cast<int>(t & 3);
  const int64_t s = (t >> 2) % nv4;
  const int g = static_cast<int>((t >> 2) / nv4);
  const int r = 4 * g + j;
  uint16_t re[4], im[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t k = 4 * s + e;
    float2 v = make_float2(0.0f, 0.0f);
    if (r < nr && k < n_vis) v = rres[k * nr + r];
    re[e] = MOp<PREC>::bits(v.x * c);
    im[e] = MOp<PREC>::bits(-v.y * c);
  }
  uint4 o;
  o.x = static_cast<uint32_t>(re[0]) | (static_cast<uint32_t>(re[1]) << 16);
  o.y = static_cast<uint32_t>(re[2]) | (static_cast<uint32_t>(re[3]) << 16);
  o.z = static_cast<uint32_t>(im[0]) | (static_cast<uint32_t>(im[1]) << 16);
  o.w = static_cast<uint32_t>(im[2]) | (static_cast<uint32_t>(im[3]) << 16);
  reinterpret_cast<uint4*>(out)[t] = o;
}

// Forward: a wavefront owns 64 VPL visibilities (lane L: wbase + 64 v + L,
// v < VPL, one A operand each, so every scalar pixel record feeds VPL
// entries per lane); blockIdx.y = pixel chunk [y pchunk, min((y + 1) pchunk,
// 4 np4)) in 32-pixel blocks (pchunk a multiple of 32).  Pixels past n_pix
// have zero images and zero records.
template <int PREC, int NG, int VPL>
__global__ __launch_bounds__(kBlock) void k_fwd_mfma(
    const PixRec<float>* __restrict__ pix, const uint16_t* __restrict__ xh, int64_t np4,
    const double* __restrict__ vu, const double* __restrict__ vv,
    const double* __restrict__ vw, int64_t n_vis, int64_t pchunk,
    const float* __restrict__ inv, float2* __restrict__ part, int n_rows, int nr) {
  typedef typename MOp<PREC>::vec V;
  const int lane = threadIdx.x & 63;
  const int64_t wbase =
      (static_cast<int64_t>(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6)) * (64 * VPL);
  double u[VPL], v[VPL], w[VPL];
#pragma unroll
  for (int q = 0; q < VPL; ++q) {
    const int64_t k = wbase + 64 * q + lane < n_vis ? wbase + 64 * q + lane : n_vis - 1;
    u[q] = vu[k];
    v[q] = vv[k];
    w[q] = vw[k];
  }
  const int jcol = lane & 3;
  const ConstPtr<PixRec<float>> cpix = as_const(pix);
  const uint2* xb = reinterpret_cast<const uint2*>(xh);
  const int64_t j0 = static_cast<int64_t>(blockIdx.y) * pchunk;
  const int64_t j1 = j0 + pchunk < 4 * np4 ? j0 + pchunk : 4 * np4;
  const double origin = kMagic;
  f4_t are[VPL][NG], aim[VPL][NG];
#pragma unroll
  for (int q = 0; q < VPL; ++q)
#pragma unroll
    for (int g = 0; g < NG; ++g) are[q][g] = aim[q][g] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
  for (int64_t jb = j0; jb < j1; jb += 32) {
    uint2 bw[NG][8];
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int s = 0; s < 8; ++s) bw[g][s] = xb[(g * np4 + jb / 4 + s) * 4 + jcol];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      f4_t cv[VPL], sv[VPL];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t jp = jb + 4 * s + e;  // records padded to 4 np4 (zeros)
        const double pl = cpix[jp].l, pm = cpix[jp].m, pn = cpix[jp].c3;
#pragma unroll
        for (int q = 0; q < VPL; ++q) {
          const double t = fma(w[q], pn, fma(v[q], pm, fma(u[q], pl, origin)));
          float c, sn;
          phasor(t, c, sn);
          cv[q][e] = c;
          sv[q][e] = -sn;
        }
      }
#pragma unroll
      for (int q = 0; q < VPL; ++q) {
        const V ac = pack4<PREC>(cv[q]), as = pack4<PREC>(sv[q]);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          const V b = as_vec<V>(bw[g][s]);
          are[q][g] = MOp<PREC>::mma(ac, b, are[q][g]);
          aim[q][g] = MOp<PREC>::mma(as, b, aim[q][g]);
        }
      }
    }
  }
  const float sc = *inv;
#pragma unroll
  for (int q = 0; q < VPL; ++q) {
    const int64_t kb = wbase + 64 * q + (lane & ~3);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int r = 4 * g + jcol;
      if (r >= nr) continue;
      float2* out = part + (static_cast<int64_t>(r) * n_rows + blockIdx.y) * n_vis;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (kb + i < n_vis) out[kb + i] = make_float2(are[q][g][i] * sc, aim[q][g][i] * sc);
    }
  }
}

// Adjoint: a wavefront owns 64 PPL pixels (lane L: wbase + 64 q + L),
// blockIdx.y = visibility chunk [y kchunk, min((y + 1) kchunk, 4 nv4)) in
// 32-visibility blocks.  Visibilities past n_vis have zero residuals and
// zero records.
template <int PREC, int NG, int PPL>
__global__ __launch_bounds__(kBlock) void k_adj_mfma(
    const VisRecD<float>* __restrict__ vrec, const uint16_t* __restrict__ rh, int64_t nv4,
    const double* __restrict__ pl, const double* __restrict__ pm,
    const double* __restrict__ pc3, int64_t n_pix, int64_t kchunk,
    const float* __restrict__ inv, float* __restrict__ part, int n_rows, int nr) {
  typedef typename MOp<PREC>::vec V;
  const int lane = threadIdx.x & 63;
  const int64_t wbase =
      (static_cast<int64_t>(blockIdx.x) * (kBlock / 64) + (threadIdx.x >> 6)) * (64 * PPL);
  double l[PPL], m[PPL], nu[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    const int64_t j = wbase + 64 * q + lane < n_pix ? wbase + 64 * q + lane : n_pix - 1;
    l[q] = pl[j];
    m[q] = pm[j];
    nu[q] = pc3[j];
  }
  const int jcol = lane & 3;
  const ConstPtr<VisRecD<float>> cvrec = as_const(vrec);
  const uint4* rb = reinterpret_cast<const uint4*>(rh);
  const int64_t k0 = static_cast<int64_t>(blockIdx.y) * kchunk;
  const int64_t k1 = k0 + kchunk < 4 * nv4 ? k0 + kchunk : 4 * nv4;
  const double origin = kMagic;
  f4_t acc[PPL][NG];
#pragma unroll
  for (int q = 0; q < PPL; ++q)
#pragma unroll
    for (int g = 0; g < NG; ++g) acc[q][g] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
  for (int64_t kb = k0; kb < k1; kb += 32) {
    uint4 bw[NG][8];
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int s = 0; s < 8; ++s) bw[g][s] = rb[(g * nv4 + kb / 4 + s) * 4 + jcol];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      f4_t cv[PPL], sv[PPL];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t kp = kb + 4 * s + e;  // records padded to 4 nv4 (zeros)
        const double u = cvrec[kp].u, v = cvrec[kp].v, w = cvrec[kp].w;
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          const double t = fma(w, nu[q], fma(v, m[q], fma(u, l[q], origin)));
          float c, sn;
          phasor(t, c, sn);
          cv[q][e] = c;
          sv[q][e] = sn;
        }
      }
#pragma unroll
      for (int q = 0; q < PPL; ++q) {
        const V ac = pack4<PREC>(cv[q]), as = pack4<PREC>(sv[q]);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          const uint4 b = bw[g][s];
          acc[q][g] = MOp<PREC>::mma(ac, as_vec<V>(make_uint2(b.x, b.y)), acc[q][g]);
          acc[q][g] = MOp<PREC>::mma(as, as_vec<V>(make_uint2(b.z, b.w)), acc[q][g]);
        }
      }
    }
  }
  const float sc = *inv;
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    const int64_t jb = wbase + 64 * q + (lane & ~3);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int r = 4 * g + jcol;
      if (r >= nr) continue;
      float* out = part + (static_cast<int64_t>(r) * n_rows + blockIdx.y) * n_pix;
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (jb + i < n_pix) out[jb + i] = acc[q][g][i] * sc;
    }
  }
}

// ---------------------------------------------------------------------------
// Square delta grids on the matrix cores (forward).  The grid evaluation of
// the FP32 kernels (sl1m_grid.h) writes the pair sum of a visibility as
//   Re = cc (m1 e1 + m2 e2 + m5 f1 + m6 f2) - cs (m3 e3 + m4 e4 + m7 f3 + m8 f4)
//   Im = -cs (m1 e1 + m2 e2 + m5 f1 + m6 f2) - cc (m3 e3 + m4 e4 + m7 f3 + m8 f4)
// with C = (cc, cs) the pair's radius phasor, m1..m8 the eight products of
// the A and B phasors of the cell and its mirror, and e1..e4, f1..f4 the
// sign combinations of the pair's amplitudes (one set per side).  So with
// the sixteen basis values b = (cc m1, cc m2, cc m5, cc m6 | -cs m3, -cs m4,
// -cs m7, -cs m8) for Re and (-cs m1, -cs m2, -cs m5, -cs m6 | -cc m3, -cc m4,
// -cc m7, -cc m8) for Im as A operands (the lane's visibility is its row) and
// the per-side vectors Be = (e1, e2, f1, f2), Bo = (e3, e4, f3, f4) as B
// operands (one per side, lane j + 4b holding side j), four 4 x 4 x 4 MFMAs
// per pair accumulate up to four sides: the VALU forms 16 basis values per
// pair whatever the side count, instead of 12 FP32 operations per pair and
// side.
// ---------------------------------------------------------------------------

// Per call: the pairs' amplitude combinations, scaled by the power of two c
// that brings 4 max|x scale| into [2^13, 2^14) (a combination adds at most
// four amplitudes), rounded to the operand type:
//   out[(g n_pairs + p) 4 + j] = (e1, e2, f1, f2 | e3, e4, f3, f4) of side 4g + j
// (zero past nr), and nu of each pair into pnu.  One thread per (g, p, j).
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_grid_mfma_pack_pairs(
    const float* __restrict__ xp, int64_t n_pix, int nr, const float* __restrict__ pscale,
    const int32_t* __restrict__ slot, const double* __restrict__ nu, int na, int64_t n_pairs,
    int ng, const float* __restrict__ bm, float* __restrict__ inv_out, double* __restrict__ pnu,
    uint4* __restrict__ out) {
  const float c = op_scale(4.0f * max_of_blocks(bm));
  if (blockIdx.x == 0 && threadIdx.x == 0) *inv_out = 1.0f / c;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= static_cast<int64_t>(ng) * n_pairs * 4) return;
  const int j = static_cast<int>(t & 3);
  const int64_t p = (t >> 2) % n_pairs;
  const int g = static_cast<int>((t >> 2) / n_pairs);
  const int r = 4 * g + j;
  float e[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  if (r < nr) {
    const PairSlots ps = grid_pair_slots(p, na, slot, xp + r * n_pix, pscale, c);
    const float* x = ps.x;
    const float* y = ps.y;
    e[0] = (x[0] + x[1]) + (x[2] + x[3]);  // e1
    e[1] = (x[1] + x[2]) - (x[0] + x[3]);  // e2
    e[2] = (y[0] + y[1]) + (y[2] + y[3]);  // f1
    e[3] = (y[1] + y[2]) - (y[0] + y[3]);  // f2
    e[4] = (x[0] + x[1]) - (x[2] + x[3]);  // e3
    e[5] = (x[0] - x[1]) + (x[2] - x[3]);  // e4
    e[6] = (y[0] + y[1]) - (y[2] + y[3]);  // f3
    e[7] = (y[0] - y[1]) + (y[2] - y[3]);  // f4
    if (r == 0) pnu[p] = nu[ps.q];
  }
  uint16_t w[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) w[i] = MOp<PREC>::bits(e[i]);
  uint4 o;
  o.x = static_cast<uint32_t>(w[0]) | (static_cast<uint32_t>(w[1]) << 16);
  o.y = static_cast<uint32_t>(w[2]) | (static_cast<uint32_t>(w[3]) << 16);
  o.z = static_cast<uint32_t>(w[4]) | (static_cast<uint32_t>(w[5]) << 16);
  o.w = static_cast<uint32_t>(w[6]) | (static_cast<uint32_t>(w[7]) << 16);
  out[t] = o;
}

// Forward: block (visibility tile of kBlock, pair chunk blockIdx.y), one
// visibility per lane as the lane's A row; partial row blockIdx.y of side r
// at part + (r n_rows + y) n_vis.  Lanes past n_vis evaluate the last
// visibility and write nothing.
template <int PREC, int NG>
__global__ __launch_bounds__(kBlock) void k_grid_fwd_pairs_mfma(
    const uint4* __restrict__ bh, const double* __restrict__ pnu, int64_t n_pairs,
    const double* __restrict__ la, const double* __restrict__ mb,
    const GridChunk* __restrict__ chunks, int na, const double* __restrict__ vu,
    const double* __restrict__ vv, const double* __restrict__ vw, int64_t n_vis,
    const float* __restrict__ inv, float2* __restrict__ part, int n_rows, int nr) {
  typedef typename MOp<PREC>::vec V;
  const int lane = threadIdx.x & 63;
  const int jcol = lane & 3;
  const ConstPtr<GridChunk> cch = as_const(chunks) + blockIdx.y;
  const int g0 = cch->g, ia0 = cch->ia0, ia1 = cch->ia1;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t kk = k < n_vis ? k : n_vis - 1;
  const double u = vu[kk], v = vv[kk], w = vw[kk];
  const ConstPtr<double> cla = as_const(la);
  const ConstPtr<double> cmb = as_const(mb);
  const ConstPtr<double> cnu = as_const(pnu);
  const double origin = kMagic;
  float bc[kGridNB], bs[kGridNB];  // B at |m|_b
  float pc[kGridNB], ps[kGridNB];  // A at |l|_b (the mirror's)
#pragma unroll
  for (int b = 0; b < kGridNB; ++b) {
    const double m = cmb[g0 * kGridNB + b];
    phasor(fma(v, m, origin), bc[b], bs[b]);
    phasor(fma(u, m, origin), pc[b], ps[b]);
  }
  f4_t are[NG], aim[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) are[g] = aim[g] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
  for (int ia = ia0; ia < ia1; ++ia) {
    const double l = cla[ia];
    float ac, as, qc, qs;  // A at |l|_ia, B at |m|_ia
    phasor(fma(u, l, origin), ac, as);
    phasor(fma(v, l, origin), qc, qs);
    const int64_t p0 = pair_rec_base(g0, na) + static_cast<int64_t>(ia - kGridNB * g0) * kGridNB;
#pragma unroll
    for (int b = 0; b < kGridNB; ++b) {
      float cc, cs;
      phasor(fma(w, cnu[p0 + b], origin), cc, cs);
      const float m1 = ac * bc[b], m2 = as * bs[b], m5 = pc[b] * qc, m6 = ps[b] * qs;
      const float m3 = ac * bs[b], m4 = as * bc[b], m7 = pc[b] * qs, m8 = ps[b] * qc;
      const float ncs = -cs, ncc = -cc;
      const V a1 = pack4<PREC>(f4_t{cc * m1, cc * m2, cc * m5, cc * m6});
      const V a2 = pack4<PREC>(f4_t{ncs * m3, ncs * m4, ncs * m7, ncs * m8});
      const V a3 = pack4<PREC>(f4_t{ncs * m1, ncs * m2, ncs * m5, ncs * m6});
      const V a4 = pack4<PREC>(f4_t{ncc * m3, ncc * m4, ncc * m7, ncc * m8});
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const uint4 bw = bh[(static_cast<int64_t>(g) * n_pairs + p0 + b) * 4 + jcol];
        const V be = as_vec<V>(make_uint2(bw.x, bw.y)), bo = as_vec<V>(make_uint2(bw.z, bw.w));
        are[g] = MOp<PREC>::mma(a1, be, are[g]);
        are[g] = MOp<PREC>::mma(a2, bo, are[g]);
        aim[g] = MOp<PREC>::mma(a3, be, aim[g]);
        aim[g] = MOp<PREC>::mma(a4, bo, aim[g]);
      }
    }
  }
  const float sc = *inv;
  const int64_t kb = static_cast<int64_t>(blockIdx.x) * kBlock + (threadIdx.x & ~3);
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int r = 4 * g + jcol;
    if (r >= nr) continue;
    float2* out = part + (static_cast<int64_t>(r) * n_rows + blockIdx.y) * n_vis;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (kb + i < n_vis) out[kb + i] = make_float2(are[g][i] * sc, aim[g][i] * sc);
  }
}

// The same forward for float16 operands with the basis formed in packed
// float16 arithmetic: the lane's A and B phasors at |l|_ia, the block's at
// |m|_b and each pair's C are rounded to float16 once, and the sixteen basis
// values of a pair are then four products of (cos, sin) halves (m1 m2 | m3 m4
// from A at ia against B at b and its swap, m5 m6 | m7 m8 from the mirror's)
// and eight products with C's components -- 12 v_pk_mul_f16 and one
// conversion per pair instead of 24 float32 products and 8 conversions.  Each
// basis value carries up to five float16 roundings (two inputs, two products,
// C) against one when formed in float32.
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
typedef float f2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ h2_t to_h2(float a, float b) {
  return __builtin_convertvector((f2_t{a, b}), h2_t);
}

__device__ __forceinline__ h4_t cat_h2(h2_t a, h2_t b) {
  return __builtin_shufflevector(a, b, 0, 1, 2, 3);
}

template <int NG>
__global__ __launch_bounds__(kBlock) void k_grid_fwd_pairs_mfma_h(
    const uint4* __restrict__ bh, const double* __restrict__ pnu, int64_t n_pairs,
    const double* __restrict__ la, const double* __restrict__ mb,
    const GridChunk* __restrict__ chunks, int na, const double* __restrict__ vu,
    const double* __restrict__ vv, const double* __restrict__ vw, int64_t n_vis,
    const float* __restrict__ inv, float2* __restrict__ part, int n_rows, int nr) {
  const int lane = threadIdx.x & 63;
  const int jcol = lane & 3;
  const ConstPtr<GridChunk> cch = as_const(chunks) + blockIdx.y;
  const int g0 = cch->g, ia0 = cch->ia0, ia1 = cch->ia1;
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t kk = k < n_vis ? k : n_vis - 1;
  const double u = vu[kk], v = vv[kk], w = vw[kk];
  const ConstPtr<double> cla = as_const(la);
  const ConstPtr<double> cmb = as_const(mb);
  const ConstPtr<double> cnu = as_const(pnu);
  const double origin = kMagic;
  h2_t bb[kGridNB], pp[kGridNB];  // (cos, sin) of B at |m|_b and of A at |l|_b
#pragma unroll
  for (int b = 0; b < kGridNB; ++b) {
    const double m = cmb[g0 * kGridNB + b];
    float c, s;
    phasor(fma(v, m, origin), c, s);
    bb[b] = to_h2(c, s);
    phasor(fma(u, m, origin), c, s);
    pp[b] = to_h2(c, s);
  }
  f4_t are[NG], aim[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) are[g] = aim[g] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
  for (int ia = ia0; ia < ia1; ++ia) {
    const double l = cla[ia];
    float c, s;
    phasor(fma(u, l, origin), c, s);
    const h2_t aa = to_h2(c, s);  // A at |l|_ia
    phasor(fma(v, l, origin), c, s);
    const h2_t qq = to_h2(c, s);  // B at |m|_ia
    const int64_t p0 = pair_rec_base(g0, na) + static_cast<int64_t>(ia - kGridNB * g0) * kGridNB;
#pragma unroll
    for (int b = 0; b < kGridNB; ++b) {
      float cc, cs;
      phasor(fma(w, cnu[p0 + b], origin), cc, cs);
      const h2_t ch = to_h2(cc, cs);
      const h2_t cx = ch.xx, cy = ch.yy;
      const h2_t m12 = aa * bb[b];           // (m1, m2)
      const h2_t m34 = aa * bb[b].yx;        // (m3, m4)
      const h2_t m56 = pp[b] * qq;           // (m5, m6)
      const h2_t m78 = pp[b] * qq.yx;        // (m7, m8)
      const h4_t a1 = cat_h2(cx * m12, cx * m56);
      const h4_t a2 = cat_h2(-(cy * m34), -(cy * m78));
      const h4_t a3 = cat_h2(-(cy * m12), -(cy * m56));
      const h4_t a4 = cat_h2(-(cx * m34), -(cx * m78));
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const uint4 bw = bh[(static_cast<int64_t>(g) * n_pairs + p0 + b) * 4 + jcol];
        const h4_t be = as_vec<h4_t>(make_uint2(bw.x, bw.y)), bo = as_vec<h4_t>(make_uint2(bw.z, bw.w));
        are[g] = __builtin_amdgcn_mfma_f32_4x4x4f16(a1, be, are[g], 0, 0, 0);
        are[g] = __builtin_amdgcn_mfma_f32_4x4x4f16(a2, bo, are[g], 0, 0, 0);
        aim[g] = __builtin_amdgcn_mfma_f32_4x4x4f16(a3, be, aim[g], 0, 0, 0);
        aim[g] = __builtin_amdgcn_mfma_f32_4x4x4f16(a4, bo, aim[g], 0, 0, 0);
      }
    }
  }
  const float sc = *inv;
  const int64_t kb = static_cast<int64_t>(blockIdx.x) * kBlock + (threadIdx.x & ~3);
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    const int r = 4 * g + jcol;
    if (r >= nr) continue;
    float2* out = part + (static_cast<int64_t>(r) * n_rows + blockIdx.y) * n_vis;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (kb + i < n_vis) out[kb + i] = make_float2(are[g][i] * sc, aim[g][i] * sc);
  }
}

// ---------------------------------------------------------------------------
// Square delta grids on the matrix cores (adjoint, float16).  The pair
// adjoint of the FP32 grid kernels accumulates, per cell pair and side, the
// eight sums G_a = sum_k p_a(k) z_a(k) with p_1..p_8 the products of the A
// and B phasors of the cell and its mirror (m1, m2, m3, m4, m5, m6, m7, m8
// of the forward above) and, with C = (cc, cs) the pair's radius phasor and
// r_k the residual record,
//   z_a = cc Re r - cs Im r  (a = 1, 2, 5, 6),  z_a = cs Re r + cc Im r  (else).
// So G_a contracts over (visibility, Re / Im) the basis (p_a cc, -p_a cs) or
// (p_a cs, p_a cc) with the residual's (Re r, Im r): one 4 x 4 x 4 MFMA per
// sum and two visibilities, its K the two visibilities' (Re, Im).  Lane
// L = i + 4b gives A row i of block b (the basis of its own cell pair), B
// column j of every block is side j's residual (lane j + 4b), and D column j
// in lane j + 4b ends as G_a of the four pairs of lanes 4b .. 4b + 3 for
// side j, which that lane writes.  The basis is formed in packed float16 as
// in the forward; the residual records are scaled by a power of two per call
// and rounded once.
// ---------------------------------------------------------------------------

// Residual records for the contraction: out[(kp ng + g) 4 + j] = (Re r, Im r)
// of visibilities 2 kp and 2 kp + 1 of side 4 g + j, times c, as float16
// (zero past n_vis or nr).  One thread per (kp, g, j).
__global__ __launch_bounds__(kBlock) void k_grid_mfma_pack_res(
    const float2* __restrict__ rres, int64_t n_vis, int nr, int64_t n_kp, int ng,
    const float* __restrict__ bm, float* __restrict__ inv_out, uint2* __restrict__ out) {
  const float c = op_scale(max_of_blocks(bm));
  if (blockIdx.x == 0 && threadIdx.x == 0) *inv_out = 1.0f / c;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (t >= n_kp * ng * 4) return;
  const int j = static_cast<int>(t & 3);
  const int g = static_cast<int>((t >> 2) % ng);
  const int64_t kp = (t >> 2) / ng;
  const int r = 4 * g + j;
  float2 v0 = make_float2(0.0f, 0.0f), v1 = make_float2(0.0f, 0.0f);
  if (r < nr) {
    if (2 * kp < n_vis) v0 = rres[2 * kp * nr + r];
    if (2 * kp + 1 < n_vis) v1 = rres[(2 * kp + 1) * nr + r];
  }
  const h4_t h = __builtin_convertvector((f4_t{v0.x * c, v0.y * c, v1.x * c, v1.y * c}), h4_t);
  out[t] = __builtin_bit_cast(uint2, h);
}

// Block (pair block x, visibility chunk y, cell slice z): the NBI cells
// b = kGridNBA g4 + bo + bi (bo = z NBI) of each lane-set, as the FP32 pair
// adjoint; side r of chunk y goes to part + r rstride + y n_pix.  Every
// thread runs the whole loop (the MFMAs are wavefront-wide): lanes past the
// block's lane-sets evaluate a dummy pair and write nothing.
template <int NG, int NBI>
__global__ __launch_bounds__(kBlock) void k_grid_adj_pairs_mfma_h(
    const VisRecD<float>* __restrict__ vrec, const uint2* __restrict__ rh,
    const double* __restrict__ vu, const double* __restrict__ vv, const double* __restrict__ la,
    const double* __restrict__ mb, const double* __restrict__ nu,
    const int32_t* __restrict__ slot, int na, const GridPairBlock* __restrict__ blocks,
    int64_t kchunk, int64_t n_vis, const float* __restrict__ inv, float* __restrict__ part,
    int64_t n_pix, int64_t rstride, int nr) {
  static_assert(kGridNBA % NBI == 0, "NBI divides the cells of a lane-set");
  constexpr int KB = kGridKBM;  // visibilities per LDS batch (even)
  __shared__ uint2 bsh[KB][kGridMaxGL][NBI];  // (B, A) at |m|_b as float16 pairs
  const ConstPtr<GridPairBlock> cb = as_const(blocks) + blockIdx.x;
  GridPairBlock pb;
  pb.g4 = cb->g4;
  pb.ia = cb->ia;
  pb.count = cb->count;
  pb.n_gl = cb->n_gl;
  const int bo = static_cast<int>(blockIdx.z) * NBI;
  const PairLane pl = pair_lane(pb, na);
  const int lane = threadIdx.x & 63;
  const int jcol = lane & 3;
  const double l = la[pl.ia];
  double nuv[NBI];
#pragma unroll
  for (int bi = 0; bi < NBI; ++bi) nuv[bi] = pl.active ? nu[pl.qbase + bo + bi] : 0.0;
  const ConstPtr<VisRecD<float>> cvrec = as_const(vrec);
  const double origin = kMagic;
  const int64_t kc = blockIdx.y;
  const int k0 = static_cast<int>(kc * kchunk);
  const int k1 = static_cast<int>(k0 + kchunk < n_vis ? k0 + kchunk : n_vis);
  f4_t acc[NBI][8][NG];
#pragma unroll
  for (int bi = 0; bi < NBI; ++bi)
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int g = 0; g < NG; ++g) acc[bi][a][g] = f4_t{0.0f, 0.0f, 0.0f, 0.0f};
  const FillSlot fs = fill_slot(pb.n_gl * NBI);
  const int fgg = fs.slot / NBI, fbi = fs.slot % NBI;
  const double fm = fs.on ? mb[(pb.g4 + fgg) * kGridNBA + bo + fbi] : 0.0;
  for (int kb = k0; kb < k1; kb += KB) {
    __syncthreads();  // the previous batch's reads are done
    if (fs.on) {
      for (int kk = fs.row0; kk < KB; kk += fs.step) {
        const int k = kb + kk;
        float bc = 0.0f, bs = 0.0f, ac = 0.0f, as = 0.0f;
        if (k < k1) {
          phasor(fma(vv[k], fm, origin), bc, bs);
          phasor(fma(vu[k], fm, origin), ac, as);
        }
        const h4_t h = __builtin_convertvector((f4_t{bc, bs, ac, as}), h4_t);
        bsh[kk][fgg][fbi] = __builtin_bit_cast(uint2, h);
      }
    }
    __syncthreads();
    const int ke = kb + KB < k1 ? kb + KB : k1;
    for (int k = kb; k < ke; k += 2) {
      // the basis of both visibilities (k + 1 may be past k1: its LDS entries
      // are zero and so is its residual record; the records past n_vis are
      // padding of the plan)
      h2_t e[2][NBI][8];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int kv = k + h;
        const double u = cvrec[kv].u, v = cvrec[kv].v, w = cvrec[kv].w;
        float c, sn;
        phasor(fma(u, l, origin), c, sn);
        const h2_t aa = to_h2(c, sn);  // A at |l|_ia
        phasor(fma(v, l, origin), c, sn);
        const h2_t qq = to_h2(c, sn);  // B at |m|_ia
#pragma unroll
        for (int bi = 0; bi < NBI; ++bi) {
          const h4_t t4 = __builtin_bit_cast(h4_t, bsh[kv - kb][pl.gl][bi]);
          const h2_t bbm = __builtin_shufflevector(t4, t4, 0, 1);  // B at |m|_b
          const h2_t pam = __builtin_shufflevector(t4, t4, 2, 3);  // A at |l|_b
          float cc, cs;
          phasor(fma(w, nuv[bi], origin), cc, cs);
          const h2_t ch = to_h2(cc, cs);
          const h2_t v1 = h2_t{ch.x, -ch.y};  // (cc, -cs)
          const h2_t v2 = ch.yx;              // (cs, cc)
          const h2_t m12 = aa * bbm, m34 = aa * bbm.yx, m56 = pam * qq, m78 = pam * qq.yx;
          e[h][bi][0] = m12.xx * v1;
          e[h][bi][1] = m12.yy * v1;
          e[h][bi][2] = m34.xx * v2;
          e[h][bi][3] = m34.yy * v2;
          e[h][bi][4] = m56.xx * v1;
          e[h][bi][5] = m56.yy * v1;
          e[h][bi][6] = m78.xx * v2;
          e[h][bi][7] = m78.yy * v2;
        }
      }
      h4_t rb[NG];
#pragma unroll
      for (int g = 0; g < NG; ++g)
        rb[g] = __builtin_bit_cast(h4_t, rh[(static_cast<int64_t>(k >> 1) * NG + g) * 4 + jcol]);
#pragma unroll
      for (int bi = 0; bi < NBI; ++bi)
#pragma unroll
        for (int a = 0; a < 8; ++a) {
          const h4_t av = cat_h2(e[0][bi][a], e[1][bi][a]);
#pragma unroll
          for (int g = 0; g < NG; ++g)
            acc[bi][a][g] = __builtin_amdgcn_mfma_f32_4x4x4f16(av, rb[g], acc[bi][a][g], 0, 0, 0);
        }
    }
  }
  // lane 4b + j writes side j (of each group) of the pairs of lanes 4b .. 4b + 3
  const float sc = *inv;
  float* out = part + kc * n_pix;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int src = (lane & ~3) + i;
    PairLane pi;
    pi.active = __shfl(pl.active ? 1 : 0, src, 64) != 0;
    pi.g4 = __shfl(pl.g4, src, 64);
    pi.ia = __shfl(pl.ia, src, 64);
    pi.gl = __shfl(pl.gl, src, 64);
    pi.qbase = __shfl(pl.qbase, src, 64);
    if (!pi.active) continue;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int r = 4 * g + jcol;
      if (r >= nr) continue;
#pragma unroll
      for (int bi = 0; bi < NBI; ++bi) {
        float G8[8];
#pragma unroll
        for (int a = 0; a < 8; ++a) G8[a] = acc[bi][a][g][i] * sc;
        pair_write(pi, na, bo + bi, G8, slot, out + r * rstride);
      }
    }
  }
}

inline unsigned nblocks(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

template <int PREC, int NG, int VPL>
hipError_t mfma_forward_t(sl1m_plan* p, const float* xp, int nr, hipStream_t st) {
  const int64_t np = p->n_pix, n = static_cast<int64_t>(nr) * np;
  hipLaunchKernelGGL(k_mfma_absmax, dim3(kMfmaRedBlocks), dim3(kBlock), 0, st, xp, n,
                     static_cast<const float*>(p->pscale), np, p->mred);
  hipLaunchKernelGGL((k_mfma_pack_x<PREC>), dim3(nblocks(NG * p->mf_np4 * 4)), dim3(kBlock), 0,
                     st, xp, static_cast<const float*>(p->pscale), np, nr, p->mf_np4, NG,
                     p->mred, p->mred + 2 * kMfmaRedBlocks, p->mx);
  const unsigned vt = static_cast<unsigned>((p->n_vis + kBlock * VPL - 1) / (kBlock * VPL));
  hipLaunchKernelGGL((k_fwd_mfma<PREC, NG, VPL>), dim3(vt, static_cast<unsigned>(p->n_mfchunks)),
                     dim3(kBlock), 0, st, static_cast<const PixRec<float>*>(p->pixrec), p->mx,
                     p->mf_np4, p->vu, p->vv, p->vw, p->n_vis, p->mf_chunk,
                     p->mred + 2 * kMfmaRedBlocks, static_cast<float2*>(p->fpart),
                     p->n_mfchunks, nr);
  return hipGetLastError();
}

template <int PREC, int NG, int PPL>
hipError_t mfma_adjoint_t(sl1m_plan* p, int nr, hipStream_t st) {
  const int64_t nv = p->n_vis;
  const float* rres = static_cast<const float*>(p->rres);  // delta slot: [n_vis][nr] complex
  hipLaunchKernelGGL(k_mfma_absmax, dim3(kMfmaRedBlocks), dim3(kBlock), 0, st, rres,
                     2 * nr * nv, static_cast<const float*>(nullptr), int64_t{1},
                     p->mred + kMfmaRedBlocks);
  hipLaunchKernelGGL((k_mfma_pack_r<PREC>), dim3(nblocks(NG * p->mf_nv4 * 4)), dim3(kBlock), 0,
                     st, reinterpret_cast<const float2*>(rres), nv, nr, p->mf_nv4, NG,
                     p->mred + kMfmaRedBlocks, p->mred + 2 * kMfmaRedBlocks + 1, p->mr);
  const unsigned pt = static_cast<unsigned>((p->n_pix + kBlock * PPL - 1) / (kBlock * PPL));
  hipLaunchKernelGGL((k_adj_mfma<PREC, NG, PPL>), dim3(pt, static_cast<unsigned>(p->n_achunks)),
                     dim3(kBlock), 0, st, static_cast<const VisRecD<float>*>(p->visrecD), p->mr,
                     p->mf_nv4, p->pl, p->pm, p->pc3, p->n_pix, p->adj_kchunk,
                     p->mred + 2 * kMfmaRedBlocks + 1, static_cast<float*>(p->apart),
                     p->n_achunks, nr);
  return hipGetLastError();
}

template <int NG, int NBI>
hipError_t grid_mfma_adjoint_t(sl1m_plan* p, int nr, hipStream_t st) {
  const GridSeg& g = p->grid_segs[0];
  const int64_t nv = p->n_vis, n_kp = (nv + 1) / 2;
  const float* rres = static_cast<const float*>(p->rres);  // delta slot: [n_vis][nr] complex
  hipLaunchKernelGGL(k_mfma_absmax, dim3(kMfmaRedBlocks), dim3(kBlock), 0, st, rres,
                     2 * nr * nv, static_cast<const float*>(nullptr), int64_t{1},
                     p->mred + kMfmaRedBlocks);
  hipLaunchKernelGGL(k_grid_mfma_pack_res, dim3(nblocks(n_kp * NG * 4)), dim3(kBlock), 0, st,
                     reinterpret_cast<const float2*>(rres), nv, nr, n_kp, NG,
                     p->mred + kMfmaRedBlocks, p->mred + 2 * kMfmaRedBlocks + 1,
                     reinterpret_cast<uint2*>(p->mr));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.pblocks == 0) return e;
  const int64_t co = g.cell_off;
  return timed(p, T_GRID_ADJ_DELTA, st, [&] {
    hipLaunchKernelGGL((k_grid_adj_pairs_mfma_h<NG, NBI>),
                       dim3(static_cast<unsigned>(g.pblocks), static_cast<unsigned>(p->n_achunks),
                            static_cast<unsigned>(kGridNBA / NBI)),
                       dim3(kBlock), 0, st, static_cast<const VisRecD<float>*>(p->visrecD),
                       reinterpret_cast<const uint2*>(p->mr), p->vu, p->vv,
                       p->grid_la + g.la_off, p->grid_mb + g.mb_off, p->grid_c3 + co,
                       p->grid_slot + 4 * co, g.na, p->d_grid_pblocks + g.pb0, p->adj_kchunk,
                       nv, p->mred + 2 * kMfmaRedBlocks + 1, static_cast<float*>(p->apart),
                       p->n_pix, static_cast<int64_t>(p->n_achunks) * p->n_pix, nr);
    return hipGetLastError();
  });
}

template <int PREC, int NG>
hipError_t grid_mfma_forward_t(sl1m_plan* p, const float* xp, int nr, hipStream_t st) {
  const GridSeg& g = p->grid_segs[0];
  const int64_t np = p->n_pix, n = static_cast<int64_t>(nr) * np;
  hipLaunchKernelGGL(k_mfma_absmax, dim3(kMfmaRedBlocks), dim3(kBlock), 0, st, xp, n,
                     static_cast<const float*>(p->pscale), np, p->mred);
  hipLaunchKernelGGL((k_grid_mfma_pack_pairs<PREC>), dim3(nblocks(NG * g.n_pairs * 4)),
                     dim3(kBlock), 0, st, xp, np, nr, static_cast<const float*>(p->pscale),
                     p->grid_slot + 4 * g.cell_off, p->grid_c3 + g.cell_off, g.na, g.n_pairs,
                     NG, p->mred, p->mred + 2 * kMfmaRedBlocks, p->grid_mfma_nu,
                     reinterpret_cast<uint4*>(p->grid_mfma_b));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned vt = static_cast<unsigned>((p->n_vis + kBlock - 1) / kBlock);
  return timed(p, T_GRID_FWD_DELTA, st, [&] {
    const dim3 grid(vt, static_cast<unsigned>(g.nfc));
    if constexpr (PREC == SL1M_PREC_MFMA_F16)
      hipLaunchKernelGGL((k_grid_fwd_pairs_mfma_h<NG>), grid, dim3(kBlock), 0, st,
                         reinterpret_cast<const uint4*>(p->grid_mfma_b), p->grid_mfma_nu,
                         g.n_pairs, p->grid_la + g.la_off, p->grid_mb + g.mb_off,
                         p->d_grid_fchunks + g.fc0, g.na, p->vu, p->vv, p->vw, p->n_vis,
                         p->mred + 2 * kMfmaRedBlocks, static_cast<float2*>(p->fpart),
                         p->grid_frows, nr);
    else
      hipLaunchKernelGGL((k_grid_fwd_pairs_mfma<PREC, NG>), grid, dim3(kBlock), 0, st,
                         reinterpret_cast<const uint4*>(p->grid_mfma_b), p->grid_mfma_nu,
                         g.n_pairs, p->grid_la + g.la_off, p->grid_mb + g.mb_off,
                         p->d_grid_fchunks + g.fc0, g.na, p->vu, p->vv, p->vw, p->n_vis,
                         p->mred + 2 * kMfmaRedBlocks, static_cast<float2*>(p->fpart),
                         p->grid_frows, nr);
    return hipGetLastError();
  });
}

template <int PREC, int NG>
hipError_t mfma_forward_v(sl1m_plan* p, const float* xp, int nr, hipStream_t st) {
  if (p->grid_mfma) return grid_mfma_forward_t<PREC, NG>(p, xp, nr, st);
  if (p->fwd_vpl == 1) return mfma_forward_t<PREC, NG, 1>(p, xp, nr, st);
  if (p->fwd_vpl == 2) return mfma_forward_t<PREC, NG, 2>(p, xp, nr, st);
  return mfma_forward_t<PREC, NG, 4>(p, xp, nr, st);
}

template <int PREC, int NG>
hipError_t mfma_adjoint_v(sl1m_plan* p, int nr, hipStream_t st) {
  if (p->adj_ppl == 1) return mfma_adjoint_t<PREC, NG, 1>(p, nr, st);
  if (p->adj_ppl == 2) return mfma_adjoint_t<PREC, NG, 2>(p, nr, st);
  return mfma_adjoint_t<PREC, NG, 4>(p, nr, st);
}

}  // namespace

hipError_t launch_mfma_forward(sl1m_plan* p, const void* xp, int nr, hipStream_t st) {
  if (p->n_vis == 0 || (p->grid_mfma ? p->grid_frows == 0 : p->n_mfchunks == 0))
    return hipSuccess;
  if (nr < 1 || nr > 8 || nr > p->max_rhs) return hipErrorInvalidValue;
  const float* x = static_cast<const float*>(xp);
  if (p->mfma == SL1M_PREC_MFMA_F16)
    return nr <= 4 ? mfma_forward_v<SL1M_PREC_MFMA_F16, 1>(p, x, nr, st)
                   : mfma_forward_v<SL1M_PREC_MFMA_F16, 2>(p, x, nr, st);
  return nr <= 4 ? mfma_forward_v<SL1M_PREC_MFMA_BF16, 1>(p, x, nr, st)
                 : mfma_forward_v<SL1M_PREC_MFMA_BF16, 2>(p, x, nr, st);
}

hipError_t launch_mfma_adjoint(sl1m_plan* p, int nr, hipStream_t st) {
  if (p->n_pix == 0 || p->n_achunks == 0) return hipSuccess;
  if (nr < 1 || nr > 8 || nr > p->max_rhs) return hipErrorInvalidValue;
  if (p->grid_mfma && p->mfma == SL1M_PREC_MFMA_F16)
    return nr <= 4 ? grid_mfma_adjoint_t<1, 2>(p, nr, st) : grid_mfma_adjoint_t<2, 1>(p, nr, st);
  if (p->mfma == SL1M_PREC_MFMA_F16)
    return nr <= 4 ? mfma_adjoint_v<SL1M_PREC_MFMA_F16, 1>(p, nr, st)
                   : mfma_adjoint_v<SL1M_PREC_MFMA_F16, 2>(p, nr, st);
  return nr <= 4 ? mfma_adjoint_v<SL1M_PREC_MFMA_BF16, 1>(p, nr, st)
                 : mfma_adjoint_v<SL1M_PREC_MFMA_BF16, 2>(p, nr, st);
}

}  // namespace sl1m
