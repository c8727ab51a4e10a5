// Device-side building blocks of the SL1M operator kernels (gfx950): phasor
// evaluation and one tile of the forward/adjoint operators.  Shared by the
// per-plan kernels (sl1m_kernels.hip) and the batched serving kernels
// (sl1m_server.hip) so both evaluate every matrix entry identically.
//
// Phase arithmetic (FP32 precision mode): theta = u l + v m + w (n - 1) is
// formed by FP64 FMAs starting from kMagic = 1.5*2^29.  Every intermediate then
// carries a unit in the last place of exactly 2^-23 turn, so the low 23 bits
// of the result's mantissa are the fractional phase; OR-ing them into the
// mantissa of 1.0f gives 1 + frac(theta) in [1, 2) at no extra arithmetic,
// which v_sin_f32 / v_cos_f32 (arguments in turns) take directly.  The
// reduction is exact up to one rounding of at most 2^-24 turn per FMA.
// FP64 precision mode: the phase is reduced as theta - rint(theta) and
// sincospi/exp run in FP64.
#pragma once

#include <type_traits>

#include "sl1m_internal.h"

namespace sl1m {
namespace dev {

template <typename R>
struct Cplx;
template <>
struct Cplx<float> {
  using T = float2;
};
template <>
struct Cplx<double> {
  using T = double2;
};
template <typename R>
using C2 = typename Cplx<R>::T;

constexpr int kSeg = 64;  // inner FP32 accumulation length (two-level sums)

template <typename R>
__device__ __forceinline__ constexpr double phase_origin() {
  return std::is_same<R, float>::value ? kMagic : 0.0;
}

// (cos 2 pi theta, sin 2 pi theta) from t = phase_origin + theta.
__device__ __forceinline__ void phasor(double t, float& c, float& s) {
  const uint32_t lo = static_cast<uint32_t>(__double2loint(t));
  const float f = __uint_as_float((lo & 0x007FFFFFu) | 0x3F800000u);  // 1 + frac(theta)
  s = __builtin_amdgcn_sinf(f);
  c = __builtin_amdgcn_cosf(f);
}
__device__ __forceinline__ void phasor(double t, double& c, double& s) {
  const double r = t - rint(t);
  sincospi(2.0 * r, &s, &c);
}

// FP32 hi/lo phase (SL1M_PREC_FP32_HILO).  For one product a b of split
// coordinates: p = fl(a_hi b_hi) and e = a_hi b_hi - p (exact, one FMA);
// p - rint(p) is exact (rint by adding and subtracting 1.5 2^23, valid for
// |p| < 2^22 turns), and e with the cross terms a_hi b_lo + a_lo b_hi (a_lo b_lo
// is below 2^-48 |a b|) goes into `lo`.  Returns p - rint(p).  Contraction is
// off so every rounding is the one written.
__device__ __forceinline__ float hl_term(float ah, float al, float bh, float bl, float& lo) {
#pragma clang fp contract(off)
  const float p = ah * bh;
  const float e = __builtin_fmaf(ah, bh, -p);
  const float n = (p + 12582912.0f) - 12582912.0f;
  lo = __builtin_fmaf(al, bh, __builtin_fmaf(ah, bl, lo + e));
  return p - n;
}

// (cos 2 pi theta, sin 2 pi theta) with theta = u l + v m + w nu from split
// coordinates: the three reduced parts, then the small terms, added in
// float32 (|result| < 2 turns, inside the range v_sin_f32 / v_cos_f32 take).
__device__ __forceinline__ void hl_phasor(const HLRec& x, float uh, float ul, float vh, float vl,
                                          float wh, float wl, float& c, float& s) {
#pragma clang fp contract(off)
  float lo = 0.0f;
  const float fu = hl_term(uh, ul, x.ah, x.al, lo);
  const float fv = hl_term(vh, vl, x.bh, x.bl, lo);
  const float fw = hl_term(wh, wl, x.ch, x.cl, lo);
  const float t = ((fu + fv) + fw) + lo;
  s = __builtin_amdgcn_sinf(t);
  c = __builtin_amdgcn_cosf(t);
}

// float32 split of a float64 value: hi + lo with hi its float32 rounding
__device__ __forceinline__ void hl_split(double a, float& hi, float& lo) {
  hi = static_cast<float>(a);
  lo = static_cast<float>(a - static_cast<double>(hi));
}

// 2^x
__device__ __forceinline__ float pow2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double pow2(double x) { return exp2(x); }

// Natural exponent scale used with pow2 for the Gaussian taper.
template <typename R>
__device__ __forceinline__ constexpr double taper_scale() {
  return 1.4426950408889634;  // log2(e): exp(x) = 2^(x log2 e)
}

// Read-only view of memory that no thread writes while a kernel runs (pixel
// records, amplitudes, visibility records, residuals).  Loads through the
// constant address space with a wavefront-uniform address become scalar loads
// into SGPRs, also when the pointer itself was loaded from memory (as in the
// batched serving kernels, where the compiler cannot otherwise prove the data
// unwritten).  Reads only.
template <typename T>
using ConstPtr = const __attribute__((address_space(4))) T*;

template <typename T>
__device__ __forceinline__ ConstPtr<T> as_const(const T* p) {
  return (ConstPtr<T>)(p);
}

// Chunk descriptor i of a table, read through the scalar unit.
__device__ __forceinline__ Chunk load_chunk(const Chunk* table, int64_t i) {
  const ConstPtr<Chunk> c = as_const(table) + i;
  Chunk r;
  r.j0 = c->j0;
  r.j1 = c->j1;
  r.sigma = c->sigma;
  r.seg = c->seg;
  r.layer = c->layer;
  return r;
}

// acc += p[0], p[stride], ..., p[(n - 1) * stride], in this order.  Four
// terms are loaded before any of them is added, so a thread waits for one
// memory round trip per four terms instead of one per term; the sum is the
// plain loop's, bit for bit.
__device__ __forceinline__ void acc_add(float& a, float v) { a += v; }
__device__ __forceinline__ void acc_add(double& a, double v) { a += v; }
__device__ __forceinline__ void acc_add(float2& a, float2 v) {
  a.x += v.x;
  a.y += v.y;
}
__device__ __forceinline__ void acc_add(double2& a, double2 v) {
  a.x += v.x;
  a.y += v.y;
}
template <typename T>
__device__ __forceinline__ void strided_sum(const T* __restrict__ p, int n, int64_t stride, T& acc) {
  int c = 0;
  for (; c + 4 <= n; c += 4) {
    const T a0 = p[c * stride], a1 = p[(c + 1) * stride];
    const T a2 = p[(c + 2) * stride], a3 = p[(c + 3) * stride];
    acc_add(acc, a0);
    acc_add(acc, a1);
    acc_add(acc, a2);
    acc_add(acc, a3);
  }
  for (; c < n; ++c) acc_add(acc, p[c * stride]);
}

// ---------------------------------------------------------------------------
// operator tiles
// ---------------------------------------------------------------------------

// One forward tile: visibilities [vtile*kBlock*VPL, +kBlock*VPL) against the
// pixel chunk `ch`; right-hand side r goes to out_row + r*row_stride.
// `xscale` multiplies every amplitude (1 except in batched power steps).
// HL: the FP32 hi/lo phase (R = float, no BEAM) from the pixels' splits
// `phl` and the lane's visibilities split once.
template <typename R, int VPL, bool BEAM, int NR, bool HL = false>
__device__ __forceinline__ void fwd_delta_tile(
    const PixRec<R>* __restrict__ pix, const R* __restrict__ xp, int64_t n_pix,
    const double* __restrict__ vu, const double* __restrict__ vv, const double* __restrict__ vw,
    const R* __restrict__ vbeta, const Chunk& ch, int64_t vtile, int64_t n_vis,
    C2<R>* __restrict__ out_row, int64_t row_stride, R xscale,
    const HLRec* __restrict__ phl = nullptr) {
  static_assert(!HL || (std::is_same<R, float>::value && !BEAM), "hi/lo phase: float32, no pair beams");
  const int64_t kbase = vtile * (kBlock * VPL) + threadIdx.x;
  const ConstPtr<PixRec<R>> cpix = as_const(pix);
  const ConstPtr<HLRec> chl = as_const(phl);
  const ConstPtr<R> cxp = as_const(xp);
  double u[VPL], v[VPL], w[VPL];
  float uh[VPL], ul[VPL], vh[VPL], vl[VPL], wh[VPL], wl[VPL];
  R beta[VPL], ore[NR][VPL], oim[NR][VPL];
#pragma unroll
  for (int i = 0; i < VPL; ++i) {
    const int64_t k = kbase + static_cast<int64_t>(i) * kBlock;
    const bool ok = k < n_vis;
    u[i] = ok ? vu[k] : 0.0;
    v[i] = ok ? vv[k] : 0.0;
    w[i] = ok ? vw[k] : 0.0;
    if (HL) {
      hl_split(u[i], uh[i], ul[i]);
      hl_split(v[i], vh[i], vl[i]);
      hl_split(w[i], wh[i], wl[i]);
    }
    beta[i] = (BEAM && ok) ? vbeta[k] : R(0);
#pragma unroll
    for (int r = 0; r < NR; ++r) ore[r][i] = oim[r][i] = R(0);
  }
  const double origin = phase_origin<R>();
  const int jb = static_cast<int>(ch.j0), je = static_cast<int>(ch.j1);
  for (int j0 = jb; j0 < je; j0 += kSeg) {
    const int j1 = j0 + kSeg < je ? j0 + kSeg : je;
    R re[NR][VPL], im[NR][VPL];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < VPL; ++i) re[r][i] = im[r][i] = R(0);
    for (int j = j0; j < j1; ++j) {
      double pl = 0.0, pm = 0.0, pn = 0.0;
      HLRec hx;
      if (HL) {
        hx.ah = chl[j].ah; hx.al = chl[j].al;
        hx.bh = chl[j].bh; hx.bl = chl[j].bl;
        hx.ch = chl[j].ch; hx.cl = chl[j].cl;
      } else {
        pl = cpix[j].l;
        pm = cpix[j].m;
        pn = cpix[j].c3;
      }
      R a[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) a[r] = cpix[j].scale * xscale * cxp[r * n_pix + j];
      const R r2 = BEAM ? cpix[j].r2r : R(0);
#pragma unroll
      for (int i = 0; i < VPL; ++i) {
        R c, s;
        if constexpr (HL) {
          hl_phasor(hx, uh[i], ul[i], vh[i], vl[i], wh[i], wl[i], c, s);
        } else {
          const double t = fma(w[i], pn, fma(v[i], pm, fma(u[i], pl, origin)));
          phasor(t, c, s);
        }
        const R b = BEAM ? pow2(beta[i] * r2) : R(1);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const R ai = BEAM ? a[r] * b : a[r];
          re[r][i] = fma(ai, c, re[r][i]);
          im[r][i] = fma(-ai, s, im[r][i]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < VPL; ++i) {
        ore[r][i] += re[r][i];
        oim[r][i] += im[r][i];
      }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    C2<R>* out = out_row + r * row_stride;
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
      const int64_t k = kbase + static_cast<int64_t>(i) * kBlock;
      if (k < n_vis) {
        C2<R> o;
        o.x = ore[r][i];
        o.y = oim[r][i];
        out[k] = o;
      }
    }
  }
}

// Gaussian pixels, eq. (samlm4)/(samlm5) in completed-square form:
//   M = g (1/n) D (1 + i s) exp(-pi sigma^2 D |(u,v) - w (l,m)|^2)
//       exp(2 pi i [D(-(u l + v m) + (w/2)(r^2 - sigma^4 rho^2)) - w kappa])
// with s = w sigma^2, D = 1/(1+s^2), kappa = n - 1 + r^2/2 (0 for paraxial).
// The factor D(1 + i s) is constant per (visibility, segment) and applied once
// to the segment's sum.
template <typename R, int VPL, bool BEAM, int NR>
__device__ __forceinline__ void fwd_gauss_tile(
    const PixRec<R>* __restrict__ pix, const R* __restrict__ xp, int64_t n_pix,
    const double* __restrict__ vu, const double* __restrict__ vv, const double* __restrict__ vw,
    const R* __restrict__ vbeta, const Chunk& ch, int64_t vtile, int64_t n_vis,
    C2<R>* __restrict__ out_row, int64_t row_stride, R xscale) {
  const int64_t kbase = vtile * (kBlock * VPL) + threadIdx.x;
  const ConstPtr<PixRec<R>> cpix = as_const(pix);
  const ConstPtr<R> cxp = as_const(xp);
  const double sig2 = ch.sigma * ch.sigma;
  double A[VPL], B[VPL], C[VPL], NW[VPL], E0[VPL];
  R ur[VPL], vr[VPL], wr[VPL], c1[VPL], Dd[VPL], Ds[VPL], beta[VPL];
  R ore[NR][VPL], oim[NR][VPL];
#pragma unroll
  for (int i = 0; i < VPL; ++i) {
    const int64_t k = kbase + static_cast<int64_t>(i) * kBlock;
    const bool ok = k < n_vis;
    const double u = ok ? vu[k] : 0.0, v = ok ? vv[k] : 0.0, w = ok ? vw[k] : 0.0;
    const double s = w * sig2;
    const double D = 1.0 / (1.0 + s * s);
    A[i] = -D * u;
    B[i] = -D * v;
    C[i] = 0.5 * D * w;
    NW[i] = -w;
    E0[i] = phase_origin<R>() - 0.5 * D * w * sig2 * sig2 * (u * u + v * v);
    ur[i] = static_cast<R>(u);
    vr[i] = static_cast<R>(v);
    wr[i] = static_cast<R>(w);
    c1[i] = static_cast<R>(-M_PI * sig2 * D * taper_scale<R>());
    Dd[i] = static_cast<R>(D);
    Ds[i] = static_cast<R>(D * s);
    beta[i] = (BEAM && ok) ? vbeta[k] : R(0);
#pragma unroll
    for (int r = 0; r < NR; ++r) ore[r][i] = oim[r][i] = R(0);
  }
  const int jb = static_cast<int>(ch.j0), je = static_cast<int>(ch.j1);
  for (int j0 = jb; j0 < je; j0 += kSeg) {
    const int j1 = j0 + kSeg < je ? j0 + kSeg : je;
    R re[NR][VPL], im[NR][VPL];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < VPL; ++i) re[r][i] = im[r][i] = R(0);
    for (int j = j0; j < j1; ++j) {
      const double pl = cpix[j].l, pm = cpix[j].m, pr2 = cpix[j].c3, pk = cpix[j].c4;
      const R lr = cpix[j].lr, mr = cpix[j].mr;
      R a[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) a[r] = cpix[j].scale * xscale * cxp[r * n_pix + j];
      const R r2 = BEAM ? cpix[j].r2r : R(0);
#pragma unroll
      for (int i = 0; i < VPL; ++i) {
        const double t = fma(A[i], pl, fma(B[i], pm, fma(C[i], pr2, fma(NW[i], pk, E0[i]))));
        R c, s;
        phasor(t, c, s);
        const R du = fma(-wr[i], lr, ur[i]);
        const R dv = fma(-wr[i], mr, vr[i]);
        const R q = fma(du, du, dv * dv);
        R e = pow2(c1[i] * q);
        if (BEAM) e *= pow2(beta[i] * r2);
        const R ec = e * c, es = e * s;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          re[r][i] = fma(a[r], ec, re[r][i]);
          im[r][i] = fma(a[r], es, im[r][i]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < VPL; ++i) {
        ore[r][i] += re[r][i];
        oim[r][i] += im[r][i];
      }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    C2<R>* out = out_row + r * row_stride;
#pragma unroll
    for (int i = 0; i < VPL; ++i) {
      const int64_t k = kbase + static_cast<int64_t>(i) * kBlock;
      if (k < n_vis) {
        C2<R> o;
        o.x = Dd[i] * ore[r][i] - Ds[i] * oim[r][i];
        o.y = Ds[i] * ore[r][i] + Dd[i] * oim[r][i];
        out[k] = o;
      }
    }
  }
}

// One adjoint tile: pixels [tl.j0 + sub_i*kBlock*PPL, +kBlock*PPL) of tile `tl`
// against visibility chunk `kc`; right-hand side r goes to
// out_row + r*row_stride (indexed by permuted pixel).
// HL: the FP32 hi/lo phase (R = float, no BEAM) from the visibilities'
// splits `vhl` and the lane's pixels split once.
template <typename R, int PPL, bool BEAM, int NR, bool HL = false>
__device__ __forceinline__ void adj_delta_tile(
    const VisRecD<R>* __restrict__ vrec, const C2<R>* __restrict__ rres,
    const R* __restrict__ vbeta, const double* __restrict__ pl, const double* __restrict__ pm,
    const double* __restrict__ pc3, const R* __restrict__ pr2, const Chunk& tl, int sub_i,
    int64_t kc, int64_t kchunk, int64_t n_vis, R* __restrict__ out_row, int64_t row_stride,
    const HLRec* __restrict__ vhl = nullptr) {
  static_assert(!HL || (std::is_same<R, float>::value && !BEAM), "hi/lo phase: float32, no pair beams");
  const int64_t jbase = tl.j0 + static_cast<int64_t>(sub_i) * (kBlock * PPL) + threadIdx.x;
  const ConstPtr<VisRecD<R>> cvrec = as_const(vrec);
  const ConstPtr<HLRec> chl = as_const(vhl);
  const ConstPtr<R> cres = as_const(reinterpret_cast<const R*>(rres));
  const ConstPtr<R> cbeta = as_const(vbeta);
  const int k0 = static_cast<int>(kc * kchunk);
  const int k1 = static_cast<int>(k0 + kchunk < n_vis ? k0 + kchunk : n_vis);
  double l[PPL], m[PPL], c3[PPL];
  HLRec px[PPL];
  R r2[PPL], og[NR][PPL];
#pragma unroll
  for (int i = 0; i < PPL; ++i) {
    const int64_t j = jbase + static_cast<int64_t>(i) * kBlock;
    const bool ok = j < tl.j1;
    l[i] = ok ? pl[j] : 0.0;
    m[i] = ok ? pm[j] : 0.0;
    c3[i] = ok ? pc3[j] : 0.0;
    if (HL) {
      hl_split(l[i], px[i].ah, px[i].al);
      hl_split(m[i], px[i].bh, px[i].bl);
      hl_split(c3[i], px[i].ch, px[i].cl);
    }
    r2[i] = (BEAM && ok) ? pr2[j] : R(0);
#pragma unroll
    for (int r = 0; r < NR; ++r) og[r][i] = R(0);
  }
  const double origin = phase_origin<R>();
  for (int kk = k0; kk < k1; kk += kSeg) {
    const int ke = kk + kSeg < k1 ? kk + kSeg : k1;
    R g[NR][PPL];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < PPL; ++i) g[r][i] = R(0);
    for (int k = kk; k < ke; ++k) {
      double u = 0.0, v = 0.0, w = 0.0;
      float uh = 0.0f, ul = 0.0f, vh = 0.0f, vl = 0.0f, wh = 0.0f, wl = 0.0f;
      if (HL) {
        uh = chl[k].ah; ul = chl[k].al;
        vh = chl[k].bh; vl = chl[k].bl;
        wh = chl[k].ch; wl = chl[k].cl;
      } else {
        u = cvrec[k].u;
        v = cvrec[k].v;
        w = cvrec[k].w;
      }
      R rre[NR], rim[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        rre[r] = cres[(static_cast<int64_t>(k) * NR + r) * 2];
        rim[r] = cres[(static_cast<int64_t>(k) * NR + r) * 2 + 1];
      }
      const R bt = BEAM ? cbeta[k] : R(0);
#pragma unroll
      for (int i = 0; i < PPL; ++i) {
        R c, s;
        if constexpr (HL) {
          hl_phasor(px[i], uh, ul, vh, vl, wh, wl, c, s);
        } else {
          const double t = fma(c3[i], w, fma(m[i], v, fma(l[i], u, origin)));
          phasor(t, c, s);
        }
        if (BEAM) {
          const R b = pow2(bt * r2[i]);
          c *= b;
          s *= b;
        }
        // Re[(c + i s)(rre + i rim)] = c rre - s rim
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          g[r][i] = fma(c, rre[r], g[r][i]);
          g[r][i] = fma(-s, rim[r], g[r][i]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < PPL; ++i) og[r][i] += g[r][i];
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    R* out = out_row + r * row_stride;
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      const int64_t j = jbase + static_cast<int64_t>(i) * kBlock;
      if (j < tl.j1) out[j] = og[r][i];
    }
  }
}

template <typename R, int PPL, bool BEAM, int NR>
__device__ __forceinline__ void adj_gauss_tile(
    const VisRecG<R>* __restrict__ vrec, const C2<R>* __restrict__ rres,
    const R* __restrict__ vbeta, const double* __restrict__ pl, const double* __restrict__ pm,
    const double* __restrict__ pc3, const double* __restrict__ pc4, const R* __restrict__ pr2,
    const Chunk& tl, int sub_i, int64_t kc, int64_t kchunk, int64_t n_vis,
    R* __restrict__ out_row, int64_t row_stride) {
  const int64_t jbase = tl.j0 + static_cast<int64_t>(sub_i) * (kBlock * PPL) + threadIdx.x;
  const ConstPtr<VisRecG<R>> crec = as_const(vrec + static_cast<int64_t>(tl.layer) * n_vis);
  const ConstPtr<R> cres =
      as_const(reinterpret_cast<const R*>(rres + static_cast<int64_t>(1 + tl.layer) * n_vis * NR));
  const ConstPtr<R> cbeta = as_const(vbeta);
  const int k0 = static_cast<int>(kc * kchunk);
  const int k1 = static_cast<int>(k0 + kchunk < n_vis ? k0 + kchunk : n_vis);
  double l[PPL], m[PPL], c3[PPL], c4[PPL];
  R lr[PPL], mr[PPL], r2[PPL], og[NR][PPL];
#pragma unroll
  for (int i = 0; i < PPL; ++i) {
    const int64_t j = jbase + static_cast<int64_t>(i) * kBlock;
    const bool ok = j < tl.j1;
    l[i] = ok ? pl[j] : 0.0;
    m[i] = ok ? pm[j] : 0.0;
    c3[i] = ok ? pc3[j] : 0.0;
    c4[i] = ok ? pc4[j] : 0.0;
    lr[i] = static_cast<R>(l[i]);
    mr[i] = static_cast<R>(m[i]);
    r2[i] = (BEAM && ok) ? pr2[j] : R(0);
#pragma unroll
    for (int r = 0; r < NR; ++r) og[r][i] = R(0);
  }
  for (int kk = k0; kk < k1; kk += kSeg) {
    const int ke = kk + kSeg < k1 ? kk + kSeg : k1;
    R g[NR][PPL];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < PPL; ++i) g[r][i] = R(0);
    for (int k = kk; k < ke; ++k) {
      const double A = crec[k].A, B = crec[k].B, C = crec[k].C, NW = crec[k].NW, E0 = crec[k].E0;
      const R ur = crec[k].ur, vr = crec[k].vr, wr = crec[k].wr, c1 = crec[k].c1;
      R rre[NR], rim[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        rre[r] = cres[(static_cast<int64_t>(k) * NR + r) * 2];
        rim[r] = cres[(static_cast<int64_t>(k) * NR + r) * 2 + 1];
      }
      const R bt = BEAM ? cbeta[k] : R(0);
#pragma unroll
      for (int i = 0; i < PPL; ++i) {
        const double t = fma(A, l[i], fma(B, m[i], fma(C, c3[i], fma(NW, c4[i], E0))));
        R c, s;
        phasor(t, c, s);
        const R du = fma(-wr, lr[i], ur);
        const R dv = fma(-wr, mr[i], vr);
        const R q = fma(du, du, dv * dv);
        R e = pow2(c1 * q);
        if (BEAM) e *= pow2(bt * r2[i]);
        const R ec = e * c, es = e * s;
        // Re[(c - i s)(rre + i rim)] = c rre + s rim
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          g[r][i] = fma(ec, rre[r], g[r][i]);
          g[r][i] = fma(es, rim[r], g[r][i]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int i = 0; i < PPL; ++i) og[r][i] += g[r][i];
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    R* out = out_row + r * row_stride;
#pragma unroll
    for (int i = 0; i < PPL; ++i) {
      const int64_t j = jbase + static_cast<int64_t>(i) * kBlock;
      if (j < tl.j1) out[j] = og[r][i];
    }
  }
}

// Writes the adjoint residual records of visibility k for right-hand side r
// from the complex value (re, im) already including the gain G_k:
//   slot 0 (delta):          conj(G_k) v
//   slot 1 + L (Gaussian L): D (1 - i s) conj(G_k) v
template <typename R>
__device__ __forceinline__ void write_res(C2<R>* __restrict__ rres, const R* __restrict__ layerDs,
                                          int n_layers, int64_t n_vis, int nr, int64_t k, int r,
                                          R gr, R gi, R re, R im,
                                          ResPolar* __restrict__ rpol = nullptr) {
  const R cr = gr * re + gi * im;
  const R ci = gr * im - gi * re;
  C2<R> o;
  o.x = cr;
  o.y = ci;
  rres[k * nr + r] = o;
  if (rpol) {  // polar form of the delta record, [r][n_vis]
    const double xr = static_cast<double>(cr), xi = static_cast<double>(ci);
    ResPolar q;
    q.org = kMagic + atan2(xi, xr) * 0.15915494309189535;  // 1 / (2 pi)
    q.mag = static_cast<float>(sqrt(xr * xr + xi * xi));
    q.pad = 0.0f;
    rpol[static_cast<int64_t>(r) * n_vis + k] = q;
  }
  for (int L = 0; L < n_layers; ++L) {
    const R D = layerDs[(static_cast<int64_t>(L) * n_vis + k) * 2];
    const R s = layerDs[(static_cast<int64_t>(L) * n_vis + k) * 2 + 1];
    o.x = D * (cr + s * ci);
    o.y = D * (ci - s * cr);
    rres[(static_cast<int64_t>(1 + L) * n_vis + k) * nr + r] = o;
  }
}

}  // namespace dev
}  // namespace sl1m
