// HIP kernels of the SL1M hot path for gfx950 (MI355X).
//
// Operator kernels evaluate every entry of M from its closed form when it is
// used (Hardy 2013, Section "On-the-fly computation versus in-memory
// computation"); nothing of M is stored.
//
//  * forward  V_k = sum_j M_kj x_j : a lane owns visibilities (VPL per lane,
//    in registers, FP64 coordinates); the pixel records stream through the
//    scalar unit, one uniform record per loop step, so every lane of a
//    wavefront reads the same pixel without LDS traffic.
//  * adjoint  g_j = Re sum_k conj(M_kj) r_k : a lane owns pixels (PPL per lane);
//    visibility records (coordinates + residual) stream through the scalar unit.
//  * Split-K: each block sums one chunk of the streamed index into its own row
//    of a partial buffer; a reduce kernel adds the rows in a fixed order, so
//    results are bitwise reproducible run to run.
//
// Phase arithmetic (FP32 precision mode): theta = u l + v m + w (n - 1) is
// formed by three FP64 FMAs starting from kMagic = 1.5*2^29.  Every
// intermediate then carries a unit in the last place of exactly 2^-23 turn, so
// the low 23 bits of the result's mantissa are the fractional phase; OR-ing
// them into the mantissa of 1.0f gives 1 + frac(theta) in [1, 2) at no extra
// arithmetic, which v_sin_f32 / v_cos_f32 (arguments in turns) take directly.
// The reduction is exact up to three roundings of at most 2^-24 turn each.
//
// FP64 precision mode: the same kernels with FP64 amplitudes and accumulators,
// the phase reduced as theta - rint(theta) and sincospi/exp in FP64.
#include <type_traits>

#include "sl1m_device.h"

namespace sl1m {

namespace {

using namespace dev;


// ---------------------------------------------------------------------------
// forward kernels
// ---------------------------------------------------------------------------
//
// NR right-hand sides share every phasor: x is [NR][n_pix] (permuted order),
// partial rows are [NR][n_rows][n_vis].

template <typename R, int VPL, bool BEAM, int NR, bool HL>
__global__ __launch_bounds__(kBlock) void k_fwd_delta(
    const PixRec<R>* __restrict__ pix, const R* __restrict__ xp, int64_t n_pix,
    const double* __restrict__ vu, const double* __restrict__ vv, const double* __restrict__ vw,
    const R* __restrict__ vbeta, const Chunk* __restrict__ chunks, int64_t n_vis,
    C2<R>* __restrict__ part, int row0, int n_rows, const HLRec* __restrict__ phl) {
  const Chunk ch = chunks[blockIdx.y];
  fwd_delta_tile<R, VPL, BEAM, NR, HL>(pix, xp, n_pix, vu, vv, vw, vbeta, ch, blockIdx.x, n_vis,
                                       part + static_cast<int64_t>(row0 + blockIdx.y) * n_vis,
                                       static_cast<int64_t>(n_rows) * n_vis, R(1), phl);
}

template <typename R, int VPL, bool BEAM, int NR>
__global__ __launch_bounds__(kBlock) void k_fwd_gauss(
    const PixRec<R>* __restrict__ pix, const R* __restrict__ xp, int64_t n_pix,
    const double* __restrict__ vu, const double* __restrict__ vv, const double* __restrict__ vw,
    const R* __restrict__ vbeta, const Chunk* __restrict__ chunks, int64_t n_vis,
    C2<R>* __restrict__ part, int row0, int n_rows) {
  const Chunk ch = chunks[blockIdx.y];
  fwd_gauss_tile<R, VPL, BEAM, NR>(pix, xp, n_pix, vu, vv, vw, vbeta, ch, blockIdx.x, n_vis,
                                   part + static_cast<int64_t>(row0 + blockIdx.y) * n_vis,
                                   static_cast<int64_t>(n_rows) * n_vis, R(1));
}

// ---------------------------------------------------------------------------
// adjoint kernels
// ---------------------------------------------------------------------------
//
// A plan's pixel tiles hold kBlock * adj_ppl pixels; a kernel with PPL pixels
// per lane covers a tile with `sub` = adj_ppl / PPL consecutive blocks.
// Residual records: rres[(layer_slot * n_vis + k) * NR + r] (slot 0 = delta,
// slot 1 + L = Gaussian layer L).  Partial rows are [NR][gridDim.y][n_pix].

template <typename R, int PPL, bool BEAM, int NR, bool HL>
__global__ __launch_bounds__(kBlock) void k_adj_delta(
    const VisRecD<R>* __restrict__ vrec, const C2<R>* __restrict__ rres,
    const R* __restrict__ vbeta, const double* __restrict__ pl, const double* __restrict__ pm,
    const double* __restrict__ pc3, const R* __restrict__ pr2, const Chunk* __restrict__ tiles,
    int sub, int64_t kchunk, int64_t n_vis, int64_t n_pix, R* __restrict__ part,
    const HLRec* __restrict__ vhl) {
  const Chunk tl = tiles[blockIdx.x / sub];
  adj_delta_tile<R, PPL, BEAM, NR, HL>(vrec, rres, vbeta, pl, pm, pc3, pr2, tl, blockIdx.x % sub,
                                       blockIdx.y, kchunk, n_vis,
                                       part + static_cast<int64_t>(blockIdx.y) * n_pix,
                                       static_cast<int64_t>(gridDim.y) * n_pix, vhl);
}

template <typename R, int PPL, bool BEAM, int NR>
__global__ __launch_bounds__(kBlock) void k_adj_gauss(
    const VisRecG<R>* __restrict__ vrec, const C2<R>* __restrict__ rres,
    const R* __restrict__ vbeta, const double* __restrict__ pl, const double* __restrict__ pm,
    const double* __restrict__ pc3, const double* __restrict__ pc4, const R* __restrict__ pr2,
    const Chunk* __restrict__ tiles, int sub, int64_t kchunk, int64_t n_vis, int64_t n_pix,
    R* __restrict__ part) {
  const Chunk tl = tiles[blockIdx.x / sub];
  adj_gauss_tile<R, PPL, BEAM, NR>(vrec, rres, vbeta, pl, pm, pc3, pc4, pr2, tl, blockIdx.x % sub,
                                   blockIdx.y, kchunk, n_vis,
                                   part + static_cast<int64_t>(blockIdx.y) * n_pix,
                                   static_cast<int64_t>(gridDim.y) * n_pix);
}

// ---------------------------------------------------------------------------
// reductions of split-K partials, residual, adjoint records, FISTA update
// ---------------------------------------------------------------------------

// vis[r][k] = G_k * sum_c part[r][c][k]  (minus data[r][k] if data != null);
// writes the adjoint residual records when `rres` is set (and the delta
// record's polar form when `rpol` is).
template <typename R>
__global__ void k_fwd_reduce(const C2<R>* __restrict__ part, int n_rows, int64_t n_vis, int nr,
                             const R* __restrict__ gain, const C2<R>* __restrict__ data,
                             C2<R>* __restrict__ out, C2<R>* __restrict__ rres,
                             const R* __restrict__ layerDs, int n_layers,
                             ResPolar* __restrict__ rpol) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n_vis) return;
  const R gr = gain ? gain[2 * k] : R(1), gi = gain ? gain[2 * k + 1] : R(0);
  for (int r = 0; r < nr; ++r) {
    C2<R> acc;
    acc.x = R(0);
    acc.y = R(0);
    strided_sum<C2<R>>(part + static_cast<int64_t>(r * n_rows) * n_vis + k, n_rows, n_vis, acc);
    R re = acc.x, im = acc.y;
    if (gain) {
      const R tr = gr * re - gi * im;
      im = gr * im + gi * re;
      re = tr;
    }
    if (data) {
      re -= data[r * n_vis + k].x;
      im -= data[r * n_vis + k].y;
    }
    if (out) {
      C2<R> o;
      o.x = re;
      o.y = im;
      out[r * n_vis + k] = o;
    }
    if (rres) write_res<R>(rres, layerDs, n_layers, n_vis, nr, k, r, gr, gi, re, im, rpol);
  }
}

// Split-K row sums of the adjoint partials for the 64 pixels of block
// blockIdx.x: wavefront w of the 4 adds rows c = w, w + 4, ... of right-hand
// side r; the four partial sums meet in LDS and are combined in a fixed order
// by wavefront 0, which gets the result (other wavefronts get 0).  Every
// thread of the block must call it (it synchronises the block).
constexpr int kRowPix = 64;
static_assert(kBlock == 4 * kRowPix, "row_sum uses four wavefronts of kRowPix lanes");
template <typename R>
__device__ __forceinline__ R row_sum(const R* __restrict__ part, int n_rows, int64_t n_pix, int r,
                                     int64_t j, R (*sh)[kRowPix]) {
  const int wv = threadIdx.x / kRowPix, ln = threadIdx.x % kRowPix;
  R g = R(0);
  if (j < n_pix && wv < n_rows)
    strided_sum<R>(part + static_cast<int64_t>(r * n_rows + wv) * n_pix + j, (n_rows - wv + 3) / 4,
                   4 * n_pix, g);
  sh[wv][ln] = g;
  __syncthreads();
  const R t = wv == 0 ? (sh[0][ln] + sh[1][ln]) + (sh[2][ln] + sh[3][ln]) : R(0);
  __syncthreads();
  return t;
}

// g[r][perm[j]] (or g[r][j]) = scale_j * sum_c part[r][c][j]; blocks of
// kBlock threads cover kRowPix pixels.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_adj_reduce(const R* __restrict__ part, int n_rows,
                                                       int64_t n_pix, int nr,
                                                       const R* __restrict__ scale,
                                                       const int32_t* __restrict__ perm,
                                                       R* __restrict__ out) {
  __shared__ R sh[4][kRowPix];
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kRowPix + threadIdx.x % kRowPix;
  for (int r = 0; r < nr; ++r) {
    const R g = row_sum<R>(part, n_rows, n_pix, r, j, sh);
    if (threadIdx.x < kRowPix && j < n_pix) out[r * n_pix + (perm ? perm[j] : j)] = g * scale[j];
  }
}

// One FISTA step on permuted vectors (Section "Implementation of SL1M"):
//   z = y - g / L;  I_k = T^{lambda/L}(z)  (eq. threshp);  y <- I_k + beta (I_k - I_{k-1})
// with g = scale_j * sum_c part[c][j] and beta = (t_k - 1) / t_{k+1}.  The
// scalars live on the device (scal[0] = t_k, scal[1] = 1/L, scal[2] = lambda/L)
// so the iteration's launches are identical every time and can be replayed
// from a captured graph; k_tstep advances t afterwards.
// A non-finite z (overflow of a diverging iteration) would be mapped to 0 by
// the threshold; it is recorded in *flag instead so the solve can report it.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_fista(const R* __restrict__ part, int n_rows,
                                                  int64_t n_pix, const R* __restrict__ scale,
                                                  R* __restrict__ y, R* __restrict__ img,
                                                  const double* __restrict__ scal,
                                                  int* __restrict__ flag) {
  __shared__ R sh[4][kRowPix];
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kRowPix + threadIdx.x % kRowPix;
  R g = row_sum<R>(part, n_rows, n_pix, 0, j, sh);
  if (threadIdx.x >= kRowPix || j >= n_pix) return;
  const double t = scal[0];
  const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
  const R beta = static_cast<R>((t - 1.0) / tn);
  const R inv_L = static_cast<R>(scal[1]), thr = static_cast<R>(scal[2]);
  g *= scale[j];
  const R z = y[j] - g * inv_L;
  if (!isfinite(z)) atomicOr(flag, 1);
  const R in = z > thr ? z - thr : R(0);
  const R io = img[j];
  y[j] = in + beta * (in - io);
  img[j] = in;
}

// MFISTA (the monotone variant of Beck & Teboulle the paper names): the
// proximal step z_k = T^{lambda/L}(y_k - g / L) into z, g as for k_fista.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_prox(const R* __restrict__ part, int n_rows,
                                                 int64_t n_pix, const R* __restrict__ scale,
                                                 const R* __restrict__ y, R* __restrict__ z,
                                                 const double* __restrict__ scal,
                                                 int* __restrict__ flag) {
  __shared__ R sh[4][kRowPix];
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kRowPix + threadIdx.x % kRowPix;
  R g = row_sum<R>(part, n_rows, n_pix, 0, j, sh);
  if (threadIdx.x >= kRowPix || j >= n_pix) return;
  const R inv_L = static_cast<R>(scal[1]), thr = static_cast<R>(scal[2]);
  g *= scale[j];
  const R v = y[j] - g * inv_L;
  if (!isfinite(v)) atomicOr(flag, 1);
  z[j] = v > thr ? v - thr : R(0);
}

// MFISTA selection and extrapolation, from F(z_k) = red[0] + lambda red[1]
// (the objective reduction of z_k) and F(x_{k-1}) = scal[4]:
//   x_k = z_k if F(z_k) <= F(x_{k-1}) else x_{k-1}
//   y_{k+1} = x_k + (t_k/t_{k+1})(z_k - x_k) + ((t_k - 1)/t_{k+1})(x_k - x_{k-1})
// img holds x_{k-1} on entry and x_k on exit.  Every block reads the same
// scalars, so every pixel takes the same choice.
template <typename R>
__global__ void k_mfista_select(R* __restrict__ y, R* __restrict__ img, const R* __restrict__ z,
                                int64_t n, const double* __restrict__ scal,
                                const double* __restrict__ red) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double Fz = red[0] + scal[3] * red[1];
  const bool take = Fz <= scal[4];
  const double t = scal[0];
  const double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * t * t));
  const R a = static_cast<R>(t / tn), b = static_cast<R>((t - 1.0) / tn);
  const R xo = img[j], zj = z[j];
  const R xk = take ? zj : xo;
  y[j] = xk + a * (zj - xk) + b * (xk - xo);
  img[j] = xk;
}

// After the selection: F(x_k) = min(F(z_k), F(x_{k-1})), t_{k+1}.
__global__ void k_mfista_step(double* __restrict__ scal, const double* __restrict__ red) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double Fz = red[0] + scal[3] * red[1];
  scal[4] = Fz < scal[4] ? Fz : scal[4];
  scal[0] = 0.5 * (1.0 + sqrt(1.0 + 4.0 * scal[0] * scal[0]));
}

// F(x_0) = red[0] + lambda red[1] into scal[4] (start of an MFISTA solve).
__global__ void k_mfista_init(double* __restrict__ scal, const double* __restrict__ red) {
  if (threadIdx.x == 0 && blockIdx.x == 0) scal[4] = red[0] + scal[3] * red[1];
}

// t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
__global__ void k_tstep(double* __restrict__ scal) {
  if (threadIdx.x == 0 && blockIdx.x == 0) scal[0] = 0.5 * (1.0 + sqrt(1.0 + 4.0 * scal[0] * scal[0]));
}

// ---------------------------------------------------------------------------
// plan preparation
// ---------------------------------------------------------------------------

// Per-pixel quantities for one segment (permuted positions [j0, j0+count)).
//   r^2 = l^2 + m^2, n = sqrt(1 - r^2), n - 1 = -r^2 / (1 + n),
//   kappa = n - 1 + r^2/2 = -r^4 / (2 (1 + n)^2), scale = (1/n) * 2^(bc r^2)
template <typename R>
__global__ void k_prep_pixels(const int32_t* __restrict__ perm, const double* __restrict__ l,
                              const double* __restrict__ m, int64_t j0, int64_t count, int kind,
                              double beam_coef, PixRec<R>* __restrict__ rec,
                              double* __restrict__ pl, double* __restrict__ pm,
                              double* __restrict__ pc3, double* __restrict__ pc4,
                              R* __restrict__ pscale, R* __restrict__ pr2) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int64_t j = j0 + t;
  const int32_t o = perm[j];
  const double L = l[o], Mm = m[o];
  const double r2 = L * L + Mm * Mm;
  const double n = sqrt(1.0 - r2);
  const double nu = -r2 / (1.0 + n);
  const double kappa = -(r2 * r2) / (2.0 * (1.0 + n) * (1.0 + n));
  const double scale = (1.0 / n) * exp2(beam_coef * r2);
  double c3, c4;
  if (kind == SL1M_PIX_DELTA) {
    c3 = nu;
    c4 = 0.0;
  } else {
    c3 = r2;
    c4 = kind == SL1M_PIX_GAUSS_WIDE ? kappa : 0.0;
  }
  PixRec<R> q;
  q.l = L;
  q.m = Mm;
  q.c3 = c3;
  q.c4 = c4;
  q.lr = static_cast<R>(L);
  q.mr = static_cast<R>(Mm);
  q.scale = static_cast<R>(scale);
  q.r2r = static_cast<R>(r2);
  rec[j] = q;
  pl[j] = L;
  pm[j] = Mm;
  pc3[j] = c3;
  pc4[j] = c4;
  pscale[j] = static_cast<R>(scale);
  pr2[j] = static_cast<R>(r2);
}

// Per-visibility data: coordinates, gains G_k = c_p conj(c_q), pair-beam
// exponent beta_k = -2 (1/F_p^2 + 1/F_q^2) (so that E_p conj(E_q) carries
// 2^(beta_k r^2)), static parts of the adjoint records, and per Gaussian layer
// the constants of the completed-square form.
template <typename R>
__global__ void k_prep_vis(const double* __restrict__ u, const double* __restrict__ v,
                           const double* __restrict__ w, const int32_t* __restrict__ ap,
                           const int32_t* __restrict__ aq, const double* __restrict__ gain,
                           const double* __restrict__ fwhm, int64_t n_vis, double* __restrict__ vu,
                           double* __restrict__ vv, double* __restrict__ vw, R* __restrict__ vgain,
                           R* __restrict__ vbeta, VisRecD<R>* __restrict__ recD,
                           VisRecG<R>* __restrict__ recG, R* __restrict__ layerDs,
                           const double* __restrict__ layer_sigma, int n_layers) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n_vis) return;
  const double U = u[k], V = v[k], W = w[k];
  vu[k] = U;
  vv[k] = V;
  vw[k] = W;
  if (vgain) {
    const int p = ap[k], q = aq[k];
    double pr = 1.0, pi = 0.0, qr = 1.0, qi = 0.0;
    if (gain) {
      pr = gain[2 * p];
      pi = gain[2 * p + 1];
      qr = gain[2 * q];
      qi = gain[2 * q + 1];
    }
    // c_p conj(c_q)
    vgain[2 * k] = static_cast<R>(pr * qr + pi * qi);
    vgain[2 * k + 1] = static_cast<R>(pi * qr - pr * qi);
  }
  if (vbeta) {
    const double Fp = fwhm[ap[k]], Fq = fwhm[aq[k]];
    vbeta[k] = static_cast<R>(-2.0 * (1.0 / (Fp * Fp) + 1.0 / (Fq * Fq)));
  }
  if (recD) {
    recD[k].u = U;
    recD[k].v = V;
    recD[k].w = W;
    recD[k].pad = 0.0;
  }
  for (int L = 0; L < n_layers; ++L) {
    const double sig2 = layer_sigma[L] * layer_sigma[L];
    const double s = W * sig2;
    const double D = 1.0 / (1.0 + s * s);
    VisRecG<R> g;
    g.A = -D * U;
    g.B = -D * V;
    g.C = 0.5 * D * W;
    g.NW = -W;
    g.E0 = phase_origin<R>() - 0.5 * D * W * sig2 * sig2 * (U * U + V * V);
    g.ur = static_cast<R>(U);
    g.vr = static_cast<R>(V);
    g.wr = static_cast<R>(W);
    g.c1 = static_cast<R>(-M_PI * sig2 * D * taper_scale<R>());
    recG[static_cast<int64_t>(L) * n_vis + k] = g;
    layerDs[(static_cast<int64_t>(L) * n_vis + k) * 2] = static_cast<R>(D);
    layerDs[(static_cast<int64_t>(L) * n_vis + k) * 2 + 1] = static_cast<R>(s);
  }
}

// Adjoint residual records from caller vectors r[nr][n_vis] (complex).
template <typename R>
__global__ void k_adj_prep(const C2<R>* __restrict__ r, int64_t n_vis, int nr,
                           const R* __restrict__ gain, C2<R>* __restrict__ rres,
                           const R* __restrict__ layerDs, int n_layers,
                           ResPolar* __restrict__ rpol) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= n_vis) return;
  const R gr = gain ? gain[2 * k] : R(1), gi = gain ? gain[2 * k + 1] : R(0);
  for (int q = 0; q < nr; ++q) {
    const C2<R> v = r[q * n_vis + k];
    write_res<R>(rres, layerDs, n_layers, n_vis, nr, k, q, gr, gi, v.x, v.y, rpol);
  }
}

template <typename R>
__global__ void k_gather(const R* __restrict__ x, const int32_t* __restrict__ perm, int64_t n,
                         int nr, R* __restrict__ xp) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t o = perm[j];
  for (int r = 0; r < nr; ++r) xp[r * n + j] = x[r * n + o];
}

template <typename R>
__global__ void k_unpermute(const R* __restrict__ src, const int32_t* __restrict__ perm, int64_t n,
                            R* __restrict__ dst) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < n) dst[perm[j]] = src[j];
}

// Dirty image in the caller's order: dst[perm[j]] = max(0, src[j] * a).
template <typename R>
__global__ void k_dirty_out(const R* __restrict__ src, const int32_t* __restrict__ perm,
                            int64_t n, double a, R* __restrict__ dst) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const R v = src[j] * static_cast<R>(a);
  dst[perm[j]] = v > R(0) ? v : R(0);
}

template <typename R>
__global__ void k_copy(const R* __restrict__ src, int64_t n, R* __restrict__ dst) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < n) dst[j] = src[j];
}

__global__ void k_fill_u32(uint32_t* __restrict__ dst, int64_t n) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < n) dst[j] = 0u;
}

template <typename R>
__global__ void k_scale(R* __restrict__ x, int64_t n, R a) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < n) x[j] *= a;
}

// SplitMix64 (Steele, Lea & Flood 2014) in counter form: the value for caller
// pixel o is mix(seed + (o + 1) * gamma); uniform = (z >> 11) * 2^-53.
template <typename R>
__global__ void k_splitmix(const int32_t* __restrict__ perm, int64_t n, uint64_t seed,
                           R* __restrict__ x) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint64_t o = static_cast<uint64_t>(perm[j]);
  uint64_t z = seed + (o + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  x[j] = static_cast<R>(static_cast<double>(z >> 11) * 0x1.0p-53);
}

// Fixed-order two-stage FP64 reductions.  Stage 1: block b reduces the
// contiguous range [b*per, (b+1)*per) with a tree in shared memory; stage 2:
// one block sums the kRedBlocks partials in order.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_red_dot(const R* __restrict__ a, const R* __restrict__ b,
                                                    int64_t n, double* __restrict__ red) {
  __shared__ double sh[kBlock];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = static_cast<int64_t>(blockIdx.x) * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  double ab = 0.0, bb = 0.0;
  for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) {
    const double bv = b[j];
    ab += static_cast<double>(a[j]) * bv;
    bb += bv * bv;
  }
  ab = block_sum(ab, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    red[2 * blockIdx.x] = ab;
    red[2 * blockIdx.x + 1] = bb;
  }
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_red_obj(const R* __restrict__ res, int64_t n_vis,
                                                    const R* __restrict__ img, int64_t n_pix,
                                                    double* __restrict__ red) {
  __shared__ double sh[kBlock];
  double rr = 0.0, s = 0.0, nz = 0.0;
  {
    const int64_t per = (n_vis + gridDim.x - 1) / gridDim.x;
    const int64_t lo = static_cast<int64_t>(blockIdx.x) * per;
    const int64_t hi = lo + per < n_vis ? lo + per : n_vis;
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
      const double a = res[2 * k], b = res[2 * k + 1];
      rr += a * a + b * b;
    }
  }
  {
    const int64_t per = (n_pix + gridDim.x - 1) / gridDim.x;
    const int64_t lo = static_cast<int64_t>(blockIdx.x) * per;
    const int64_t hi = lo + per < n_pix ? lo + per : n_pix;
    for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) {
      const double v = img[j];
      s += v;
      nz += v != 0.0 ? 1.0 : 0.0;
    }
  }
  rr = block_sum(rr, sh);
  s = block_sum(s, sh);
  nz = block_sum(nz, sh);
  if (threadIdx.x == 0) {
    red[3 * blockIdx.x] = rr;
    red[3 * blockIdx.x + 1] = s;
    red[3 * blockIdx.x + 2] = nz;
  }
}

__global__ __launch_bounds__(kBlock) void k_red_final(const double* __restrict__ red, int n_blocks,
                                                      int width, double* __restrict__ out,
                                                      double first_scale) {
  __shared__ double sh[kBlock];
  for (int c = 0; c < width; ++c) {
    double v = 0.0;
    for (int b = threadIdx.x; b < n_blocks; b += blockDim.x) v += red[width * b + c];
    v = block_sum(v, sh);
    if (threadIdx.x == 0) out[c] = c == 0 ? v * first_scale : v;
  }
}

__global__ void k_domain(const double* __restrict__ l, const double* __restrict__ m,
                         const double* __restrict__ sigma, int64_t n_pix,
                         const double* __restrict__ u, const double* __restrict__ v,
                         const double* __restrict__ w, int64_t n_vis, int* __restrict__ flag) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  int bad = 0;
  if (t < n_pix) {
    const double L = l[t], Mm = m[t];
    const double r2 = L * L + Mm * Mm;
    if (!(r2 < 1.0)) bad = 1;  // also catches NaN
    if (sigma) {
      const double s = sigma[t];
      if (!(s >= 0.0) || !isfinite(s)) bad = 1;
    }
  }
  if (t < n_vis) {
    if (!isfinite(u[t]) || !isfinite(v[t]) || !isfinite(w[t])) bad = 1;
  }
  if (bad) atomicAdd(flag, 1);
}

inline unsigned grid1(int64_t n, int b = kBlock) { return static_cast<unsigned>((n + b - 1) / b); }

// Direct-evaluation forward launches.  With `grid` only the segments that are
// not on the grid path are evaluated here (chunk lists fd1, fg1), into the
// partial rows after the grid segments' rows.
template <typename R, int VPL, bool BEAM, int NR, bool HL = false>
hipError_t fwd_launch_t(sl1m_plan* p, const void* xp, hipStream_t st, bool grid = false) {
  const int64_t vt = (p->n_vis + kBlock * VPL - 1) / (kBlock * VPL);
  C2<R>* part = static_cast<C2<R>*>(p->fpart);
  const Chunk* dch = grid ? p->d_chunks1 : p->d_fchunks;
  const int nd = static_cast<int>(grid ? p->fd1.size() : p->fchunks_delta.size());
  const int ng = static_cast<int>(grid ? p->fg1.size() : p->fchunks_gauss.size());
  const int row0 = grid ? p->grid_frows : 0;
  const int rows = row0 + nd + ng;
  if (nd > 0) {
    hipLaunchKernelGGL((k_fwd_delta<R, VPL, BEAM, NR, HL>), dim3(static_cast<unsigned>(vt), nd),
                       dim3(kBlock), 0, st, static_cast<const PixRec<R>*>(p->pixrec),
                       static_cast<const R*>(xp), p->n_pix, p->vu, p->vv, p->vw,
                       static_cast<const R*>(p->vbeta), dch, p->n_vis, part, row0, rows,
                       static_cast<const HLRec*>(p->phl));
  }
  if (ng > 0) {
    hipLaunchKernelGGL((k_fwd_gauss<R, VPL, BEAM, NR>), dim3(static_cast<unsigned>(vt), ng),
                       dim3(kBlock), 0, st, static_cast<const PixRec<R>*>(p->pixrec),
                       static_cast<const R*>(xp), p->n_pix, p->vu, p->vv, p->vw,
                       static_cast<const R*>(p->vbeta), dch + nd, p->n_vis, part, row0 + nd,
                       rows);
  }
  return hipGetLastError();
}

// Direct-evaluation adjoint launches; with `grid` only the tiles of segments
// that are not on the grid path (pd1, pg1).
template <typename R, int PPL, bool BEAM, int NR, bool HL = false>
hipError_t adj_launch_t(sl1m_plan* p, hipStream_t st, bool grid = false) {
  R* part = static_cast<R*>(p->apart);
  const Chunk* dt = grid ? p->d_chunks1 + p->fd1.size() + p->fg1.size() : p->d_ptiles;
  const int nd = static_cast<int>(grid ? p->pd1.size() : p->ptiles_delta.size());
  const int ng = static_cast<int>(grid ? p->pg1.size() : p->ptiles_gauss.size());
  const int sub = p->adj_ppl / PPL;  // blocks per plan tile
  const C2<R>* rres = static_cast<const C2<R>*>(p->rres);
  if (nd > 0) {
    hipLaunchKernelGGL((k_adj_delta<R, PPL, BEAM, NR, HL>), dim3(nd * sub, p->n_achunks),
                       dim3(kBlock), 0, st, static_cast<const VisRecD<R>*>(p->visrecD), rres,
                       static_cast<const R*>(p->vbeta), p->pl, p->pm, p->pc3,
                       static_cast<const R*>(p->pr2), dt, sub, p->adj_kchunk, p->n_vis,
                       p->n_pix, part, static_cast<const HLRec*>(p->vhl));
  }
  if (ng > 0) {
    hipLaunchKernelGGL((k_adj_gauss<R, PPL, BEAM, NR>), dim3(ng * sub, p->n_achunks), dim3(kBlock),
                       0, st, static_cast<const VisRecG<R>*>(p->visrecG), rres,
                       static_cast<const R*>(p->vbeta), p->pl, p->pm, p->pc3, p->pc4,
                       static_cast<const R*>(p->pr2), dt + nd, sub, p->adj_kchunk,
                       p->n_vis, p->n_pix, part);
  }
  return hipGetLastError();
}

}  // namespace

#define SL1M_DISPATCH_R(p, FN, ...) \
  ((p)->precision == SL1M_PREC_FP64 ? FN<double>(__VA_ARGS__) : FN<float>(__VA_ARGS__))

template <typename R>
static hipError_t prep_pixels_t(sl1m_plan* p, const double* l, const double* m, double bc,
                                hipStream_t st) {
  for (const Segment& s : p->segs) {
    if (s.count == 0) continue;
    hipLaunchKernelGGL((k_prep_pixels<R>), dim3(grid1(s.count)), dim3(kBlock), 0, st, p->perm, l,
                       m, s.start, s.count, s.kind, bc, static_cast<PixRec<R>*>(p->pixrec), p->pl,
                       p->pm, p->pc3, p->pc4, static_cast<R*>(p->pscale), static_cast<R*>(p->pr2));
  }
  return hipGetLastError();
}

hipError_t launch_prep_pixels(sl1m_plan* p, const double* l, const double* m, const double*,
                              double beam_coef, hipStream_t st) {
  return SL1M_DISPATCH_R(p, prep_pixels_t, p, l, m, beam_coef, st);
}

template <typename R>
static hipError_t prep_vis_t(sl1m_plan* p, const double* u, const double* v, const double* w,
                             const int32_t* ap, const int32_t* aq, const double* gain,
                             const double* fwhm, const double* d_layer_sigma, hipStream_t st) {
  if (p->n_vis == 0) return hipSuccess;
  hipLaunchKernelGGL((k_prep_vis<R>), dim3(grid1(p->n_vis)), dim3(kBlock), 0, st, u, v, w, ap, aq,
                     gain, fwhm, p->n_vis, p->vu, p->vv, p->vw, static_cast<R*>(p->vgain),
                     static_cast<R*>(p->vbeta), static_cast<VisRecD<R>*>(p->visrecD),
                     static_cast<VisRecG<R>*>(p->visrecG), static_cast<R*>(p->layerDs),
                     d_layer_sigma, p->n_layers);
  return hipGetLastError();
}

hipError_t launch_prep_vis(sl1m_plan* p, const double* u, const double* v, const double* w,
                           const int32_t* ap, const int32_t* aq, const double* gain,
                           const double* fwhm, int32_t, hipStream_t st) {
  // layer sigmas travel in the reduction scratch (plan creation only)
  return SL1M_DISPATCH_R(p, prep_vis_t, p, u, v, w, ap, aq, gain, fwhm, p->red, st);
}

// Float32 hi/lo splits of (l, m, n - 1) per pixel and (u, v, w) per
// visibility (SL1M_PREC_FP32_HILO), from the plan's float64 arrays.
__global__ void k_prep_hilo(const double* __restrict__ a, const double* __restrict__ b,
                            const double* __restrict__ c, int64_t n, HLRec* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  HLRec r;
  hl_split(a[i], r.ah, r.al);
  hl_split(b[i], r.bh, r.bl);
  hl_split(c[i], r.ch, r.cl);
  r.pad0 = r.pad1 = 0.0f;
  out[i] = r;
}

hipError_t launch_prep_hilo(sl1m_plan* p, hipStream_t st) {
  if (!p->hilo) return hipSuccess;
  if (p->n_pix > 0)
    hipLaunchKernelGGL(k_prep_hilo, dim3(grid1(p->n_pix)), dim3(kBlock), 0, st, p->pl, p->pm,
                       p->pc3, p->n_pix, p->phl);
  if (p->n_vis > 0)
    hipLaunchKernelGGL(k_prep_hilo, dim3(grid1(p->n_vis)), dim3(kBlock), 0, st, p->vu, p->vv,
                       p->vw, p->n_vis, p->vhl);
  return hipGetLastError();
}

template <typename R>
static hipError_t gather_t(sl1m_plan* p, const void* x, void* xp, int nr, hipStream_t st) {
  if (p->n_pix == 0) return hipSuccess;
  hipLaunchKernelGGL((k_gather<R>), dim3(grid1(p->n_pix)), dim3(kBlock), 0, st,
                     static_cast<const R*>(x), p->perm, p->n_pix, nr, static_cast<R*>(xp));
  return hipGetLastError();
}
hipError_t launch_gather(sl1m_plan* p, const void* x, void* xp, int nr, hipStream_t st) {
  return SL1M_DISPATCH_R(p, gather_t, p, x, xp, nr, st);
}

// A matrix-core plan whose pixels form one square delta grid has both
// evaluations at hand and takes, per side count, the faster of the two as
// measured at config 2's shape (65,536 pixels x 97,536 visibilities, ms;
// FP32 grid / float16 / bfloat16 matrix cores):
//   forward  2 sides 0.83 / 0.84 / -,  4 sides 1.31 / 0.84 / 1.47,
//            8 sides 2.59 / 1.18 / 1.86
//   adjoint  4 sides 1.45 / 1.22 / -,  8 sides 2.78 / 2.40 / 4.88
// so float16 plans use the matrix-core grid forward and adjoint from 4
// sides, bfloat16 plans the matrix-core forward at 8 only; everything else
// runs the FP32 grid evaluation (the more accurate one).
static bool mfma_forward_call(const sl1m_plan* p, int nr) {
  if (!p->mfma) return false;
  if (!p->grid_mfma) return true;
  return nr >= (p->mfma == SL1M_PREC_MFMA_F16 ? 4 : 8);
}
static bool mfma_adjoint_call(const sl1m_plan* p, int nr) {
  if (!p->mfma) return false;
  if (!p->grid_mfma) return true;
  return p->mfma == SL1M_PREC_MFMA_F16 && nr >= 4;
}

// FP32 hi/lo phase plans: delta pixels, no pair beams, no grid; lanes per
// thread chosen as for the FP32 direct kernels.
static hipError_t forward_hilo(sl1m_plan* p, const void* xp, int nr, hipStream_t st) {
  switch (nr) {
    case 1:
      if (p->fwd_vpl == 1) return fwd_launch_t<float, 1, false, 1, true>(p, xp, st);
      if (p->fwd_vpl == 2) return fwd_launch_t<float, 2, false, 1, true>(p, xp, st);
      return fwd_launch_t<float, 4, false, 1, true>(p, xp, st);
    case 2:
      if (p->fwd_vpl >= 4) return fwd_launch_t<float, 4, false, 2, true>(p, xp, st);
      return fwd_launch_t<float, 2, false, 2, true>(p, xp, st);
    case 4:
      if (p->fwd_vpl >= 2) return fwd_launch_t<float, 2, false, 4, true>(p, xp, st);
      return fwd_launch_t<float, 1, false, 4, true>(p, xp, st);
    case 8:
      if (p->fwd_vpl >= 2) return fwd_launch_t<float, 2, false, 8, true>(p, xp, st);
      return fwd_launch_t<float, 1, false, 8, true>(p, xp, st);
    default:
      return hipErrorInvalidValue;
  }
}
static hipError_t adjoint_hilo(sl1m_plan* p, int nr, hipStream_t st) {
  switch (nr) {
    case 1:
      if (p->adj_ppl == 1) return adj_launch_t<float, 1, false, 1, true>(p, st);
      if (p->adj_ppl == 2) return adj_launch_t<float, 2, false, 1, true>(p, st);
      return adj_launch_t<float, 4, false, 1, true>(p, st);
    case 2:
      if (p->adj_ppl == 1) return adj_launch_t<float, 1, false, 2, true>(p, st);
      return adj_launch_t<float, 2, false, 2, true>(p, st);
    case 4:
      return adj_launch_t<float, 1, false, 4, true>(p, st);
    case 8:
      return adj_launch_t<float, 1, false, 8, true>(p, st);
    default:
      return hipErrorInvalidValue;
  }
}

template <typename R>
static hipError_t forward_t(sl1m_plan* p, const void* xp, int nr, hipStream_t st) {
  if (mfma_forward_call(p, nr)) return launch_mfma_forward(p, xp, nr, st);
  if constexpr (std::is_same<R, float>::value) {
    if (p->hilo) {
      if (p->n_vis == 0 || p->n_fchunks == 0) return hipSuccess;
      return forward_hilo(p, xp, nr, st);
    }
  }
  if (p->n_vis == 0 || p->n_fchunks == 0) return hipSuccess;
  const bool bm = p->beam_pair;
  if (nr == 1 && p->grid) {
    // grid segments first, then the direct segments (no per-pair beams here)
    hipError_t e = launch_grid_forward(p, xp, st);
    if (e != hipSuccess || (p->fd1.empty() && p->fg1.empty())) return e;
    if (p->fwd_vpl == 1) return fwd_launch_t<R, 1, false, 1>(p, xp, st, true);
    if (p->fwd_vpl == 2) return fwd_launch_t<R, 2, false, 1>(p, xp, st, true);
    return fwd_launch_t<R, 4, false, 1>(p, xp, st, true);
  }
  if (grid_multi_ok(p, nr)) {
    hipError_t e = launch_grid_forward_multi(p, xp, nr, st);
    if (e != hipSuccess || (p->fd1.empty() && p->fg1.empty())) return e;
    if (nr == 2) return fwd_launch_t<R, 2, false, 2>(p, xp, st, true);
    if (nr == 4) return fwd_launch_t<R, 1, false, 4>(p, xp, st, true);
    return fwd_launch_t<R, 1, false, 8>(p, xp, st, true);
  }
  switch (nr) {
    case 1:
      if (bm) return fwd_launch_t<R, 4, true, 1>(p, xp, st);
      if (p->fwd_vpl == 1) return fwd_launch_t<R, 1, false, 1>(p, xp, st);
      if (p->fwd_vpl == 2) return fwd_launch_t<R, 2, false, 1>(p, xp, st);
      return fwd_launch_t<R, 4, false, 1>(p, xp, st);
    // several right-hand sides: keep >= 2 visibilities per lane when the plan
    // has enough visibilities, so each scalar pixel load feeds more work
    case 2:
      if (p->fwd_vpl >= 4)
        return bm ? fwd_launch_t<R, 4, true, 2>(p, xp, st) : fwd_launch_t<R, 4, false, 2>(p, xp, st);
      return bm ? fwd_launch_t<R, 2, true, 2>(p, xp, st) : fwd_launch_t<R, 2, false, 2>(p, xp, st);
    case 4:
      if (p->fwd_vpl >= 2)
        return bm ? fwd_launch_t<R, 2, true, 4>(p, xp, st) : fwd_launch_t<R, 2, false, 4>(p, xp, st);
      return bm ? fwd_launch_t<R, 1, true, 4>(p, xp, st) : fwd_launch_t<R, 1, false, 4>(p, xp, st);
    case 8:
      if (p->fwd_vpl >= 2)
        return bm ? fwd_launch_t<R, 2, true, 8>(p, xp, st) : fwd_launch_t<R, 2, false, 8>(p, xp, st);
      return bm ? fwd_launch_t<R, 1, true, 8>(p, xp, st) : fwd_launch_t<R, 1, false, 8>(p, xp, st);
    default:
      return hipErrorInvalidValue;
  }
}
hipError_t launch_forward(sl1m_plan* p, const void* xp, int nr, hipStream_t st) {
  return SL1M_DISPATCH_R(p, forward_t, p, xp, nr, st);
}

int forward_rows(const sl1m_plan* p, int nr) {
  if (p->mfma) return p->grid_mfma ? p->grid_frows : p->n_mfchunks;
  if ((nr == 1 && p->grid) || grid_multi_ok(p, nr))
    return static_cast<int>(p->grid_frows + p->fd1.size() + p->fg1.size());
  return p->n_fchunks;
}

template <typename R>
static hipError_t fwd_reduce_t(sl1m_plan* p, const void* data, void* out, bool recs, int nr,
                               hipStream_t st) {
  if (p->n_vis == 0) return hipSuccess;
  hipLaunchKernelGGL((k_fwd_reduce<R>), dim3(grid1(p->n_vis)), dim3(kBlock), 0, st,
                     static_cast<const C2<R>*>(p->fpart), forward_rows(p, nr), p->n_vis, nr,
                     static_cast<const R*>(p->vgain), static_cast<const C2<R>*>(data),
                     static_cast<C2<R>*>(out), recs ? static_cast<C2<R>*>(p->rres) : nullptr,
                     static_cast<const R*>(p->layerDs), p->n_layers,
                     recs && nr == 1 ? p->rpol : nullptr);
  return hipGetLastError();
}
hipError_t launch_forward_reduce(sl1m_plan* p, const void* data, void* out, bool recs, int nr,
                                 hipStream_t st) {
  return SL1M_DISPATCH_R(p, fwd_reduce_t, p, data, out, recs, nr, st);
}

template <typename R>
static hipError_t adj_prep_t(sl1m_plan* p, const void* r, int nr, hipStream_t st) {
  if (p->n_vis == 0) return hipSuccess;
  hipLaunchKernelGGL((k_adj_prep<R>), dim3(grid1(p->n_vis)), dim3(kBlock), 0, st,
                     static_cast<const C2<R>*>(r), p->n_vis, nr, static_cast<const R*>(p->vgain),
                     static_cast<C2<R>*>(p->rres), static_cast<const R*>(p->layerDs),
                     p->n_layers, nr == 1 ? p->rpol : nullptr);
  return hipGetLastError();
}
hipError_t launch_adjoint_prep(sl1m_plan* p, const void* r, int nr, hipStream_t st) {
  return SL1M_DISPATCH_R(p, adj_prep_t, p, r, nr, st);
}

template <typename R>
static hipError_t adjoint_t(sl1m_plan* p, int nr, hipStream_t st) {
  if (mfma_adjoint_call(p, nr)) return launch_mfma_adjoint(p, nr, st);
  if (p->n_pix == 0 || p->n_achunks == 0) return hipSuccess;
  if constexpr (std::is_same<R, float>::value) {
    if (p->hilo) return adjoint_hilo(p, nr, st);
  }
  const bool bm = p->beam_pair;
  if (nr == 1 && p->grid) {
    hipError_t e = launch_grid_adjoint(p, st);
    if (e != hipSuccess || (p->pd1.empty() && p->pg1.empty())) return e;
    if (p->adj_ppl == 1) return adj_launch_t<R, 1, false, 1>(p, st, true);
    if (p->adj_ppl == 2) return adj_launch_t<R, 2, false, 1>(p, st, true);
    return adj_launch_t<R, 4, false, 1>(p, st, true);
  }
  if (grid_multi_ok(p, nr)) {
    hipError_t e = launch_grid_adjoint_multi(p, nr, st);
    if (e != hipSuccess || (p->pd1.empty() && p->pg1.empty())) return e;
    if (nr == 2) return adj_launch_t<R, 1, false, 2>(p, st, true);
    if (nr == 4) return adj_launch_t<R, 1, false, 4>(p, st, true);
    return adj_launch_t<R, 1, false, 8>(p, st, true);
  }
  switch (nr) {
    case 1:
      if (bm) return adj_launch_t<R, 4, true, 1>(p, st);
      if (p->adj_ppl == 1) return adj_launch_t<R, 1, false, 1>(p, st);
      if (p->adj_ppl == 2) return adj_launch_t<R, 2, false, 1>(p, st);
      return adj_launch_t<R, 4, false, 1>(p, st);
    case 2:
      if (p->adj_ppl == 1)
        return bm ? adj_launch_t<R, 1, true, 2>(p, st) : adj_launch_t<R, 1, false, 2>(p, st);
      return bm ? adj_launch_t<R, 2, true, 2>(p, st) : adj_launch_t<R, 2, false, 2>(p, st);
    case 4:
      return bm ? adj_launch_t<R, 1, true, 4>(p, st) : adj_launch_t<R, 1, false, 4>(p, st);
    case 8:
      return bm ? adj_launch_t<R, 1, true, 8>(p, st) : adj_launch_t<R, 1, false, 8>(p, st);
    default:
      return hipErrorInvalidValue;
  }
}
hipError_t launch_adjoint(sl1m_plan* p, int nr, hipStream_t st) {
  return SL1M_DISPATCH_R(p, adjoint_t, p, nr, st);
}

template <typename R>
static hipError_t adj_reduce_t(sl1m_plan* p, void* g, bool unpermute, int nr, hipStream_t st) {
  if (p->n_pix == 0) return hipSuccess;
  hipLaunchKernelGGL((k_adj_reduce<R>), dim3(grid1(p->n_pix, kRowPix)), dim3(kBlock), 0, st,
                     static_cast<const R*>(p->apart), p->n_achunks, p->n_pix, nr,
                     static_cast<const R*>(p->pscale), unpermute ? p->perm : nullptr,
                     static_cast<R*>(g));
  return hipGetLastError();
}
hipError_t launch_adjoint_reduce(sl1m_plan* p, void* g, bool unpermute, int nr, hipStream_t st) {
  return SL1M_DISPATCH_R(p, adj_reduce_t, p, g, unpermute, nr, st);
}

template <typename R>
static hipError_t fista_t(sl1m_plan* p, hipStream_t st) {
  if (p->n_pix > 0)
    hipLaunchKernelGGL((k_fista<R>), dim3(grid1(p->n_pix, kRowPix)), dim3(kBlock), 0, st,
                       static_cast<const R*>(p->apart), p->n_achunks, p->n_pix,
                       static_cast<const R*>(p->pscale), static_cast<R*>(p->xperm),
                       static_cast<R*>(p->img), p->scal, p->flag);
  hipLaunchKernelGGL(k_tstep, dim3(1), dim3(64), 0, st, p->scal);
  return hipGetLastError();
}
hipError_t launch_fista_update(sl1m_plan* p, hipStream_t st) {
  return SL1M_DISPATCH_R(p, fista_t, p, st);
}

template <typename R>
static hipError_t prox_t(sl1m_plan* p, hipStream_t st) {
  if (p->n_pix > 0)
    hipLaunchKernelGGL((k_prox<R>), dim3(grid1(p->n_pix, kRowPix)), dim3(kBlock), 0, st,
                       static_cast<const R*>(p->apart), p->n_achunks, p->n_pix,
                       static_cast<const R*>(p->pscale), static_cast<const R*>(p->xperm),
                       static_cast<R*>(p->zbuf), p->scal, p->flag);
  return hipGetLastError();
}
hipError_t launch_prox(sl1m_plan* p, hipStream_t st) {
  return SL1M_DISPATCH_R(p, prox_t, p, st);
}

template <typename R>
static hipError_t mfista_select_t(sl1m_plan* p, hipStream_t st) {
  if (p->n_pix > 0)
    hipLaunchKernelGGL((k_mfista_select<R>), dim3(grid1(p->n_pix)), dim3(kBlock), 0, st,
                       static_cast<R*>(p->xperm), static_cast<R*>(p->img),
                       static_cast<const R*>(p->zbuf), p->n_pix, p->scal, p->red_out);
  hipLaunchKernelGGL(k_mfista_step, dim3(1), dim3(64), 0, st, p->scal, p->red_out);
  return hipGetLastError();
}
hipError_t launch_mfista_select(sl1m_plan* p, hipStream_t st) {
  return SL1M_DISPATCH_R(p, mfista_select_t, p, st);
}

hipError_t launch_mfista_init(sl1m_plan* p, hipStream_t st) {
  hipLaunchKernelGGL(k_mfista_init, dim3(1), dim3(64), 0, st, p->scal, p->red_out);
  return hipGetLastError();
}

hipError_t launch_fill(void* dst, size_t n_elems, size_t elem_bytes, hipStream_t st) {
  const int64_t words = static_cast<int64_t>((n_elems * elem_bytes + 3) / 4);
  if (words == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid1(words)), dim3(kBlock), 0, st,
                     static_cast<uint32_t*>(dst), words);
  return hipGetLastError();
}

template <typename R>
static hipError_t splitmix_t(sl1m_plan* p, uint64_t seed, void* dst, hipStream_t st) {
  if (p->n_pix == 0) return hipSuccess;
  hipLaunchKernelGGL((k_splitmix<R>), dim3(grid1(p->n_pix)), dim3(kBlock), 0, st, p->perm,
                     p->n_pix, seed, static_cast<R*>(dst));
  return hipGetLastError();
}
hipError_t launch_splitmix_start(sl1m_plan* p, uint64_t seed, void* dst, hipStream_t st) {
  return SL1M_DISPATCH_R(p, splitmix_t, p, seed, dst, st);
}

template <typename R>
static hipError_t scale_t(sl1m_plan*, void* x, int64_t n, double a, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_scale<R>), dim3(grid1(n)), dim3(kBlock), 0, st, static_cast<R*>(x), n,
                     static_cast<R>(a));
  return hipGetLastError();
}
hipError_t launch_scale(sl1m_plan* p, void* x, int64_t n, double a, hipStream_t st) {
  return SL1M_DISPATCH_R(p, scale_t, p, x, n, a, st);
}

template <typename R>
static hipError_t unpermute_t(sl1m_plan* p, const void* src, void* dst, hipStream_t st) {
  if (p->n_pix == 0) return hipSuccess;
  hipLaunchKernelGGL((k_unpermute<R>), dim3(grid1(p->n_pix)), dim3(kBlock), 0, st,
                     static_cast<const R*>(src), p->perm, p->n_pix, static_cast<R*>(dst));
  return hipGetLastError();
}
hipError_t launch_unpermute(sl1m_plan* p, const void* src, void* dst, hipStream_t st) {
  return SL1M_DISPATCH_R(p, unpermute_t, p, src, dst, st);
}

template <typename R>
static hipError_t dirty_out_t(sl1m_plan* p, const void* src, void* dst, double a, hipStream_t st) {
  if (p->n_pix == 0) return hipSuccess;
  hipLaunchKernelGGL((k_dirty_out<R>), dim3(grid1(p->n_pix)), dim3(kBlock), 0, st,
                     static_cast<const R*>(src), p->perm, p->n_pix, a, static_cast<R*>(dst));
  return hipGetLastError();
}
hipError_t launch_dirty_out(sl1m_plan* p, const void* src, void* dst, double a, hipStream_t st) {
  return SL1M_DISPATCH_R(p, dirty_out_t, p, src, dst, a, st);
}

template <typename R>
static hipError_t copy_t(sl1m_plan*, const void* src, void* dst, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_copy<R>), dim3(grid1(n)), dim3(kBlock), 0, st, static_cast<const R*>(src),
                     n, static_cast<R*>(dst));
  return hipGetLastError();
}
hipError_t launch_copy_real(sl1m_plan* p, const void* src, void* dst, int64_t n, hipStream_t st) {
  return SL1M_DISPATCH_R(p, copy_t, p, src, dst, n, st);
}

template <typename R>
static hipError_t dot_t(sl1m_plan* p, const void* a, const void* b, hipStream_t st) {
  hipLaunchKernelGGL((k_red_dot<R>), dim3(kRedBlocks), dim3(kBlock), 0, st,
                     static_cast<const R*>(a), static_cast<const R*>(b), p->n_pix, p->red);
  hipLaunchKernelGGL(k_red_final, dim3(1), dim3(kBlock), 0, st, p->red, kRedBlocks, 2, p->red_out,
                     1.0);
  return hipGetLastError();
}
hipError_t launch_dot_norm(sl1m_plan* p, const void* a, const void* b, hipStream_t st) {
  return SL1M_DISPATCH_R(p, dot_t, p, a, b, st);
}

template <typename R>
static hipError_t obj_t(sl1m_plan* p, const void* res, const void* img, hipStream_t st) {
  hipLaunchKernelGGL((k_red_obj<R>), dim3(kRedBlocks), dim3(kBlock), 0, st,
                     static_cast<const R*>(res), p->n_vis, static_cast<const R*>(img), p->n_pix,
                     p->red);
  hipLaunchKernelGGL(k_red_final, dim3(1), dim3(kBlock), 0, st, p->red, kRedBlocks, 3, p->red_out,
                     0.5);
  return hipGetLastError();
}
hipError_t launch_objective_terms(sl1m_plan* p, const void* res, const void* img,
                                  hipStream_t st) {
  return SL1M_DISPATCH_R(p, obj_t, p, res, img, st);
}

hipError_t launch_domain_check(sl1m_plan* p, const double* l, const double* m,
                               const double* sigma, const double* u, const double* v,
                               const double* w, hipStream_t st) {
  const int64_t n = p->n_pix > p->n_vis ? p->n_pix : p->n_vis;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_domain, dim3(grid1(n)), dim3(kBlock), 0, st, l, m, sigma, p->n_pix, u, v,
                     w, p->n_vis, p->flag);
  return hipGetLastError();
}

}  // namespace sl1m
