// Harmonic-space kernels: the wavelet tiling of Eqs. (4), (6) and (8) (a diagonal multiply by
// the real kernels kappa_j(l), eta(l), with truncation / zero-extension between band-limits
// in the multiresolution algorithm of Sect. 3.1), and the conversion between the user's
// f_lm layout (index l*l + l + m) and the packed (m, l) column layout of the Legendre kernels.
// Every row of band-limit k: (m, l), 0 <= m <= l < k, at tri_off(k, m) + l - m, C columns.
#include "common.h"
#include "../../include/s2let_mi355x.h"

namespace s2let {

// blockIdx.y = m; threads over (l - m) * C + c.
// herm (real maps only): use the Hermitian part (f_lm + (-1)^m conj f_{l,-m}) / 2 of the input.
__global__ void k_unpack(const double2* __restrict__ flm, double* __restrict__ S,
                         const double* __restrict__ dfac, int k, int Lt, int C, int nb, int real,
                         long long map_stride, int herm) {
  const int m = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int len = k - m;
  if (idx >= len * C) return;
  const int r = idx / C, c = idx % C;
  const int l = m + r;
  const double d = dfac[tri_off(Lt, m) + r];
  double v = 0.0;
  if (real) {
    const int a = c >> 1;
    if (a < nb) {
      const double2 f = flm[(size_t)a * map_stride + (size_t)l * l + l + m];
      v = (c & 1) ? f.y : f.x;
      if (herm) {
        const double2 g = flm[(size_t)a * map_stride + (size_t)l * l + l - m];
        const double sg = (m & 1) ? -1.0 : 1.0;
        v = 0.5 * (v + sg * ((c & 1) ? -g.y : g.x));
      }
    }
  } else {
    const int a = c >> 2, part = c & 3;
    if (a < nb) {
      if (part < 2) {
        const double2 f = flm[(size_t)a * map_stride + (size_t)l * l + l + m];
        v = (part & 1) ? f.y : f.x;
      } else if (m > 0) {
        const double2 f = flm[(size_t)a * map_stride + (size_t)l * l + l - m];
        const double sg = (m & 1) ? -1.0 : 1.0;
        v = sg * ((part & 1) ? f.y : f.x);
      }
    }
  }
  S[(tri_off(k, m) + r) * C + c] = d * v;
}

// One thread per (m, l, map).
__global__ void k_pack(const double* __restrict__ R, int nparts, long long pstride, double2* __restrict__ flm,
                       const double* __restrict__ dfac, int k, int Lt, int C, int nb, int real,
                       long long map_stride) {
  const int m = blockIdx.y;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int len = k - m;
  if (idx >= len * nb) return;
  const int r = idx / nb, a = idx % nb;
  const int l = m + r;
  const double d = dfac[tri_off(Lt, m) + r];
  const double* row = R + (tri_off(k, m) + r) * C;
  double2* out = flm + (size_t)a * map_stride;
  const double sg = (m & 1) ? -1.0 : 1.0;
  const int c0 = real ? 2 * a : 4 * a;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int g = 0; g < nparts; ++g) {
    const double* rg = row + (size_t)g * pstride;
    v[0] += rg[c0];
    v[1] += rg[c0 + 1];
    if (!real) {
      v[2] += rg[c0 + 2];
      v[3] += rg[c0 + 3];
    }
  }
  if (real) {
    const double2 f = make_double2(d * v[0], d * v[1]);
    out[(size_t)l * l + l + m] = f;
    if (m > 0) out[(size_t)l * l + l - m] = make_double2(sg * f.x, -sg * f.y);
  } else {
    out[(size_t)l * l + l + m] = make_double2(d * v[0], d * v[1]);
    if (m > 0) out[(size_t)l * l + l - m] = make_double2(sg * d * v[2], sg * d * v[3]);
  }
}

// Row q of the triangle of band-limit kl (rows ordered by m, then r = l - m): the largest m with
// tri_off(kl, m) <= q, from the smaller root of m^2 - (2 kl + 1) m + 2 q = 0, then corrected.
__device__ __forceinline__ void tri_row_mr(int kl, long long q, int& m, int& r) {
  const double b = 2.0 * kl + 1.0;
  int mm = (int)floor(0.5 * (b - sqrt(b * b - 8.0 * (double)q)));
  mm = mm < 0 ? 0 : (mm > kl - 1 ? kl - 1 : mm);
  while (mm > 0 && tri_off(kl, mm) > q) --mm;
  while (mm + 1 < kl && tri_off(kl, mm + 1) <= q) ++mm;
  m = mm;
  r = (int)(q - tri_off(kl, mm));
}

// dst (band-limit kd) (+= for rows l < kacc, = above) kern[l] d_lm^2 src (band-limit ks), over the
// triangle of band-limit klim: one thread per (row, column pair); rows with kern[l] = 0 give zero
// without reading src.  klim = min(ks, kd), or kd to zero-fill the rows l >= ks of dst.
__global__ void k_tile(const double* __restrict__ src, int ks, int nparts, long long pstride,
                       double* __restrict__ dst, int kd, int klim, const double* __restrict__ kern,
                       const double* __restrict__ dfac, int Lt, int C, int kacc) {
  const int CP = C / 2;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tri_rows(klim) * CP) return;
  const long long q = idx / CP;
  const int cp = (int)(idx % CP);
  int m, r;
  tri_row_mr(klim, q, m, r);
  const int l = m + r;
  double2 v = make_double2(0.0, 0.0);
  // rows where the kernel vanishes are not read (a forward transform with a degree floor leaves them
  // unwritten)
  if (l < ks && kern[l] != 0.0) {
    const double d = dfac[tri_off(Lt, m) + r];
    const double2* at = reinterpret_cast<const double2*>(src + (tri_off(ks, m) + r) * C) + cp;
    double2 x = make_double2(0.0, 0.0);
    for (int g = 0; g < nparts; ++g) {
      const double2 y = at[(size_t)g * (pstride / 2)];
      x.x += y.x;
      x.y += y.y;
    }
    const double f = kern[l] * d * d;
    v = make_double2(f * x.x, f * x.y);
  }
  double2* o = reinterpret_cast<double2*>(dst + (tri_off(kd, m) + r) * C) + cp;
  if (l < kacc)
    *o = make_double2(o->x + v.x, o->y + v.y);
  else
    *o = v;
}

// dst = scale * src with the (theta, m) rows transposed: src[(a*k + b)*C + c] -> dst[(b*k + a)*C + c].
// Used by the adjoint transforms, which skip the theta quadrature (inverse adjoint) or run it
// between the Legendre step and the phi stage (forward adjoint).
__global__ void k_transpose_rows(const double* __restrict__ src, double* __restrict__ dst, int k, int C,
                                 double scale) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)k * k * C;
  if (idx >= total) return;
  const int c = (int)(idx % C);
  const size_t row = idx / C;
  const int a = (int)(row / k), b = (int)(row % k);
  dst[((size_t)b * k + a) * C + c] = scale * src[idx];
}

hipError_t launch_transpose_rows(const Batch& b, int k, const double* src, double* dst, double scale,
                                 hipStream_t s) {
  const size_t total = (size_t)k * k * b.C;
  const unsigned nblk = (unsigned)((total + 255) / 256);
  k_transpose_rows<<<nblk, 256, 0, s>>>(src, dst, k, b.C, scale);
  return hipGetLastError();
}

// Hard thresholding (Eq. (23)): samples [off, off + n) of every map (map stride `stride`
// samples) with magnitude below thr are set to zero; complex samples are (re, im) pairs.
__global__ void k_hard_threshold(double* __restrict__ w, long long off, long long n, long long stride, int nmaps,
                                 int cplx, double thr) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (i >= n || a >= nmaps) return;
  if (cplx) {
    double2* p = reinterpret_cast<double2*>(w) + (size_t)a * stride + off + i;
    const double2 v = *p;
    if (hypot(v.x, v.y) < thr) *p = make_double2(0.0, 0.0);
  } else {
    double* p = w + (size_t)a * stride + off + i;
    if (fabs(*p) < thr) *p = 0.0;
  }
}

hipError_t launch_hard_threshold(double* w, long long off, long long n, long long stride, int nmaps, bool cplx,
                                 double thr, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const size_t esz = cplx ? 2 : 1;
  for (int a0 = 0; a0 < nmaps; a0 += 65535) {   // grid.y stays within its limit
    const int na = std::min(65535, nmaps - a0);
    dim3 grid((unsigned)((n + 255) / 256), na);
    k_hard_threshold<<<grid, 256, 0, s>>>(w + (size_t)a0 * stride * esz, off, n, stride, na, cplx ? 1 : 0, thr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_unpack_flm(const LegTables& G, const Batch& b, int k, const double2* flm, double* S,
                             hipStream_t s, bool herm) {
  dim3 grid((k * b.C + 255) / 256, k);
  k_unpack<<<grid, 256, 0, s>>>(flm, S, G.dfac, k, G.Lt, b.C, b.nb, b.reality == S2LET_REAL,
                                (long long)k * k, herm ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_pack_flm(const LegTables& G, const Batch& b, int k, const double* R, int nparts,
                           long long part_stride, double2* flm, hipStream_t s) {
  dim3 grid((k * b.nb + 255) / 256, k);
  k_pack<<<grid, 256, 0, s>>>(R, nparts, part_stride, flm, G.dfac, k, G.Lt, b.C, b.nb,
                              b.reality == S2LET_REAL, (long long)k * k);
  return hipGetLastError();
}

hipError_t launch_tile(const LegTables& G, const Batch& b, const double* src, int ks, int nparts,
                       long long part_stride, double* dst, int kd, const double* kern, int kacc, bool zero_fill,
                       hipStream_t s) {
  const int klim = zero_fill ? kd : (ks < kd ? ks : kd);
  if (b.C & 1) return hipErrorInvalidValue;
  const long long total = tri_rows(klim) * (b.C / 2);
  if (total == 0) return hipSuccess;
  k_tile<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(src, ks, nparts, part_stride, dst, kd, klim, kern, G.dfac,
                                                         G.Lt, b.C, kacc);
  return hipGetLastError();
}

}  // namespace s2let
