// Host-side tables of the transform, computed in long double and copied to device memory once
// per (device, size): odd-length DFT chirps and their Bluestein kernels, the theta-quadrature
// weight kernel, FFT twiddles, MW node cosines/sines, and the Legendre recursion factors.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <vector>

#include "../../include/s2let_mi355x.h"
#include "common.h"
#include "plan.h"

namespace s2let {

typedef long double LD;
typedef std::complex<LD> cLD;
static const LD PI_L = 3.141592653589793238462643383279502884L;

// exp(-i pi q^2 / n) with the angle reduced exactly: q^2 mod 2n in integers.
static cLD chirp_value(long long q, long long n) {
  const long long r = ((q % (2 * n)) * (q % (2 * n))) % (2 * n);
  const LD ang = -PI_L * (LD)r / (LD)n;
  return cLD(cosl(ang), sinl(ang));
}

// In-place radix-2 FFT (sign -1), long double, size a power of two.
static void host_fft(std::vector<cLD>& a) {
  const size_t N = a.size();
  for (size_t i = 1, j = 0; i < N; ++i) {
    size_t bit = N >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= N; len <<= 1) {
    for (size_t i = 0; i < N; i += len) {
      for (size_t q = 0; q < len / 2; ++q) {
        const LD ang = -2.0L * PI_L * (LD)q / (LD)len;
        const cLD w(cosl(ang), sinl(ang));
        const cLD u = a[i + q], v = a[i + q + len / 2] * w;
        a[i + q] = u + v;
        a[i + q + len / 2] = u - v;
      }
    }
  }
}

template <typename T>
static hipError_t upload(T** dst, const std::vector<T>& src) {
  hipError_t e = hipMalloc((void**)dst, sizeof(T) * (src.empty() ? 1 : src.size()));
  if (e != hipSuccess) return e;
  if (!src.empty()) e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
  return e;
}

static std::vector<double2> to_d2(const std::vector<cLD>& v) {
  std::vector<double2> o(v.size());
  for (size_t i = 0; i < v.size(); ++i) o[i] = make_double2((double)v[i].real(), (double)v[i].imag());
  return o;
}

// n = product of odd radices <= 13 (largest first), or false.
static bool factor_odd(int n, int* rad, int* nrad) {
  static const int cand[] = {13, 11, 9, 7, 5, 3};
  int cnt = 0;
  for (int r : cand) {
    while (n % r == 0 && n > 1) {
      if (cnt == 8) return false;
      rad[cnt++] = r;
      n /= r;
    }
  }
  *nrad = cnt;
  return n == 1;
}

static std::vector<cLD> roots_two_level(long long N, long long base, int count) {
  std::vector<cLD> v(count > 0 ? count : 1);
  for (int p = 0; p < count; ++p) {
    const long long e = ((long long)p * base) % N;
    const LD ang = -2.0L * PI_L * (LD)e / (LD)N;
    v[p] = cLD(cosl(ang), sinl(ang));
  }
  return v;
}

hipError_t build_sht_tables(int k, ShtTables* T) {
  const int n = 2 * k - 1;
  T->k = k;
  T->n = n;
  int rad[8], nrad = 0;
  const bool mixed = n > 1 && factor_odd(n, rad, &nrad);
  T->nrad = mixed ? nrad : 0;
  for (int s = 0; s < 8; ++s) T->rad[s] = (mixed && s < nrad) ? rad[s] : 0;
  T->M = mixed ? 0 : next_pow2(2 * n - 1);
  T->logM = mixed ? 0 : ilog2(T->M);
  T->Nc = next_pow2(2 * k - 1);
  T->logNc = ilog2(T->Nc);
  const int P = std::max(T->M, T->Nc);
  T->logP = ilog2(P);
  T->loglo = T->logP < 6 ? T->logP : 6;   // 64-entry low table (the compiled transforms read it so)
  hipError_t e;

  // W_n two-level table (64-entry low part)
  {
    const int nhi = (n + 63) / 64;
    if ((e = upload(&T->twn_lo, to_d2(roots_two_level(n, 1, 64)))) != hipSuccess) return e;
    if ((e = upload(&T->twn_hi, to_d2(roots_two_level(n, 64, nhi)))) != hipSuccess) return e;
  }
  // Bluestein tables
  if (!mixed) {
    const int M = T->M;
    std::vector<cLD> chirp(n);
    for (int q = 0; q < n; ++q) chirp[q] = chirp_value(q, n);
    std::vector<cLD> b(M, cLD(0, 0));
    for (int q = -(n - 1); q <= n - 1; ++q) b[((q % M) + M) % M] = std::conj(chirp[q < 0 ? -q : q]);
    host_fft(b);
    for (auto& v : b) v /= (LD)M;
    if ((e = upload(&T->chirp, to_d2(chirp))) != hipSuccess) return e;
    if ((e = upload(&T->bhat, to_d2(b))) != hipSuccess) return e;
  }
  // correlation kernels of the two frequency-parity classes:
  //   Kt_Q(c) = w_e(2Q - 2c) for c in [Q-(k-1), Q+(k-1)], wrapped mod Nc; stored as FFT / (Nc n^2)
  for (int Q = 0; Q < 2; ++Q) {
    const int Nc = T->Nc;
    std::vector<cLD> kt(Nc, cLD(0, 0));
    for (int c = Q - (k - 1); c <= Q + (k - 1); ++c) {
      const LD pp = (LD)(2 * Q - 2 * c);
      kt[((c % Nc) + Nc) % Nc] = cLD(2.0L / (1.0L - pp * pp), 0);
    }
    host_fft(kt);
    for (auto& v : kt) v /= (LD)Nc * (LD)n * (LD)n;
    if ((e = upload(Q == 0 ? &T->khat0 : &T->khat1, to_d2(kt))) != hipSuccess) return e;
    if (Q == 0) {
      std::vector<double> kr(Nc);
      for (int q = 0; q < Nc; ++q) kr[q] = (double)kt[q].real();
      if ((e = upload(&T->khr, kr)) != hipSuccess) return e;
    }
  }
  // W_P two-level table
  {
    const int nlo = 1 << T->loglo, nhi = P / nlo;
    if ((e = upload(&T->tw_lo, to_d2(roots_two_level(P, 1, nlo)))) != hipSuccess) return e;
    if ((e = upload(&T->tw_hi, to_d2(roots_two_level(P, nlo, nhi)))) != hipSuccess) return e;
  }

  std::vector<double> xt(k), st(k), ut(k), sx(k);
  for (int t = 0; t < k; ++t) {
    const LD th = PI_L * (LD)(2 * t + 1) / (LD)n;
    xt[t] = (double)cosl(th);
    st[t] = (double)sinl(th);
    // |cos| - 1 = -2 sin^2(theta'/2) with theta' the angular distance to the nearer pole
    const LD thp = (2 * t + 1 <= n / 2) ? th : PI_L * (LD)(n - 2 * t - 1) / (LD)n;
    const LD h = sinl(0.5L * thp);
    ut[t] = (double)(-2.0L * h * h);
    sx[t] = (2 * (2 * t + 1) <= n) ? 1.0 : -1.0;
  }
  st[k - 1] = 0.0;   // theta_{k-1} = pi exactly
  xt[k - 1] = -1.0;
  ut[k - 1] = 0.0;
  sx[k - 1] = -1.0;

  // Pole column of the odd-parity theta operator.  For odd m the weight's p = +-1 terms, which
  // the kernels leave out, cancel everywhere except in row and column t = k-1 (the south
  // pole), where they are c_t = Q(t, k-1) = Q(k-1, t): the steps of the quadrature applied to
  // the unit input at the pole, g = delta_{k-1} (Ghat_j = (-1)^j / n), with the full weight
  //   I_j' = sum_j Ghat_j w(j + j'),  H(theta_t) = (1/n) sum_j' I_j' e^{-i j' theta_t},
  //   c_t = H(t) - H(n-1-t) (t < k-1),  c_{k-1} = H(k-1)   (real up to rounding).
  std::vector<double> pole(k), pole_s;
  {
    std::vector<cLD> I(n);
    for (int jp = -(k - 1); jp <= k - 1; ++jp) {
      cLD acc(0, 0);
      for (int j = -(k - 1); j <= k - 1; ++j) {
        const int pp = j + jp;
        cLD wv(0, 0);
        if ((pp & 1) == 0) wv = cLD(2.0L / (1.0L - (LD)pp * (LD)pp), 0);
        else if (pp == 1) wv = cLD(0, PI_L / 2);
        else if (pp == -1) wv = cLD(0, -PI_L / 2);
        acc += ((j & 1) ? -1.0L : 1.0L) * wv;
      }
      I[jp + k - 1] = acc / (LD)n;
    }
    // e^{-i j' theta_t} = e^{-i pi j' (2t+1) / n}: table over the residue of j'(2t+1) mod 2n
    std::vector<cLD> ex(2 * n);
    for (int q = 0; q < 2 * n; ++q) ex[q] = cLD(cosl(-PI_L * q / n), sinl(-PI_L * q / n));
    auto H = [&](int t) {
      cLD acc(0, 0);
      for (int jp = -(k - 1); jp <= k - 1; ++jp) {
        const long long q = (((long long)jp * (2 * t + 1)) % (2 * n) + 2 * n) % (2 * n);
        acc += I[jp + k - 1] * ex[q];
      }
      return acc / (LD)n;
    };
    for (int t = 0; t < k - 1; ++t) pole[t] = (double)(H(t) - H(n - 1 - t)).real();
    pole[k - 1] = (double)H(k - 1).real();
    if (k == 2048 || k == 1024 || k == 512 || k == 256 || k == 128 || k == 64) {
      // the same operator evaluated on the psi grid (N = 2k points psi_s = pi (2s+1) / N):
      //   H(psi_s) = (1/N) sum_j' I_j' e^{-i j' psi_s},  c_s = H(s) - H(N-1-s)  (odd fold), s < k
      const int N = 2 * k;
      std::vector<cLD> exN(2 * N);
      for (int q = 0; q < 2 * N; ++q) exN[q] = cLD(cosl(-PI_L * q / N), sinl(-PI_L * q / N));
      auto Hs = [&](int t) {
        cLD acc(0, 0);
        for (int jp = -(k - 1); jp <= k - 1; ++jp) {
          const long long q = (((long long)jp * (2 * t + 1)) % (2 * N) + 2 * N) % (2 * N);
          acc += I[jp + k - 1] * exN[q];
        }
        return acc / (LD)N;
      };
      pole_s.resize(k);
      for (int t = 0; t < k; ++t) pole_s[t] = (double)(Hs(t) - Hs(N - 1 - t)).real();
    }
  }

  std::vector<cLD> hph(2 * k - 1);
  for (int j = -(k - 1); j <= k - 1; ++j) {
    const LD ang = -PI_L * (LD)j / (LD)n;
    hph[j + k - 1] = cLD(cosl(ang), sinl(ang));
  }

  if ((e = upload(&T->xt, xt)) != hipSuccess) return e;
  if ((e = upload(&T->st, st)) != hipSuccess) return e;
  if ((e = upload(&T->ut, ut)) != hipSuccess) return e;
  if ((e = upload(&T->sx, sx)) != hipSuccess) return e;
  if ((e = upload(&T->hphase, to_d2(hph))) != hipSuccess) return e;
  if ((e = upload(&T->pole, pole)) != hipSuccess) return e;

  if (k == 2048 || k == 1024 || k == 512 || k == 256 || k == 128 || k == 64) {
    const int N = 2 * k, kh = k / 2;
    std::vector<double> us(kh), ss(kh), xs(kh, 1.0);
    for (int t = 0; t < kh; ++t) {
      const LD ps = PI_L * (LD)(2 * t + 1) / (LD)N;
      const LD h = sinl(0.5L * ps);
      us[t] = (double)(-2.0L * h * h);
      ss[t] = (double)sinl(ps);
    }
    std::vector<cLD> pph(2 * k - 1), rph(2 * k - 1);
    for (int j = -(k - 1); j <= k - 1; ++j) {
      const LD a = -PI_L * (LD)j / (LD)N;
      pph[j + k - 1] = cLD(cosl(a), sinl(a)) * ((LD)n / (LD)N);
      const LD b = a + PI_L * (LD)j / (LD)n;
      rph[j + k - 1] = cLD(cosl(b), sinl(b)) / (LD)(2 * N);
    }
    if ((e = upload(&T->ut_s, us)) != hipSuccess) return e;
    if ((e = upload(&T->st_s, ss)) != hipSuccess) return e;
    if ((e = upload(&T->sx_s, xs)) != hipSuccess) return e;
    if ((e = upload(&T->psph, to_d2(pph))) != hipSuccess) return e;
    if ((e = upload(&T->rsph, to_d2(rph))) != hipSuccess) return e;
    if ((e = upload(&T->pole_s, pole_s)) != hipSuccess) return e;
    T->sym = 1;
  }
  return hipSuccess;
}

void free_sht_tables(ShtTables* T) {
  hipFree(T->twn_lo);
  hipFree(T->twn_hi);
  hipFree(T->chirp);
  hipFree(T->bhat);
  hipFree(T->khat0);
  hipFree(T->khat1);
  hipFree(T->khr);
  hipFree(T->tw_lo);
  hipFree(T->tw_hi);
  hipFree(T->xt);
  hipFree(T->st);
  hipFree(T->ut);
  hipFree(T->sx);
  hipFree(T->hphase);
  hipFree(T->pole);
  hipFree(T->ut_s);
  hipFree(T->st_s);
  hipFree(T->sx_s);
  hipFree(T->psph);
  hipFree(T->pole_s);
  hipFree(T->rsph);
  *T = ShtTables();
}

// Recursion factors.  The normalised recursion (Condon-Shortley, orthonormal)
//   lambda_l = a_l (x lambda_{l-1} - b_l lambda_{l-2}),
//   a_l = sqrt((4l^2-1)/(l^2-m^2)),  b_l = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)),
//   lambda_{m+1} = sqrt(2m+3) x lambda_m,
// is rewritten as z_l = alpha_l x z_{l-1} - z_{l-2} with lambda_l = d_l z_l:
//   d_m = d_{m+1} = 1,  d_l = a_l b_l d_{l-2},  alpha_l = a_l d_{l-1} / d_l,
//   alpha_{m+1} = sqrt(2m+3)  (z_{m-1} = 0).
void leg_factors_host(int Lt, std::vector<double>* alpha, std::vector<double>* beta,
                      std::vector<double>* dfac, std::vector<double>* cm) {
  const size_t rows = (size_t)tri_rows(Lt);
  alpha->assign(rows, 0.0);
  beta->assign(rows, -2.0);
  dfac->assign(rows, 0.0);
  cm->assign(Lt, 0.0);
  for (int m = 0; m < Lt; ++m) {
    const size_t off = (size_t)tri_off(Lt, m);
    std::vector<LD> d(Lt - m + 1, 0.0L);
    d[0] = 1.0L;
    (*alpha)[off] = 0.0;
    (*dfac)[off] = 1.0;
    if (m + 1 < Lt) {
      d[1] = 1.0L;
      (*alpha)[off + 1] = (double)sqrtl((LD)(2 * m + 3));
      (*beta)[off + 1] = (double)(sqrtl((LD)(2 * m + 3)) - 2.0L);
      (*dfac)[off + 1] = 1.0;
    }
    for (int l = m + 2; l < Lt; ++l) {
      const LD ll = l, mm = m;
      const LD a = sqrtl((4.0L * ll * ll - 1.0L) / (ll * ll - mm * mm));
      const LD bb = sqrtl(((ll - 1.0L) * (ll - 1.0L) - mm * mm) / (4.0L * (ll - 1.0L) * (ll - 1.0L) - 1.0L));
      d[l - m] = a * bb * d[l - m - 2];
      const LD al = a * d[l - m - 1] / d[l - m];
      (*alpha)[off + l - m] = (double)al;
      (*beta)[off + l - m] = (double)(al - 2.0L);
      (*dfac)[off + l - m] = (double)d[l - m];
    }
  }
  // lambda_mm = (-1)^m sqrt((2m+1)/(4 pi) prod_{i=1}^m (2i-1)/(2i)) sin^m(theta)
  LD prod = 1.0L;
  for (int m = 0; m < Lt; ++m) {
    if (m > 0) prod *= (LD)(2 * m - 1) / (LD)(2 * m);
    const LD v = sqrtl((LD)(2 * m + 1) / (4.0L * PI_L) * prod);
    (*cm)[m] = (double)((m & 1) ? -v : v);
  }
}

hipError_t build_leg_tables(int Lt, LegTables* G) {
  std::vector<double> alpha, beta, dfac, cm;
  leg_factors_host(Lt, &alpha, &beta, &dfac, &cm);
  G->Lt = Lt;
  hipError_t e;
  if ((e = upload(&G->alpha, alpha)) != hipSuccess) return e;
  if ((e = upload(&G->beta, beta)) != hipSuccess) return e;
  if ((e = upload(&G->dfac, dfac)) != hipSuccess) return e;
  if ((e = upload(&G->cm, cm)) != hipSuccess) return e;
  return hipSuccess;
}

void free_leg_tables(LegTables* G) {
  hipFree(G->alpha);
  hipFree(G->beta);
  hipFree(G->dfac);
  hipFree(G->cm);
  *G = LegTables();
}

// ------------------------------------------------------------------------------------------
// Scale-discretised generating functions, Eqs. (10)-(14), by composite Gauss-Legendre
// quadrature (nodes from Newton iteration on P_n in long double).
// ------------------------------------------------------------------------------------------
namespace {
struct GaussRule {
  std::vector<LD> x, w;
  explicit GaussRule(int n) : x(n), w(n) {
    for (int i = 0; i < n; ++i) {
      LD z = cosl(PI_L * ((LD)i + 0.75L) / ((LD)n + 0.5L));
      for (int it = 0; it < 100; ++it) {
        LD p0 = 1.0L, p1 = z;
        for (int j = 2; j <= n; ++j) {
          const LD p2 = ((2.0L * j - 1.0L) * z * p1 - (j - 1.0L) * p0) / (LD)j;
          p0 = p1;
          p1 = p2;
        }
        const LD dp = (LD)n * (z * p1 - p0) / (z * z - 1.0L);
        const LD dz = p1 / dp;
        z -= dz;
        if (fabsl(dz) < 1e-19L) {
          // weight from the final derivative
          LD q0 = 1.0L, q1 = z;
          for (int j = 2; j <= n; ++j) {
            const LD q2 = ((2.0L * j - 1.0L) * z * q1 - (j - 1.0L) * q0) / (LD)j;
            q0 = q1;
            q1 = q2;
          }
          const LD dq = (LD)n * (z * q1 - q0) / (z * z - 1.0L);
          x[i] = z;
          w[i] = 2.0L / ((1.0L - z * z) * dq * dq);
          break;
        }
      }
    }
  }
};

LD schwartz_sq_over_u(LD u, LD lam) {
  const LD xx = 2.0L * lam * (u - 1.0L / lam) / (lam - 1.0L) - 1.0L;
  if (xx <= -1.0L || xx >= 1.0L) return 0.0L;
  const LD s = expl(-1.0L / (1.0L - xx * xx));
  return s * s / u;
}

// int_a^b s_lambda^2(u)/u du with `panels` panels of a 20-point rule
LD integrate(LD a, LD b, LD lam, int panels) {
  static const GaussRule rule(20);
  if (b <= a) return 0.0L;
  LD sum = 0.0L;
  const LD h = (b - a) / (LD)panels;
  for (int p = 0; p < panels; ++p) {
    const LD lo = a + h * (LD)p;
    const LD mid = lo + 0.5L * h;
    LD part = 0.0L;
    for (size_t i = 0; i < rule.x.size(); ++i) part += rule.w[i] * schwartz_sq_over_u(mid + 0.5L * h * rule.x[i], lam);
    sum += 0.5L * h * part;
  }
  return sum;
}
}  // namespace

// k_lambda(t) of Eq. (12): 1 for t <= 1/lambda, 0 for t >= 1.
double k_lambda_host(double t, double lam) {
  const LD L = lam;
  if (t <= 1.0 / lam) return 1.0;
  if (t >= 1.0) return 0.0;
  const int panels = 128;
  const LD den = integrate(1.0L / L, 1.0L, L, panels);
  const LD num = integrate((LD)t, 1.0L, L, panels);
  return (double)(num / den);
}

// B-spline generating function (footnote to Sect. 2.2): k(t) = (3/2) B_3(2 t lambda^(J-1) / L) with
// the cubic B-spline B_3(x) = (|x-2|^3 - 4|x-1|^3 + 6|x|^3 - 4|x+1|^3 + |x+2|^3) / 12.  eta(l) =
// sqrt k(l / lambda^J_min), kappa_j(l) = sqrt(k(l / lambda^(j+1)) - k(l / lambda^j)) for j < J and,
// so that the tiling sums to one below L, kappa_J(l) = sqrt(1 - k(l / lambda^J)).
static void tiling_bspline(int L, int B, int J_min, int J, double* kappa, double* eta) {
  const LD lam = (LD)B;
  // Cubic B-spline of Eq. (18) in its piecewise-polynomial form (the five-term sum of cubes is
  // the same function but cancels badly near the end of the support, where kappa_j is small).
  auto b3 = [](LD x) {
    x = x < 0 ? -x : x;
    if (x >= 2.0L) return 0.0L;
    if (x >= 1.0L) {
      const LD r = 2.0L - x;
      return r * r * r / 6.0L;
    }
    return 2.0L / 3.0L - x * x + x * x * x / 2.0L;
  };
  LD pJ1 = 1.0L;
  for (int i = 0; i < J - 1; ++i) pJ1 *= lam;
  auto k = [&](LD t) {
    const LD x = 2.0L * t * pJ1 / (LD)L;
    return x >= 2.0L ? 0.0L : 1.5L * b3(x);
  };
  std::vector<LD> pw(J + 2);
  pw[0] = 1.0L;
  for (int j = 1; j < J + 2; ++j) pw[j] = pw[j - 1] * lam;
  for (int l = 0; l < L; ++l) {
    eta[l] = (double)sqrtl(std::max(0.0L, k((LD)l / pw[J_min])));
    for (int j = J_min; j <= J; ++j) {
      const LD k2 = j < J ? k((LD)l / pw[j + 1]) - k((LD)l / pw[j]) : 1.0L - k((LD)l / pw[J]);
      kappa[(size_t)(j - J_min) * L + l] = (double)sqrtl(std::max(0.0L, k2));
    }
  }
}

void tiling_host_kernel(int L, int B, int J_min, int J, int kernel, double* kappa, double* eta) {
  if (kernel == S2LET_KERNEL_BSPLINE)
    tiling_bspline(L, B, J_min, J, kappa, eta);
  else
    tiling_host(L, B, J_min, J, kappa, eta);
}

void tiling_host(int L, int B, int J_min, int J, double* kappa, double* eta) {
  const LD lam = (LD)B;
  const int panels = 128;
  const LD den = integrate(1.0L / lam, 1.0L, lam, panels);
  std::map<LD, double> memo;
  auto kfun = [&](LD t) -> double {
    if (t <= 1.0L / lam) return 1.0;
    if (t >= 1.0L) return 0.0;
    auto it = memo.find(t);
    if (it != memo.end()) return it->second;
    const double v = (double)(integrate(t, 1.0L, lam, panels) / den);
    memo.emplace(t, v);
    return v;
  };
  std::vector<LD> pw(J + 2);
  pw[0] = 1.0L;
  for (int j = 1; j < J + 2; ++j) pw[j] = pw[j - 1] * lam;
  // kappa^2 = k(t/lambda) - k(t) is one integral of the same integrand over
  // [max(t/lambda, 1/lambda), min(t, 1)]: evaluated as such, without cancellation.
  auto kappa2 = [&](LD t) -> LD {
    const LD lo = std::max(t / lam, 1.0L / lam), hi = std::min(t, 1.0L);
    if (hi <= lo) return 0.0L;
    return integrate(lo, hi, lam, panels) / den;
  };
  for (int l = 0; l < L; ++l) {
    eta[l] = std::sqrt(std::fmax(0.0, kfun((LD)l / pw[J_min])));
    for (int j = J_min; j <= J; ++j)
      kappa[(size_t)(j - J_min) * L + l] = (double)sqrtl(std::max(0.0L, kappa2((LD)l / pw[j])));
  }
}

}  // namespace s2let
