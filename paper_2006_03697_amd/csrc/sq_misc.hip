// sq_misc.hip -- width-independent gfx950 kernels of the infinite-cell
// Clenshaw-Curtis SQ hot path (arXiv 2006.03697, Sec. IV and App. A):
// spectral bounds from the Lanczos tridiagonals, the Fermi level, the
// Clenshaw-Curtis coefficients, density and band energy per node, the
// reductions and the local potential; and the dispatch of the recurrence
// kernels over cube widths.
#include <mutex>

#include "sq.h"
#include "sq_devfn.h"

namespace {
// Number of eigenvalues of the tridiagonal (a, b) below x (Sturm count).
__device__ int sturm_count(const double* a, const double* b, int n, double x) {
  int c = 0;
  double d = a[0] - x;
  if (d < 0) ++c;
  for (int i = 1; i < n; ++i) {
    if (d == 0.0) d = -1e-300;
    d = a[i] - x - b[i - 1] * b[i - 1] / d;
    if (d < 0) ++c;
  }
  return c;
}

// Square of the last component of the unit eigenvector of eigenvalue x:
// p_{n-1}(x) / p_n'(x) with p_k the characteristic polynomials of the
// leading k x k blocks (three-term recurrence, rescaled against overflow).
__device__ double last_component_sq(const double* a, const double* b, int n, double x) {
  double pm2 = 1.0, pm1 = x - a[0];
  double dm2 = 0.0, dm1 = 1.0;
  for (int k = 1; k < n; ++k) {
    const double bb = b[k - 1] * b[k - 1];
    const double p = (x - a[k]) * pm1 - bb * pm2;
    const double d = pm1 + (x - a[k]) * dm1 - bb * dm2;
    pm2 = pm1;
    pm1 = p;
    dm2 = dm1;
    dm1 = d;
    const double mx = fmax(fabs(pm1), fabs(dm1));
    if (mx > 1e150) {
      pm1 *= 1e-150;
      pm2 *= 1e-150;
      dm1 *= 1e-150;
      dm2 *= 1e-150;
    }
  }
  // p_{n-1} = pm2, p_n' = dm1
  return pm2 / dm1;
}

__global__ void k_bounds(PlanDev P, const long long* items, const int* item_cell, long long nitems) {
  const long long it = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (it >= nitems) return;
  const long long g = items[it];
  const double* lan = P.lan + g * (2 * SQ_KL_MAX);
  // the first K steps (a longer run for the moments repeats them exactly)
  const int n = min(P.lan_steps[g], P.cells[item_cell[it]].K);
  const double* a = lan;
  const double* b = lan + SQ_KL_MAX;
  double lo, hi;
  if (n <= 1) {
    lo = a[0] - b[0];
    hi = a[0] + b[0];
  } else {
    // Gershgorin interval
    double glo = a[0] - fabs(b[0]), ghi = a[0] + fabs(b[0]);
    for (int i = 1; i < n; ++i) {
      const double r = fabs(b[i - 1]) + (i < n - 1 ? fabs(b[i]) : 0.0);
      glo = fmin(glo, a[i] - r);
      ghi = fmax(ghi, a[i] + r);
    }
    const double pad = 1e-12 * fmax(fabs(glo), fabs(ghi)) + 1e-300;
    glo -= pad;
    ghi += pad;
    // smallest eigenvalue: count(x) goes 0 -> 1
    double l = glo, u = ghi;
    for (int i = 0; i < 200; ++i) {
      const double mid = 0.5 * (l + u);
      if (mid <= l || mid >= u) break;
      if (sturm_count(a, b, n, mid) >= 1) u = mid; else l = mid;
    }
    const double tmin = 0.5 * (l + u);
    // largest eigenvalue: count(x) goes n-1 -> n
    l = glo;
    u = ghi;
    for (int i = 0; i < 200; ++i) {
      const double mid = 0.5 * (l + u);
      if (mid <= l || mid >= u) break;
      if (sturm_count(a, b, n, mid) >= n) u = mid; else l = mid;
    }
    const double tmax = 0.5 * (l + u);
    const double smin = sqrt(fabs(last_component_sq(a, b, n, tmin)));
    const double smax = sqrt(fabs(last_component_sq(a, b, n, tmax)));
    lo = tmin - b[n - 1] * smin;
    hi = tmax + b[n - 1] * smax;
  }
  if (P.inject & SQ_INJECT_NARROW) {   // error-path tests: half the interval
    const double c = 0.5 * (hi + lo), r = 0.25 * (hi - lo);
    lo = c - r;
    hi = c + r;
  }
  double* bd = P.bnd + 4 * g;
  bd[0] = lo;
  bd[1] = hi;
  bd[2] = 0.5 * (hi + lo);
  bd[3] = 0.5 * (hi - lo);
}

// ---------------------------------------------------------------------------
// Clenshaw-Curtis coefficients and the Fermi level (Sec. IV, App. A)
//
// c_j = (2/M) sum_k g(cos th_k) cos(j th_k), th_k = pi (k + 1/2) / M.  Off a
// window of +-40 kT around mu the FP64 occupation is exactly 0 or 1, so the
// sum splits into a closed-form tail  sum_{k >= a} cos(j th_k) =
//   sin((M - a) j pi / 2M) cos((a + M) j pi / 2M) / sin(j pi / 2M)
// and the window points.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double tail_cos_sum(int j, int a, int M) {
  if (a >= M) return 0.0;
  if (j == 0) return (double)(M - a);
  const double tm = 2.0 * (double)M;
  return sinpi((double)(M - a) * j / tm) * cospi((double)(a + M) * j / tm) / sinpi((double)j / tm);
}

struct Window {
  int M, kb, ka;
  double muh, sigh;
};

__device__ __forceinline__ Window fermi_window(double mu, double chi, double zeta, const CellDev& C) {
  Window W;
  const double kT = C.kT;
  W.M = C.mq > 0 ? C.mq : quad_points(zeta, kT, C.npl);
  W.muh = (mu - chi) / zeta;
  W.sigh = kT / zeta;
  const double xb = W.muh + 40.0 * W.sigh;   // above: occupation 0
  const double xa = W.muh - 40.0 * W.sigh;   // below: occupation 1
  const double M = (double)W.M;
  // x_k <= xb  <=>  k >= M acos(xb)/pi - 1/2
  int kb = xb >= 1.0 ? 0 : (xb <= -1.0 ? W.M : (int)floor(M * acos(xb) / M_PI - 0.5) - 1);
  int ka = xa <= -1.0 ? W.M - 1 : (xa >= 1.0 ? -1 : (int)ceil(M * acos(xa) / M_PI - 0.5) + 1);
  W.kb = kb < 0 ? 0 : (kb > W.M ? W.M : kb);
  W.ka = ka > W.M - 1 ? W.M - 1 : (ka < -1 ? -1 : ka);
  return W;
}

__device__ __forceinline__ double occupation(double x, const Window& W) {
  return 0.5 * (1.0 - tanh((x - W.muh) / (2.0 * W.sigh)));
}

// One wave per node: N_q(mu) = sum'_j c_q^j(mu) rho_q^j.
__global__ void __launch_bounds__(256) k_mu_eval(PlanDev P, const long long* items,
                                                 const int* item_cell, long long nitems) {
  __shared__ double smom[4][260];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long it = blockIdx.x * 4ll + wv;
  if (it >= nitems) return;   // whole wave leaves; only wave-level syncs below
  const long long g = items[it];
  const int ci = item_cell[it];
  const double* mus = P.mus + SQ_MU_STRIDE * ci;
  if (mus[MU_DONE] != 0.0) return;
  const CellDev& C = P.cells[ci];
  const int npl = C.npl;
  const double* mom = P.mom + g * P.mstride;
  for (int j = lane; j <= npl; j += 64) smom[wv][j] = mom[j];
  wave_sync();
  const double chi = P.bnd[4 * g + 2], zeta = P.bnd[4 * g + 3];
  const Window W = fermi_window(mus[MU_MID], chi, zeta, C);
  double acc = 0.0, dacc = 0.0;
  // occupied tail: sum'_j rho^j S_j(ka + 1)
  for (int j = lane; j <= npl; j += 64) {
    const double r = j == 0 ? 0.5 * smom[wv][0] : smom[wv][j];
    acc += r * tail_cos_sum(j, W.ka + 1, W.M);
  }
  // window points: g_k * sum'_j rho^j T_j(x_k) (Clenshaw); the derivative
  // in mu uses dg/dmu = g (1 - g) / kT, zero on the tails
  for (int k = W.kb + lane; k <= W.ka; k += 64) {
    const double x = cospi(((double)k + 0.5) / (double)W.M);
    const double occ = occupation(x, W);
    double b1 = 0.0, b2 = 0.0;
    for (int j = npl; j >= 1; --j) {
      const double b0 = smom[wv][j] + 2.0 * x * b1 - b2;
      b2 = b1;
      b1 = b0;
    }
    const double R = 0.5 * smom[wv][0] + x * b1 - b2;
    acc += occ * R;
    dacc += occ * (1.0 - occ) * R;
  }
  acc = warp_sum(acc);
  dacc = warp_sum(dacc);
  if (lane == 0) {
    P.nq[g] = (2.0 / (double)W.M) * acc;
    P.nqd[g] = (2.0 / (double)W.M) * dacc / C.kT;
  }
}

// LDA exchange-correlation of the unpolarised uniform electron gas at
// density r > 0: Slater exchange e_x = -(3/4)(3r/pi)^(1/3), v_x = 4 e_x / 3;
// Perdew-Wang 1992 correlation with r_s = (3 / (4 pi r))^(1/3),
// e_c = -2A(1 + a1 r_s) ln(1 + 1/(2A(b1 r_s^1/2 + b2 r_s + b3 r_s^3/2 + b4 r_s^2))),
// v_c = e_c - (r_s/3) de_c/dr_s.  Returns e_xc and v_xc.
__device__ void lda_xc(double r, double& exc, double& vxc) {
  const double ex = -0.75 * cbrt(3.0 * r / M_PI);
  const double A = 0.031091, a1 = 0.21370, b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294;
  const double rs = cbrt(3.0 / (4.0 * M_PI * r));
  const double srs = sqrt(rs);
  const double q0 = -2.0 * A * (1.0 + a1 * rs);
  const double q1 = 2.0 * A * srs * (b1 + srs * (b2 + srs * (b3 + b4 * srs)));
  const double q1p = A * (b1 / srs + 2.0 * b2 + 3.0 * b3 * srs + 4.0 * b4 * rs);
  const double lg = log1p(1.0 / q1);
  const double ec = q0 * lg;
  const double dec = -2.0 * A * a1 * lg - q0 * q1p / (q1 * (q1 + 1.0));
  exc = ex + ec;
  vxc = 4.0 / 3.0 * ex + ec - rs / 3.0 * dec;
}

// One wave per node: c_j, d_j at the final mu, rho_q and e_q.
__global__ void __launch_bounds__(256) k_coeffs(PlanDev P, const long long* items,
                                                const int* item_cell, long long nitems) {
  __shared__ double sg[4][256];
  __shared__ double sc[4][264];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long it = blockIdx.x * 4ll + wv;
  const bool live = it < nitems;
  const long long g = live ? items[it] : 0;
  const int ci = live ? item_cell[it] : 0;
  const CellDev& C = P.cells[ci];
  const int npl = C.npl;
  const double chi = P.bnd[4 * g + 2], zeta = P.bnd[4 * g + 3];
  const double mu = P.mus[SQ_MU_STRIDE * ci + MU_VAL];
  const Window W = fermi_window(mu, chi, zeta, C);
  const double* mom = P.mom + g * P.mstride;
  // per lane: coefficients j = lane + 64 r
  double cacc[5] = {0, 0, 0, 0, 0};
  for (int r = 0; r < 5; ++r) {
    const int j = lane + 64 * r;
    if (j <= npl + 1) cacc[r] = tail_cos_sum(j, W.ka + 1, W.M);
  }
  for (int base = W.kb; base <= W.ka; base += 256) {
    // occupations of 256 window points into LDS
    for (int t = lane; t < 256; t += 64) {
      const int k = base + t;
      double o = 0.0;
      if (k <= W.ka) o = occupation(cospi(((double)k + 0.5) / (double)W.M), W);
      sg[wv][t] = o;
    }
    wave_sync();
    const int kend = min(base + 256, W.ka + 1);
    for (int r = 0; r < 5; ++r) {
      const int j = lane + 64 * r;
      if (j > npl + 1) break;
      // cos(j theta_k), theta_k = (k + 1/2) pi / M: exact at every 4th point,
      // rotated by j pi / M in between (three rotations keep it within a few
      // ulp; sixteen left a bias of 1e-11 in the band energy of a 64000-node
      // cell)
      double sd, cd;
      sincospi((double)j / (double)W.M, &sd, &cd);
      double a = 0.0;
      for (int k0 = base; k0 < kend; k0 += 4) {
        double sn, cs;
        sincospi((double)j * ((double)k0 + 0.5) / (double)W.M, &sn, &cs);
        const int k1 = min(k0 + 4, kend);
        for (int k = k0; k < k1; ++k) {
          a += sg[wv][k - base] * cs;
          const double cn = cs * cd - sn * sd;
          sn = sn * cd + cs * sd;
          cs = cn;
        }
      }
      cacc[r] += a;
    }
    wave_sync();
  }
  const double f = 2.0 / (double)W.M;
  for (int r = 0; r < 5; ++r) {
    const int j = lane + 64 * r;
    if (j <= npl + 1) sc[wv][j] = f * cacc[r];
  }
  wave_sync();
  if (!live) return;
  double rs = 0.0, es = 0.0;
  for (int j = lane; j <= npl; j += 64) {
    const double cj = sc[wv][j];
    const double dj = 0.5 * (sc[wv][j + 1] + sc[wv][j == 0 ? 1 : j - 1]);
    const double wgt = j == 0 ? 0.5 : 1.0;
    rs += wgt * cj * mom[j];
    es += wgt * (chi * cj + zeta * dj) * mom[j];
    P.coef[g * P.mstride + j] = cj;
  }
  rs = warp_sum(rs);
  es = warp_sum(es);
  // rho, band-energy density, local-potential energy dV V_q rho_q, the LDA
  // exchange-correlation terms; the stress columns (K, N, nonlocal energy)
  // start at zero until the stress pass
  double* rec = P.rec + g * SQ_REC;
  if (lane == 0) {
    const double rho = 2.0 / C.dV * rs;
    rec[0] = rho;
    rec[1] = 2.0 * es;
    rec[21] = 2.0 * C.vloc[g - C.node_base] * rs;
    // LDA exchange-correlation energy and isotropic stress densities
    double exc = 0.0, vxc = 0.0;
    if (rho > 0.0) lda_xc(rho, exc, vxc);
    rec[22] = C.dV * rho * exc;
    rec[23] = C.dV * rho * (exc - vxc);
  }
  if (lane >= 2 && lane <= 20) rec[lane] = 0.0;
}

// Neumaier-compensated fixed-order sum of x[i * stride] over [0, n).
__device__ void block_neumaier(const double* x, long long n, long long stride, double* out,
                               double* red_s, double* red_c) {
  double s = 0.0, c = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = x[i * stride];
    const double t = s + v;
    c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
    s = t;
  }
  red_s[threadIdx.x] = s;
  red_c[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    double S = 0.0, Cc = 0.0;
    for (int i = 0; i < (int)blockDim.x; ++i) {
      const double v = red_s[i];
      const double t = S + v;
      Cc += fabs(S) >= fabs(v) ? (S - t) + v : (v - t) + S;
      S = t;
      Cc += red_c[i];
    }
    *out = S + Cc;
  }
  __syncthreads();
}

// Fermi-level bracket: [min lam_lo - 40 kT, max lam_hi + 40 kT].
__global__ void __launch_bounds__(256) k_mu_init(PlanDev P, const int* cells, const int* fixed_mode) {
  __shared__ double slo[256], shi[256];
  const int ci = cells[blockIdx.x];
  const CellDev& C = P.cells[ci];
  double lo = 1e300, hi = -1e300;
  for (long long q = threadIdx.x; q < C.Nd; q += blockDim.x) {
    const double* b = P.bnd + 4 * (C.node_base + q);
    lo = fmin(lo, b[0]);
    hi = fmax(hi, b[1]);
  }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 256; ++i) {
      lo = fmin(lo, slo[i]);
      hi = fmax(hi, shi[i]);
    }
    double* m = P.mus + SQ_MU_STRIDE * ci;
    m[MU_LO] = lo - 40.0 * C.kT;
    m[MU_HI] = hi + 40.0 * C.kT;
    m[MU_IT] = 0.0;
    m[MU_N] = 0.0;
    if (fixed_mode[blockIdx.x]) {
      m[MU_DONE] = 1.0;
      m[MU_PHASE] = 3.0;
      m[MU_VAL] = C.mu0;
      m[MU_MID] = C.mu0;
    } else {
      m[MU_DONE] = 0.0;
      m[MU_PHASE] = 0.0;
      m[MU_MID] = m[MU_LO];
    }
  }
}

// Electron count of each cell at its trial mu and the update of the
// bracket.  The root of N(mu) = N_e is searched inside the bracket by a
// Newton step from the trial point when it lands inside, else by the
// Illinois variant of regula falsi (the retained end point's value is halved
// when the same end is kept twice), with a bisection step whenever four
// updates have not halved the bracket; it stops at |N - N_e| <= 1e-13 N_e,
// the criterion of the plain bisection, or after 200 updates.
__global__ void __launch_bounds__(256) k_mu_step(PlanDev P, const int* cells) {
  __shared__ double rs[256], rc[256];
  __shared__ double tot, dtot;
  const int ci = cells[blockIdx.x];
  const CellDev& C = P.cells[ci];
  double* m = P.mus + SQ_MU_STRIDE * ci;
  if (m[MU_DONE] != 0.0) return;
  block_neumaier(P.nq + C.node_base, C.Nd, 1, &tot, rs, rc);
  block_neumaier(P.nqd + C.node_base, C.Nd, 1, &dtot, rs, rc);
  if (threadIdx.x != 0) return;
  const double N = 2.0 * tot;
  const double dN = 2.0 * dtot;
  const double Ne = C.ne;
  m[MU_N] = N;
  const int phase = (int)m[MU_PHASE];
  if (phase == 0) {
    if (!(N < Ne)) { m[MU_DONE] = 2.0; return; }
    m[MU_FLO] = N - Ne;
    m[MU_PHASE] = 1.0;
    m[MU_MID] = m[MU_HI];
    return;
  }
  const double mid = m[MU_MID];
  double lo = m[MU_LO], hi = m[MU_HI];
  double flo = m[MU_FLO], fhi = m[MU_FHI];
  if (phase == 1) {
    if (!(Ne < N)) { m[MU_DONE] = 2.0; return; }
    fhi = N - Ne;
    m[MU_PHASE] = 2.0;
    m[MU_SIDE] = 0.0;
    m[MU_WID] = hi - lo;
  } else {
    const double f = N - Ne;
    if (fabs(f) <= 1e-13 * Ne) {
      m[MU_VAL] = mid;
      m[MU_DONE] = 1.0;
      return;
    }
    const double side = m[MU_SIDE];
    if (f > 0.0) {
      hi = mid;
      fhi = f;
      if (side > 0.0) flo *= 0.5;
      m[MU_SIDE] = 1.0;
    } else {
      lo = mid;
      flo = f;
      if (side < 0.0) fhi *= 0.5;
      m[MU_SIDE] = -1.0;
    }
    m[MU_IT] += 1.0;
    // a bracket collapsed to rounding level is a root to machine precision;
    // the update cap without that is a search that did not converge
    const bool collapsed = !(hi - lo > 4.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)));
    const double cap = (P.inject & SQ_INJECT_MU_CAP) ? 2.0 : 200.0;
    if (collapsed || m[MU_IT] >= cap) {
      m[MU_VAL] = mid;
      m[MU_DONE] = collapsed ? 1.0 : 3.0;
      m[MU_LO] = lo;
      m[MU_HI] = hi;
      return;
    }
  }
  // next trial point: Newton from the trial point, else regula falsi, or
  // bisection if progress stalls
  double x = (lo * fhi - hi * flo) / (fhi - flo);
  const int it = (int)m[MU_IT];
  bool newton = false;
  if (phase == 2 && dN > 0.0) {
    const double xn = mid - (N - Ne) / dN;
    if (xn > lo && xn < hi) {
      x = xn;
      newton = true;
    }
  }
  if (!newton && it > 0 && it % 4 == 0) {
    if (hi - lo > 0.5 * m[MU_WID]) x = 0.5 * (lo + hi);
    m[MU_WID] = hi - lo;
  }
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
  m[MU_LO] = lo;
  m[MU_HI] = hi;
  m[MU_FLO] = flo;
  m[MU_FHI] = fhi;
  m[MU_MID] = x;
}

__global__ void __launch_bounds__(256) k_reduce(PlanDev P, const int* cells, int col0, int ncol) {
  __shared__ double rs[256], rc[256];
  const int ci = cells[blockIdx.x];
  const CellDev& C = P.cells[ci];
  for (int c = col0; c < col0 + ncol; ++c) {
    block_neumaier(P.rec + C.node_base * SQ_REC + c, C.Nd, SQ_REC, P.sums + ci * (SQ_REC + 4) + c,
                   rs, rc);
  }
}

// p[0 .. n) = v.  Clears counters and flags with an ordinary kernel (also
// inside a captured graph).
__global__ void __launch_bounds__(256) k_fill_u32(unsigned* p, unsigned v, long long n) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  if (i < n) p[i] = v;
}

// Local potential on the periodic grid: sum over atom images within v_rcut.
__global__ void __launch_bounds__(256) k_vloc(const CellDev* cell, double* out) {
  const CellDev& C = *cell;
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= C.Nd) return;
  const long long ix = i % C.n[0], iy = (i / C.n[0]) % C.n[1], iz = i / ((long long)C.n[0] * C.n[1]);
  double v = 0.0;
  for (int I = 0; I < C.nimg; ++I) {
    const double* R = C.img + 4 * I;
    const SpecDev& s = C.sp[(int)R[3]];
    const double dx = node_coord(ix, C.h, R[0]);
    const double dy = node_coord(iy, C.h, R[1]);
    const double dz = node_coord(iz, C.h, R[2]);
    const double r2 = sq_add(sq_sum2(dx, dy), dz);
    if (r2 < s.v_rc * s.v_rc) v += -s.v_amp * exp(-r2 / (2.0 * s.v_sig * s.v_sig));
  }
  out[i] = v;
}

}  // namespace


bool sq_nc_supported(int nc) {
#define SQ_CASE(N) if (nc == N) return true;
  SQ_NC_LIST(SQ_CASE)
#undef SQ_CASE
  return false;
}

int sq_kc_variant(bool fused, int kc) { return sq_kc_pick(fused, kc); }

int sq_img_limit(int nc) { return sq_img_max(nc); }

int sq_gram_limit(int nc) { return sq_gram_cap(nc); }

hipError_t sq_launch_lanczos(const RecLaunch& R, const PlanDev& P, const long long* items,
                             const int* item_cell, long long nitems, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
#define SQ_CASE(N) \
  if (R.nc == N) return sq_launch_lanczos_##N(R, P, items, item_cell, nitems, s);
  SQ_NC_LIST(SQ_CASE)
#undef SQ_CASE
  return hipErrorInvalidValue;
}

hipError_t sq_launch_gram(int nc, const PlanDev& P, const long long* items,
                          const int* item_cell, long long nitems, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
#define SQ_CASE(N) if (nc == N) return sq_launch_gram_##N(P, items, item_cell, nitems, s);
  SQ_NC_LIST(SQ_CASE)
#undef SQ_CASE
  return hipErrorInvalidValue;
}

hipError_t sq_launch_moments(const RecLaunch& R, bool fp64, const PlanDev& P,
                             const long long* items, const int* item_cell, long long nitems,
                             hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
#define SQ_CASE(N) \
  if (R.nc == N) return sq_launch_moments_##N(R, fp64, P, items, item_cell, nitems, s);
  SQ_NC_LIST(SQ_CASE)
#undef SQ_CASE
  return hipErrorInvalidValue;
}

hipError_t sq_launch_stress(const RecLaunch& R, bool fp64, const PlanDev& P,
                            const long long* items, const int* item_cell, long long nitems,
                            hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
#define SQ_CASE(N) \
  if (R.nc == N) return sq_launch_stress_##N(R, fp64, P, items, item_cell, nitems, s);
  SQ_NC_LIST(SQ_CASE)
#undef SQ_CASE
  return hipErrorInvalidValue;
}

hipError_t sq_launch_fill_u32(unsigned* p, unsigned v, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t sq_launch_census(int nc, const PlanDev& P, const long long* items, const int* item_cell,
                            long long nitems, int* stats, long long* pairs, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
#define SQ_CASE(N) \
  if (nc == N) return sq_launch_census_##N(P, items, item_cell, nitems, stats, pairs, s);
  SQ_NC_LIST(SQ_CASE)
#undef SQ_CASE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Chebyshev moments from the Lanczos tridiagonal.  k Lanczos steps from w_q
// give the tridiagonal T (diagonal alpha_1..alpha_k, couplings
// beta_1..beta_k) of H_q on the Krylov space of w_q; for every polynomial p
// of degree <= 2k, w_q^T p(H_q) w_q = e_1^T p(T') e_1 with T' the
// (k + 1) x (k + 1) extension of T (its last diagonal entry never enters at
// that degree).  So rho^j = w_q^T T_j(Hhat_q) w_q = e_1^T T_j(That') e_1,
// That' = (T' - chi_q) / zeta_q, for j <= npl <= 2k: the same moments as
// the three-term recurrence on the cube (Sec. IV), from the small
// recurrence t^{j+1} = 2 That' t^j - t^{j-1}, t^0 = e_1.  A Lanczos run that
// stopped early found an invariant subspace, where the identity holds at
// every degree.  One wave per node; lane i holds component i (k + 1 <= 64).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_qmoments(PlanDev P, const long long* items,
                                                   const int* item_cell, long long nitems) {
  const long long it = blockIdx.x * 4LL + (threadIdx.x >> 6);
  if (it >= nitems) return;   // the whole wave
  const int l = threadIdx.x & 63;
  const long long g = items[it];
  const int npl = P.cells[item_cell[it]].npl;
  const double chi = P.bnd[4 * g + 2], zeta = P.bnd[4 * g + 3];
  const int ns = P.lan_steps[g];
  const double* lan = P.lan + g * (2 * SQ_KL_MAX);
  // That': diagonal, coupling to the next and to the previous component
  // (zero past the steps taken; the extension's diagonal entry is zero)
  const double a = l < ns ? (lan[l] - chi) / zeta : 0.0;
  const double b = l < ns ? lan[SQ_KL_MAX + l] / zeta : 0.0;
  const double bp = __shfl_up(b, 1);
  const double bl = l > 0 ? bp : 0.0;
  auto apply = [&](double v) {
    const double vu = __shfl_up(v, 1), vd = __shfl_down(v, 1);
    return a * v + (bl * vu + b * vd);   // lane 0: bl = 0; lane 63: b = 0
  };
  double mj[2] = {0.0, 0.0};   // rho^j kept by lane j % 64 in slot j / 64
  double t0 = l == 0 ? 1.0 : 0.0;
  double t1 = apply(t0);
  if (l == 0) mj[0] = 1.0;
  {
    const double r = __shfl(t1, 0);
    if (l == 1) mj[0] = r;
  }
  for (int j = 2; j <= npl; ++j) {
    const double t2 = 2.0 * apply(t1) - t0;
    t0 = t1;
    t1 = t2;
    const double r = __shfl(t1, 0);
    if (l == (j & 63)) mj[j >> 6] = r;
  }
  double* mom = P.mom + g * P.mstride;
  bool bad = false;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = 64 * h + l;
    if (j <= npl) {
      mom[j] = mj[h];
      if (!(fabs(mj[h]) <= 1.0 + 1e-6)) bad = true;   // as the recurrence kernel (FP64)
    }
  }
  if (bad) atomicOr(P.err, SQ_ERR_BOUNDS);
}

hipError_t sq_launch_qmoments(const PlanDev& P, const long long* items, const int* item_cell,
                              long long nitems, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_qmoments, dim3((unsigned)((nitems + 3) / 4)), dim3(256), 0, s, P, items,
                     item_cell, nitems);
  return hipGetLastError();
}

hipError_t sq_launch_vloc(const CellDev* d_cell, const CellDev& h_cell, double* vloc, hipStream_t s) {
  const long long nb = (h_cell.Nd + 255) / 256;
  hipLaunchKernelGGL(k_vloc, dim3((unsigned)nb), dim3(256), 0, s, d_cell, vloc);
  return hipGetLastError();
}

hipError_t sq_launch_bounds(const PlanDev& P, const long long* items, const int* item_cell,
                            long long nitems, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bounds, dim3((unsigned)((nitems + 127) / 128)), dim3(128), 0, s, P, items,
                     item_cell, nitems);
  return hipGetLastError();
}

hipError_t sq_launch_mu_init(const PlanDev& P, const int* cells, int ncells, const int* fixed_mode,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_mu_init, dim3(ncells), dim3(256), 0, s, P, cells, fixed_mode);
  return hipGetLastError();
}

hipError_t sq_launch_mu_eval(const PlanDev& P, const long long* items, const int* item_cell,
                             long long nitems, hipStream_t s) {
  hipLaunchKernelGGL(k_mu_eval, dim3((unsigned)((nitems + 3) / 4)), dim3(256), 0, s, P, items,
                     item_cell, nitems);
  return hipGetLastError();
}

hipError_t sq_launch_mu_step(const PlanDev& P, const int* cells, int ncells, hipStream_t s) {
  hipLaunchKernelGGL(k_mu_step, dim3(ncells), dim3(256), 0, s, P, cells);
  return hipGetLastError();
}

hipError_t sq_launch_coeffs(const PlanDev& P, const long long* items, const int* item_cell,
                            long long nitems, hipStream_t s) {
  hipLaunchKernelGGL(k_coeffs, dim3((unsigned)((nitems + 3) / 4)), dim3(256), 0, s, P, items,
                     item_cell, nitems);
  return hipGetLastError();
}

hipError_t sq_launch_reduce(const PlanDev& P, const int* cells, int ncells, int col0, int ncol,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(ncells), dim3(256), 0, s, P, cells, col0, ncol);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Static scratch: per-cell sums of the stress reduction for sq_stress_static
// (SQ_STATIC_CELLS rows of SQ_REC + 4 doubles; each GPU the library runs on
// holds its own copy until the process ends).  Host code never passes the
// array's name to a kernel: that is a host-side stand-in, not the device
// address.  The address comes from hipGetSymbolAddress, once per device with
// that device current, and is kept per device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[SQ_STATIC_CELLS * (SQ_REC + 4)];

hipError_t sq_static_scratch(double** out) {
  static std::mutex mu;
  static double* ptr[SQ_STATIC_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= SQ_STATIC_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptr[dev] = static_cast<double*>(p);
  }
  *out = ptr[dev];
  return hipSuccess;
}
