/*
 * sq_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference for the infinite-cell Clenshaw-Curtis
 * Spectral Quadrature (SQ) evaluation of the electron density, band energy
 * and density-matrix (kinetic + nonlocal) stress of Sharma, Hamel,
 * Bethkenhagen, Pask and Suryanarayana, "Real-space formulation of the stress
 * tensor for O(N) density functional theory" (arXiv 2006.03697), Sec. IV.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this file's library.  It shares no code with the HIP path: every
 * quantity (grid, cube, projector values, FD weights are passed in from the
 * oracle's own Python driver) is recomputed here with plain loops, no
 * blocking, no fusion, no SIMD intrinsics.  Build flags:
 *     gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared
 * OpenMP is used only to run independent node columns side by side; the
 * arithmetic inside one node is a straight transcription of the equations.
 *
 * Conventions (the paper leaves them open; the readings are listed in the
 * design notes of the repository):
 *   - grid node i = ix + n0*(iy + n1*iz), position h*(ix,iy,iz);
 *   - the cube (region of influence, Sec. IV) of node q holds the nodes
 *     q + a, a in [-m, m]^3, at UNWRAPPED positions h*(q + a); the local
 *     potential there is the periodic V_loc at the wrapped node;
 *   - every atom image R_I + n L whose projector support meets the cube is
 *     a separate rank-one term (infinite-cell formulation, Sec. IV);
 *   - V_nl restricted to the cube is gamma dV chi chi^T (chi sampled at nodes);
 *   - FD terms whose index leaves the cube are dropped (restriction of H,
 *     of the gradient matrices and of the unit vector, Sec. IV).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Species record layout: v_amp, v_sigma, v_rcut, p_sigma, p_rcut, gamma, z */
#define SP_STRIDE 7

typedef struct {
  int n[3];           /* nodes per axis */
  double h;           /* mesh size (Bohr) */
  double L[3];        /* cell sides (Bohr) */
  int m;              /* cube half width in nodes, n_c = 2m+1 */
  int M;              /* FD half order (6 -> 12th order) */
  const double* c2;   /* [M+1] second-derivative weights, scaled by 1/h^2 later */
  const double* c1;   /* [M+1] first-derivative weights (c1[0] unused), by 1/h */
  const double* vloc; /* [N_d] local potential on the periodic grid */
  int nimg;           /* atom images considered */
  const double* img;  /* [nimg][3] image centres, unwrapped (Bohr) */
  const int* img_sp;  /* [nimg] species of each image */
  const double* sp;   /* [nspec][SP_STRIDE] */
} or_cell;

typedef struct {
  int nc, Nc;
  int q[3];
  double* V;      /* [Nc] local potential on the cube */
  int nprj;       /* projectors (atom images) with support in the cube */
  int* prj_img;   /* [nprj] image index */
  double* gdv;    /* [nprj] gamma * dV */
  int* ptr;       /* [nprj+1] CSR row pointers */
  int* pt;        /* cube point index of each entry */
  double* val;    /* chi value of each entry */
} or_cube;

static int wrapi(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

/* Cube-local index of offset (ax, ay, az), each in [-m, m]. */
static int cidx(int m, int ax, int ay, int az) {
  int nc = 2 * m + 1;
  return (ax + m) + nc * ((ay + m) + nc * (az + m));
}

/* Build the nodal Hamiltonian data of node q (Sec. IV: restriction of H to
 * the cuboid of side 2 R_cut centred at q). */
static void cube_build(const or_cell* c, long qnode, or_cube* cb) {
  int m = c->m, nc = 2 * m + 1, Nc = nc * nc * nc;
  int q0 = (int)(qnode % c->n[0]);
  int q1 = (int)((qnode / c->n[0]) % c->n[1]);
  int q2 = (int)(qnode / ((long)c->n[0] * c->n[1]));
  cb->nc = nc; cb->Nc = Nc;
  cb->q[0] = q0; cb->q[1] = q1; cb->q[2] = q2;
  cb->V = (double*)malloc(sizeof(double) * Nc);
  for (int az = -m; az <= m; ++az)
    for (int ay = -m; ay <= m; ++ay)
      for (int ax = -m; ax <= m; ++ax) {
        int ix = wrapi(q0 + ax, c->n[0]);
        int iy = wrapi(q1 + ay, c->n[1]);
        int iz = wrapi(q2 + az, c->n[2]);
        cb->V[cidx(m, ax, ay, az)] =
            c->vloc[ix + (long)c->n[0] * (iy + (long)c->n[1] * iz)];
      }
  /* projector columns: plain scan of every image against every cube point */
  int cap = 64, ecap = 4096, ne = 0, np = 0;
  cb->prj_img = (int*)malloc(sizeof(int) * cap);
  cb->gdv = (double*)malloc(sizeof(double) * cap);
  cb->ptr = (int*)malloc(sizeof(int) * (cap + 1));
  cb->pt = (int*)malloc(sizeof(int) * ecap);
  cb->val = (double*)malloc(sizeof(double) * ecap);
  cb->ptr[0] = 0;
  double dV = c->h * c->h * c->h;
  for (int I = 0; I < c->nimg; ++I) {
    const double* s = c->sp + SP_STRIDE * c->img_sp[I];
    double ps = s[3], rp = s[4], gam = s[5];
    const double* R = c->img + 3 * I;
    /* an image farther than r_p from the cube's box cannot reach a node */
    double bd2 = 0.0;
    for (int al = 0; al < 3; ++al) {
      int qa = al == 0 ? q0 : (al == 1 ? q1 : q2);
      double lo = (double)(qa - m) * c->h, hi = (double)(qa + m) * c->h;
      double e = R[al] < lo ? lo - R[al] : (R[al] > hi ? R[al] - hi : 0.0);
      bd2 += e * e;
    }
    if (bd2 >= rp * rp) continue;
    int start = ne;
    for (int az = -m; az <= m; ++az)
      for (int ay = -m; ay <= m; ++ay)
        for (int ax = -m; ax <= m; ++ax) {
          double dx = (double)(q0 + ax) * c->h - R[0];
          double dy = (double)(q1 + ay) * c->h - R[1];
          double dz = (double)(q2 + az) * c->h - R[2];
          double d2 = dx * dx + dy * dy + dz * dz;
          if (d2 < rp * rp) {
            if (ne == ecap) {
              ecap *= 2;
              cb->pt = (int*)realloc(cb->pt, sizeof(int) * ecap);
              cb->val = (double*)realloc(cb->val, sizeof(double) * ecap);
            }
            cb->pt[ne] = cidx(m, ax, ay, az);
            cb->val[ne] = exp(-d2 / (2.0 * ps * ps));
            ++ne;
          }
        }
    if (ne > start) {
      if (np == cap) {
        cap *= 2;
        cb->prj_img = (int*)realloc(cb->prj_img, sizeof(int) * cap);
        cb->gdv = (double*)realloc(cb->gdv, sizeof(double) * cap);
        cb->ptr = (int*)realloc(cb->ptr, sizeof(int) * (cap + 1));
      }
      cb->prj_img[np] = I;
      cb->gdv[np] = gam * dV;
      cb->ptr[np + 1] = ne;
      ++np;
    }
  }
  cb->nprj = np;
}

static void cube_free(or_cube* cb) {
  free(cb->V); free(cb->prj_img); free(cb->gdv); free(cb->ptr); free(cb->pt); free(cb->val);
}

/* y = H_q v: -1/2 times the 12th-order FD Laplacian (Sec. V: twelfth-order
 * accurate finite differences), plus the local potential, plus the nonlocal
 * projectors gamma dV chi (chi^T v).  Stencil terms leaving the cube are
 * dropped (restriction to the region of influence, Sec. IV). */
static void apply_H(const or_cell* c, const or_cube* cb, const double* v, double* y) {
  int m = c->m, nc = cb->nc, M = c->M;
  int stride[3] = {1, nc, nc * nc};
  double s = -0.5 / (c->h * c->h);
  for (int az = -m; az <= m; ++az)
    for (int ay = -m; ay <= m; ++ay)
      for (int ax = -m; ax <= m; ++ax) {
        int a = cidx(m, ax, ay, az);
        int co[3] = {ax, ay, az};
        double lap = 0.0;
        for (int al = 0; al < 3; ++al) {
          lap += c->c2[0] * v[a];
          for (int k = 1; k <= M; ++k) {
            if (co[al] + k <= m) lap += c->c2[k] * v[a + k * stride[al]];
            if (co[al] - k >= -m) lap += c->c2[k] * v[a - k * stride[al]];
          }
        }
        y[a] = s * lap + cb->V[a] * v[a];
      }
  for (int p = 0; p < cb->nprj; ++p) {
    double dot = 0.0;
    for (int e = cb->ptr[p]; e < cb->ptr[p + 1]; ++e) dot += cb->val[e] * v[cb->pt[e]];
    for (int e = cb->ptr[p]; e < cb->ptr[p + 1]; ++e) y[cb->pt[e]] += cb->gdv[p] * cb->val[e] * dot;
  }
}

/* Restricted FD gradient along axis al: (grad v)_a = (1/h) sum_k w_k
 * (v_{a+k e} - v_{a-k e}), terms outside the cube dropped. */
static void apply_grad(const or_cell* c, const or_cube* cb, int al, const double* v, double* g) {
  int m = c->m, nc = cb->nc, M = c->M;
  int stride[3] = {1, nc, nc * nc};
  for (int az = -m; az <= m; ++az)
    for (int ay = -m; ay <= m; ++ay)
      for (int ax = -m; ax <= m; ++ax) {
        int a = cidx(m, ax, ay, az);
        int co[3] = {ax, ay, az};
        double acc = 0.0;
        for (int k = 1; k <= M; ++k) {
          if (co[al] + k <= m) acc += c->c1[k] * v[a + k * stride[al]];
          if (co[al] - k >= -m) acc -= c->c1[k] * v[a - k * stride[al]];
        }
        g[a] = acc / c->h;
      }
}

static double dot(const double* a, const double* b, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* ---------------------------------------------------------------------------
 * Spectral bounds of H_q (Sec. IV: chi_q, zeta_q come from the extreme
 * eigenvalues of H_q).  K-step Lanczos from the unit vector w_q without
 * reorthogonalisation; stops early when beta_k < 1e-14 (|alpha_1| + beta_1).
 * Returns the number of steps taken; alpha[k], beta[k] for k < steps.
 * ------------------------------------------------------------------------- */
int or_node_lanczos(const or_cell* c, long qnode, int K, double* alpha, double* beta,
                    double* Hqq) {
  or_cube cb;
  cube_build(c, qnode, &cb);
  int Nc = cb.Nc;
  double* v = (double*)calloc(Nc, sizeof(double));
  double* vp = (double*)calloc(Nc, sizeof(double));
  double* w = (double*)calloc(Nc, sizeof(double));
  v[cidx(c->m, 0, 0, 0)] = 1.0;
  double bprev = 0.0, tol = 0.0;
  int steps = 0;
  for (int k = 0; k < K; ++k) {
    apply_H(c, &cb, v, w);
    for (int i = 0; i < Nc; ++i) w[i] -= bprev * vp[i];
    double a = dot(v, w, Nc);
    for (int i = 0; i < Nc; ++i) w[i] -= a * v[i];
    double b = sqrt(dot(w, w, Nc));
    alpha[k] = a;
    beta[k] = b;
    steps = k + 1;
    if (k == 0) {
      tol = 1e-14 * (fabs(a) + b);
      if (Hqq) *Hqq = a;
    }
    if (b < tol) break;
    for (int i = 0; i < Nc; ++i) { vp[i] = v[i]; v[i] = w[i] / b; }
    bprev = b;
  }
  free(v); free(vp); free(w);
  cube_free(&cb);
  return steps;
}

/* Chebyshev three-term recurrence on the scaled nodal Hamiltonian
 * Hhat = (H_q - chi I)/zeta (Sec. IV): t^0 = w_q, t^1 = Hhat w_q,
 * t^{j+1} = 2 Hhat t^j - t^{j-1}; moments rho^j = w_q^T t^j, j = 0..npl. */
void or_node_moments(const or_cell* c, long qnode, double chi, double zeta, int npl,
                     double* mom) {
  or_cube cb;
  cube_build(c, qnode, &cb);
  int Nc = cb.Nc, ctr = cidx(c->m, 0, 0, 0);
  double* t0 = (double*)calloc(Nc, sizeof(double));
  double* t1 = (double*)calloc(Nc, sizeof(double));
  double* t2 = (double*)calloc(Nc, sizeof(double));
  double* y = (double*)calloc(Nc, sizeof(double));
  t0[ctr] = 1.0;
  mom[0] = t0[ctr];
  if (npl >= 1) {
    apply_H(c, &cb, t0, y);
    for (int i = 0; i < Nc; ++i) t1[i] = (y[i] - chi * t0[i]) / zeta;
    mom[1] = t1[ctr];
  }
  for (int j = 1; j < npl; ++j) {
    apply_H(c, &cb, t1, y);
    for (int i = 0; i < Nc; ++i) t2[i] = 2.0 * (y[i] - chi * t1[i]) / zeta - t0[i];
    mom[j + 1] = t2[ctr];
    double* tmp = t0; t0 = t1; t1 = t2; t2 = tmp;
  }
  free(t0); free(t1); free(t2); free(y);
  cube_free(&cb);
}

/* DM column d_q = sum'_{j=0}^{npl} c_j t^j (primed: first term halved), then
 * the density-matrix stress functionals of Sec. IV at node q:
 *   K_ab(q) = 2 w_q^T grad_a grad_b d_q                     (kinetic)
 *   N_ab(q) = -2 sum_I gamma dV chi_I(x_q) [ delta_ab chi_I^T d_q
 *             + 2 sum_y chi_I(y) (y_b - R_Ib) (grad_a d_q)(y) ] (nonlocal)
 * The sum over I runs over the images whose projector is nonzero at x_q.
 * out[0..8] = K row-major (a,b), out[9..17] = N row-major (a,b);
 * out[18] = the E_nl density 2 sum_I gamma dV chi_I(x_q) chi_I^T d_q;
 * out[19] = w_q^T d_q.  If dcol != NULL the column is copied there. */
void or_node_stress(const or_cell* c, long qnode, double chi, double zeta, int npl,
                    const double* coef, double* out, double* dcol) {
  or_cube cb;
  cube_build(c, qnode, &cb);
  int Nc = cb.Nc, m = c->m, ctr = cidx(m, 0, 0, 0);
  double* t0 = (double*)calloc(Nc, sizeof(double));
  double* t1 = (double*)calloc(Nc, sizeof(double));
  double* t2 = (double*)calloc(Nc, sizeof(double));
  double* y = (double*)calloc(Nc, sizeof(double));
  double* d = (double*)calloc(Nc, sizeof(double));
  t0[ctr] = 1.0;
  for (int i = 0; i < Nc; ++i) d[i] = 0.5 * coef[0] * t0[i];
  if (npl >= 1) {
    apply_H(c, &cb, t0, y);
    for (int i = 0; i < Nc; ++i) t1[i] = (y[i] - chi * t0[i]) / zeta;
    for (int i = 0; i < Nc; ++i) d[i] += coef[1] * t1[i];
  }
  for (int j = 1; j < npl; ++j) {
    apply_H(c, &cb, t1, y);
    for (int i = 0; i < Nc; ++i) t2[i] = 2.0 * (y[i] - chi * t1[i]) / zeta - t0[i];
    for (int i = 0; i < Nc; ++i) d[i] += coef[j + 1] * t2[i];
    double* tmp = t0; t0 = t1; t1 = t2; t2 = tmp;
  }
  /* gradients of d along each axis */
  double* g[3];
  for (int al = 0; al < 3; ++al) {
    g[al] = (double*)calloc(Nc, sizeof(double));
    apply_grad(c, &cb, al, d, g[al]);
  }
  double* gg = (double*)calloc(Nc, sizeof(double));
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      /* (grad_a grad_b d)_q: gradient matrices applied right to left */
      apply_grad(c, &cb, a, g[b], gg);
      out[3 * a + b] = 2.0 * gg[ctr];
    }
  for (int k = 0; k < 9; ++k) out[9 + k] = 0.0;
  double enl = 0.0;
  for (int p = 0; p < cb.nprj; ++p) {
    /* chi_I at the node itself (the centre of the cube) */
    double chiq = 0.0;
    for (int e = cb.ptr[p]; e < cb.ptr[p + 1]; ++e)
      if (cb.pt[e] == ctr) chiq = cb.val[e];
    if (chiq == 0.0) continue;
    const double* R = c->img + 3 * cb.prj_img[p];
    double s = 0.0;
    for (int e = cb.ptr[p]; e < cb.ptr[p + 1]; ++e) s += cb.val[e] * d[cb.pt[e]];
    enl += 2.0 * cb.gdv[p] * chiq * s;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double gab = 0.0;
        for (int e = cb.ptr[p]; e < cb.ptr[p + 1]; ++e) {
          int pt = cb.pt[e];
          int o[3] = {pt % cb.nc - m, (pt / cb.nc) % cb.nc - m, pt / (cb.nc * cb.nc) - m};
          double yb = (double)(cb.q[b] + o[b]) * c->h;
          gab += cb.val[e] * (yb - R[b]) * g[a][pt];
        }
        out[9 + 3 * a + b] += -2.0 * cb.gdv[p] * chiq * ((a == b ? s : 0.0) + 2.0 * gab);
      }
  }
  out[18] = enl;
  out[19] = d[ctr];
  if (dcol) memcpy(dcol, d, sizeof(double) * Nc);
  for (int al = 0; al < 3; ++al) free(g[al]);
  free(gg); free(t0); free(t1); free(t2); free(y); free(d);
  cube_free(&cb);
}

/* Dense H_q (for tests on tiny cubes): column k = H_q e_k. */
void or_node_dense_H(const or_cell* c, long qnode, double* Hout) {
  or_cube cb;
  cube_build(c, qnode, &cb);
  int Nc = cb.Nc;
  double* e = (double*)calloc(Nc, sizeof(double));
  double* y = (double*)calloc(Nc, sizeof(double));
  for (int k = 0; k < Nc; ++k) {
    e[k] = 1.0;
    apply_H(c, &cb, e, y);
    for (int i = 0; i < Nc; ++i) Hout[(long)i * Nc + k] = y[i];
    e[k] = 0.0;
  }
  free(e); free(y);
  cube_free(&cb);
}

/* Number of projectors (images) with support in the cube, and the number of
 * (point, projector) pairs -- used to size the oracle's work, and in tests. */
void or_node_counts(const or_cell* c, long qnode, int* nprj, int* npairs) {
  or_cube cb;
  cube_build(c, qnode, &cb);
  *nprj = cb.nprj;
  *npairs = cb.ptr[cb.nprj];
  cube_free(&cb);
}

/* Local potential on the periodic grid: V_loc(x_i) = sum over images of
 * V(|x_i - R|), V(r) = -v_amp exp(-r^2/(2 v_sigma^2)) for r < v_rcut. */
void or_vloc(const or_cell* c, double* out) {
  long Nd = (long)c->n[0] * c->n[1] * c->n[2];
#pragma omp parallel for schedule(static)
  for (long i = 0; i < Nd; ++i) {
    int ix = (int)(i % c->n[0]);
    int iy = (int)((i / c->n[0]) % c->n[1]);
    int iz = (int)(i / ((long)c->n[0] * c->n[1]));
    double x = (double)ix * c->h, y = (double)iy * c->h, z = (double)iz * c->h;
    double v = 0.0;
    for (int I = 0; I < c->nimg; ++I) {
      const double* s = c->sp + SP_STRIDE * c->img_sp[I];
      double dx = x - c->img[3 * I], dy = y - c->img[3 * I + 1], dz = z - c->img[3 * I + 2];
      double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < s[2] * s[2]) v += -s[0] * exp(-r2 / (2.0 * s[1] * s[1]));
    }
    out[i] = v;
  }
}

/* ---- batch drivers: independent node columns side by side ---------------- */

void or_batch_lanczos(const or_cell* c, const long* nodes, long n, int K,
                      double* alpha, double* beta, int* steps) {
#pragma omp parallel for schedule(dynamic, 1)
  for (long i = 0; i < n; ++i)
    steps[i] = or_node_lanczos(c, nodes[i], K, alpha + i * K, beta + i * K, NULL);
}

void or_batch_moments(const or_cell* c, const long* nodes, long n, const double* chi,
                      const double* zeta, int npl, double* mom) {
#pragma omp parallel for schedule(dynamic, 1)
  for (long i = 0; i < n; ++i)
    or_node_moments(c, nodes[i], chi[i], zeta[i], npl, mom + i * (npl + 1));
}

void or_batch_stress(const or_cell* c, const long* nodes, long n, const double* chi,
                     const double* zeta, int npl, const double* coef, double* out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (long i = 0; i < n; ++i)
    or_node_stress(c, nodes[i], chi[i], zeta[i], npl, coef + i * (npl + 1), out + i * 20, NULL);
}

/* For tests: per projector touching the cube of node q, the image index and
 * sum_a chi(a).  Returns the number of projectors written (<= cap). */
int or_node_projector_sums(const or_cell* c, long qnode, int cap, int* img, double* sums) {
  or_cube cb;
  cube_build(c, qnode, &cb);
  int n = cb.nprj < cap ? cb.nprj : cap;
  for (int p = 0; p < n; ++p) {
    double s = 0.0;
    for (int e = cb.ptr[p]; e < cb.ptr[p + 1]; ++e) s += cb.val[e];
    img[p] = cb.prj_img[p];
    sums[p] = s;
  }
  cube_free(&cb);
  return n;
}
