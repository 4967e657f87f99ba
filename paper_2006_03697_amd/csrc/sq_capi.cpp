// sq_capi.cpp -- the C ABI (include/sq.h): validation, per-cell tables
// (grid, atom images, per-tile image lists), device memory, and the order
// of kernel launches for density, band energy and stress.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "sq.h"
#include "sq_dev.h"

namespace {

struct CellHost {
  int n[3];
  long long Nd, node_base;
  int m, nc, npl, K, mu_mode;
  double h, L[3], dV, vol, kT, ne, mu0;
  std::vector<double> pos;
  std::vector<int> species;
  std::vector<sq_species> sp;
  std::vector<double> img;   // [nimg][4]
  int ntile[3];
  std::vector<int> tile_ptr, tile_img;
  int max_tile;
  int census_img = 0, census_col = 0, census_near = 0;   // measured capacities
  long long census_pairs = 0;                             // (node, projector) pairs
  double c2[SQ_FDM + 1], c1[SQ_FDM + 1];
  double* d_vloc = nullptr;
  double* d_img = nullptr;
  int* d_tile_ptr = nullptr;
  int* d_tile_img = nullptr;
};

struct Group {
  int nc, kc;
  bool fused;   // the nodes' Gram matrices fit: one sweep per recurrence step
  long long n;
  long long* items;
  int* cell;
};

struct Selection {
  std::vector<Group> groups;   // nodes grouped by cube size
  long long nall = 0;
  long long* items = nullptr;  // every node of the selection
  int* item_cell = nullptr;
  std::vector<int> cells;
  int* d_cells = nullptr;
  int* d_fixed = nullptr;
};

}  // namespace

enum Phase { PH_LANCZOS, PH_BOUNDS, PH_MOMENTS, PH_MU, PH_COEFFS, PH_STRESS, PH_REDUCE, PH_N };

struct sq_plan_s {
  std::vector<CellHost> cells;
  hipEvent_t ev0[PH_N] = {}, ev1[PH_N] = {};
  bool ev_open[PH_N] = {};
  double phase_ms[PH_N] = {};
  long long phase_n[PH_N] = {};
  sq_options opt{};
  hipStream_t stream = nullptr;
  int device = 0;
  PlanDev P{};
  CellDev* d_cells = nullptr;
  std::vector<void*> allocs;
  Selection all;
  std::vector<Selection> per_cell;
  std::vector<int> density_done, stress_done;
  long long Ntot = 0;
  std::vector<CellDev> host_cells;   // what was uploaded to d_cells
  std::string err;
};

namespace {

thread_local std::string g_setup_err;

sq_status fail(sq_plan p, sq_status s, const std::string& msg) {
  if (p) p->err = msg;
  g_setup_err = msg;
  return s;
}

void* dalloc(sq_plan p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  void* ptr = nullptr;
  if (p->opt.dev_alloc) {
    ptr = p->opt.dev_alloc(bytes, p->opt.alloc_ctx);
  } else if (hipMalloc(&ptr, bytes) != hipSuccess) {
    ptr = nullptr;
  }
  if (ptr) p->allocs.push_back(ptr);
  return ptr;
}

// Central FD weights of order 2M (closed form): second derivative c_k, first
// derivative w_k; integer arithmetic is exact in binary64 for M <= 6.
void fd_weights(int M, double* c2, double* c1) {
  auto fact = [](int k) {
    double f = 1.0;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
  };
  long double s = 0.0L;
  c1[0] = 0.0;
  for (int k = 1; k <= M; ++k) {
    const double num = fact(M) * fact(M);
    const double den = fact(M - k) * fact(M + k);
    const double sgn = (k % 2 == 1) ? 1.0 : -1.0;
    c2[k] = sgn * 2.0 * num / (den * (double)(k * k));
    c1[k] = sgn * num / (den * (double)k);
    s += (long double)sgn * 2.0L * (long double)num / ((long double)den * (long double)(k * k));
  }
  c2[0] = (double)(-2.0L * s);
}

double box_dist2(const double* R, const double* lo, const double* hi) {
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double e = R[a] < lo[a] ? lo[a] - R[a] : (R[a] > hi[a] ? R[a] - hi[a] : 0.0);
    d2 += e * e;
  }
  return d2;
}

sq_status build_cell(sq_plan p, const sq_cell& in, CellHost& c, int idx) {
  const std::string tag = "cell " + std::to_string(idx) + ": ";
  if (!(in.h > 0)) return fail(p, SQ_E_ARG, tag + "h must be positive");
  c.h = in.h;
  for (int a = 0; a < 3; ++a) {
    const double f = in.L[a] / in.h;
    const double r = std::nearbyint(f);
    if (!(in.L[a] > 0) || std::fabs(f - r) > 1e-9 * f || r < 1)
      return fail(p, SQ_E_ARG, tag + "L/h is not a positive integer");
    c.n[a] = (int)r;
    c.L[a] = in.L[a];
  }
  if (in.fd_half_order != SQ_FDM) return fail(p, SQ_E_ARG, tag + "only 12th-order FD (M = 6)");
  if (!(in.rcut >= in.h)) return fail(p, SQ_E_ARG, tag + "R_cut must be at least h");
  c.m = (int)std::floor(in.rcut / in.h + 1e-9);
  c.nc = 2 * c.m + 1;
  if (!sq_nc_supported(c.nc)) return fail(p, SQ_E_ARG, tag + "cube width must be odd in [7, 25]");
  if (in.npl < 1 || in.npl > 256) return fail(p, SQ_E_ARG, tag + "npl must be in [1, 256]");
  if (!(in.kT > 0)) return fail(p, SQ_E_ARG, tag + "kT must be positive");
  c.K = in.lanczos_steps == 0 ? 20 : in.lanczos_steps;
  if (c.K < 2 || c.K > SQ_KL_MAX) return fail(p, SQ_E_ARG, tag + "lanczos_steps must be in [2, 64]");
  if (in.n_species < 1 || in.n_species > SQ_MAX_SPECIES || !in.sp)
    return fail(p, SQ_E_ARG, tag + "1..4 species required");
  if (in.n_atoms < 0 || (in.n_atoms > 0 && (!in.pos || !in.species)))
    return fail(p, SQ_E_ARG, tag + "atom arrays missing");
  c.sp.assign(in.sp, in.sp + in.n_species);
  for (const auto& s : c.sp)
    if (!(s.v_sigma > 0 && s.p_sigma > 0 && s.v_rcut > 0 && s.p_rcut > 0))
      return fail(p, SQ_E_ARG, tag + "species widths and cutoffs must be positive");
  c.npl = in.npl;
  c.kT = in.kT;
  c.mu_mode = in.mu_mode;
  c.mu0 = in.mu;
  c.Nd = (long long)c.n[0] * c.n[1] * c.n[2];
  c.dV = c.h * c.h * c.h;
  c.vol = c.L[0] * c.L[1] * c.L[2];
  c.pos.resize(3 * (size_t)in.n_atoms);
  c.species.resize(in.n_atoms);
  double zsum = 0.0;
  for (int I = 0; I < in.n_atoms; ++I) {
    const int s = in.species[I];
    if (s < 0 || s >= in.n_species) return fail(p, SQ_E_ARG, tag + "species index out of range");
    c.species[I] = s;
    zsum += c.sp[s].z_val;
    for (int a = 0; a < 3; ++a) {
      const double x = in.pos[3 * I + a];
      c.pos[3 * I + a] = x - c.L[a] * std::floor(x / c.L[a]);
    }
  }
  c.ne = in.n_electrons < 0 ? zsum : in.n_electrons;
  if (in.mu_mode == SQ_MU_SOLVE && !(c.ne > 0 && c.ne < 2.0 * (double)c.Nd))
    return fail(p, SQ_E_ARG, tag + "N_e must lie in (0, 2 N_d)");
  fd_weights(SQ_FDM, c.c2, c.c1);

  // atom images that reach any node's cube (projector) or any node (potential)
  double reach = 0.0, rpmax = 0.0;
  for (const auto& s : c.sp) {
    reach = std::max(reach, std::max(s.v_rcut, s.p_rcut));
    rpmax = std::max(rpmax, s.p_rcut);
  }
  double blo[3], bhi[3];
  for (int a = 0; a < 3; ++a) {
    blo[a] = -c.m * c.h;
    bhi[a] = (c.n[a] - 1 + c.m) * c.h;
  }
  c.img.clear();
  for (int I = 0; I < in.n_atoms; ++I) {
    int r0[3], r1[3];
    for (int a = 0; a < 3; ++a) {
      const double x = c.pos[3 * I + a];
      r0[a] = (int)std::floor((blo[a] - reach - x) / c.L[a]) - 1;
      r1[a] = (int)std::ceil((bhi[a] + reach - x) / c.L[a]) + 1;
    }
    for (int i = r0[0]; i <= r1[0]; ++i)
      for (int j = r0[1]; j <= r1[1]; ++j)
        for (int k = r0[2]; k <= r1[2]; ++k) {
          double R[3];
          const int sh[3] = {i, j, k};
          for (int a = 0; a < 3; ++a) R[a] = c.pos[3 * I + a] + (double)sh[a] * c.L[a];
          if (box_dist2(R, blo, bhi) < reach * reach) {
            c.img.push_back(R[0]);
            c.img.push_back(R[1]);
            c.img.push_back(R[2]);
            c.img.push_back((double)c.species[I]);
          }
        }
  }
  const int nimg = (int)(c.img.size() / 4);

  // per-tile lists of the images whose projector may reach a cube of a node
  // of the tile (superset: each node filters it again)
  for (int a = 0; a < 3; ++a) c.ntile[a] = (c.n[a] + SQ_TILE - 1) / SQ_TILE;
  const long long ntiles = (long long)c.ntile[0] * c.ntile[1] * c.ntile[2];
  c.tile_ptr.assign(ntiles + 1, 0);
  c.tile_img.clear();
  c.max_tile = 0;
  // bin images by the tile-aligned cell they fall in to avoid an all-pairs scan
  const double span = SQ_TILE * c.h;
  const double margin = c.m * c.h + rpmax;
  for (long long t = 0; t < ntiles; ++t) {
    const int tx = (int)(t % c.ntile[0]);
    const int ty = (int)((t / c.ntile[0]) % c.ntile[1]);
    const int tz = (int)(t / ((long long)c.ntile[0] * c.ntile[1]));
    const int tt[3] = {tx, ty, tz};
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      const int n0 = tt[a] * SQ_TILE;
      const int n1 = std::min(c.n[a], (tt[a] + 1) * SQ_TILE) - 1;
      lo[a] = (n0 - c.m) * c.h;
      hi[a] = (n1 + c.m) * c.h;
    }
    int cnt = 0;
    for (int I = 0; I < nimg; ++I) {
      const double* R = &c.img[4 * (size_t)I];
      // quick reject on each axis
      bool ok = true;
      for (int a = 0; a < 3 && ok; ++a) ok = R[a] > lo[a] - rpmax - span && R[a] < hi[a] + rpmax + span;
      if (!ok) continue;
      const double rp = c.sp[(int)R[3]].p_rcut;
      if (box_dist2(R, lo, hi) < rp * rp * (1.0 + 1e-9) + 1e-12) {
        c.tile_img.push_back(I);
        ++cnt;
      }
    }
    c.tile_ptr[t + 1] = c.tile_ptr[t] + cnt;
    c.max_tile = std::max(c.max_tile, cnt);
  }
  (void)margin;
  return SQ_OK;
}

template <typename T>
T* upload(sq_plan p, const std::vector<T>& v, sq_status* st) {
  T* d = (T*)dalloc(p, sizeof(T) * std::max<size_t>(v.size(), 1));
  if (!d) {
    *st = fail(p, SQ_E_ALLOC, "device allocation failed");
    return nullptr;
  }
  if (!v.empty()) {
    // the source is pageable host memory owned by the caller's scope: the
    // copy must have completed before it returns
    hipError_t e = hipMemcpyAsync(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice,
                                  p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
      *st = fail(p, SQ_E_DEVICE, std::string("upload: ") + hipGetErrorString(e));
      return nullptr;
    }
  }
  return d;
}

// Nodes grouped by (cube width, slot capacity, Gram matrix stored); gn is
// the per-node Gram entry count (-1: over capacity), or NULL before it is known.
sq_status make_selection(sq_plan p, const std::vector<int>& cells, Selection& S,
                         const std::vector<int>* gn = nullptr) {
  S.cells = cells;
  std::map<std::tuple<int, int, bool>, std::vector<std::pair<long long, int>>> by_nc;
  std::vector<long long> all_items;
  std::vector<int> all_cells;
  for (int ci : cells) {
    const CellHost& c = p->cells[ci];
    for (long long q = 0; q < c.Nd; ++q) {
      const bool fused = !gn || (*gn)[c.node_base + q] >= 0;
      by_nc[std::make_tuple(c.nc, c.census_col, fused)].emplace_back(c.node_base + q, ci);
      all_items.push_back(c.node_base + q);
      all_cells.push_back(ci);
    }
  }
  sq_status st = SQ_OK;
  S.nall = (long long)all_items.size();
  S.items = upload(p, all_items, &st);
  S.item_cell = upload(p, all_cells, &st);
  std::vector<int> fixed;
  for (int ci : cells) fixed.push_back(p->cells[ci].mu_mode == SQ_MU_FIXED ? 1 : 0);
  S.d_cells = upload(p, cells, &st);
  S.d_fixed = upload(p, fixed, &st);
  for (auto& kv : by_nc) {
    std::vector<long long> it;
    std::vector<int> ce;
    for (auto& pr : kv.second) {
      it.push_back(pr.first);
      ce.push_back(pr.second);
    }
    Group g;
    g.nc = std::get<0>(kv.first);
    g.kc = std::get<1>(kv.first);
    g.fused = std::get<2>(kv.first);
    g.n = (long long)it.size();
    g.items = upload(p, it, &st);
    g.cell = upload(p, ce, &st);
    S.groups.push_back(g);
  }
  return st;
}

sq_status check_hip(sq_plan p, hipError_t e, const char* what) {
  if (e != hipSuccess)
    return fail(p, SQ_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return SQ_OK;
}

void phase_begin(sq_plan p, Phase ph) {
  if (p->ev0[ph] && hipEventRecord(p->ev0[ph], p->stream) == hipSuccess) p->ev_open[ph] = true;
}

void phase_end(sq_plan p, Phase ph) {
  if (p->ev_open[ph]) (void)hipEventRecord(p->ev1[ph], p->stream);
}

// After the stream has been synchronised: fold the recorded phases in.
void phase_collect(sq_plan p) {
  for (int ph = 0; ph < PH_N; ++ph) {
    if (!p->ev_open[ph]) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev0[ph], p->ev1[ph]) == hipSuccess) {
      p->phase_ms[ph] += ms;
      p->phase_n[ph] += 1;
    }
    p->ev_open[ph] = false;
  }
}

// The device copy of the cell table must never change after set-up.
sq_status verify_cells(sq_plan p, const char* where) {
  std::vector<CellDev> back(p->host_cells.size());
  hipError_t e = hipMemcpyAsync(back.data(), p->d_cells, sizeof(CellDev) * back.size(),
                                hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return check_hip(p, e, where);
  if (std::memcmp(back.data(), p->host_cells.data(), sizeof(CellDev) * back.size()) != 0) {
    const unsigned char* a = (const unsigned char*)back.data();
    const unsigned char* b = (const unsigned char*)p->host_cells.data();
    size_t off = 0;
    while (off < sizeof(CellDev) * back.size() && a[off] == b[off]) ++off;
    return fail(p, SQ_E_DEVICE, std::string(where) + ": device cell table differs from the uploaded one at byte " +
                                    std::to_string(off));
  }
  return SQ_OK;
}

sq_status select(sq_plan p, int cell, Selection** S) {
  if (cell == -1) {
    *S = &p->all;
    return SQ_OK;
  }
  if (cell < 0 || cell >= (int)p->cells.size()) return fail(p, SQ_E_ARG, "cell index out of range");
  *S = &p->per_cell[cell];
  return SQ_OK;
}

sq_status check_errors(sq_plan p) {
  unsigned h = 0;
  hipError_t e = hipMemcpyAsync(&h, p->P.err, sizeof(unsigned), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return check_hip(p, e, "device");
  if (h & SQ_ERR_IMAGES) return fail(p, SQ_E_ARG, "more atom images reach a cube than supported");
  if (h & SQ_ERR_SLOTS) return fail(p, SQ_E_ARG, "more atom images cross a cube column than supported");
  if (h & SQ_ERR_NEAR) return fail(p, SQ_E_ARG, "more projectors are nonzero at one node than supported");
  if (h & SQ_ERR_BOUNDS) return fail(p, SQ_E_BOUNDS, "a Chebyshev moment left [-1, 1]: spectral bounds too narrow");
  return SQ_OK;
}

sq_status copy_out(sq_plan p, void* dst, const void* src, size_t bytes) {
  const hipMemcpyKind k = p->opt.outputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  return check_hip(p, hipMemcpyAsync(dst, src, bytes, k, p->stream), "copy");
}

// Host value(s) to a caller's output buffer (device or host per the options).
sq_status put_out(sq_plan p, void* dst, const void* src, size_t bytes) {
  if (p->opt.outputs_on_device) return check_hip(p, hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), "output");
  std::memcpy(dst, src, bytes);
  return SQ_OK;
}

// Reduced per-cell records (every cell of the plan) to the host.
sq_status read_sums(sq_plan p, std::vector<double>& sums) {
  sums.assign((SQ_REC + 4) * p->cells.size(), 0.0);
  sq_status st = check_hip(p, hipMemcpyAsync(sums.data(), p->P.sums, sizeof(double) * sums.size(),
                                             hipMemcpyDeviceToHost, p->stream), "sums");
  if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(p->stream), "sums");
  return st;
}

// The stress pass over a selection: density-matrix columns, their gradients,
// K and N per node, the nonlocal energy per node, and the node sums of those
// columns.  Marks the cells' stress as done.
sq_status stress_pass(sq_plan p, Selection* S, std::vector<double>& sums) {
  for (int ci : S->cells)
    if (!p->density_done[ci]) return fail(p, SQ_E_STATE, "sq_stress / sq_pressure before sq_density");
  const bool fp64 = p->opt.precision == SQ_FP64;
  hipStream_t s = p->stream;
  sq_status st = check_hip(p, hipMemsetAsync(p->P.err, 0, sizeof(unsigned), s), "memset");
  phase_begin(p, PH_STRESS);
  for (const Group& g : S->groups)
    if (st == SQ_OK)
      st = check_hip(p, sq_launch_stress(g.nc, g.kc, fp64, g.fused, p->P, g.items, g.cell, g.n, s),
                     "stress");
  phase_end(p, PH_STRESS);
  phase_begin(p, PH_REDUCE);
  if (st == SQ_OK)
    st = check_hip(p, sq_launch_reduce(p->P, S->d_cells, (int)S->cells.size(), 2, 19, s), "reduce");
  phase_end(p, PH_REDUCE);
  if (st == SQ_OK) st = check_errors(p);
  phase_collect(p);
  if (st == SQ_OK) st = read_sums(p, sums);
  if (st == SQ_OK)
    for (int ci : S->cells) p->stress_done[ci] = 1;
  return st;
}

}  // namespace

extern "C" {

const char* sq_status_str(sq_status s) {
  switch (s) {
    case SQ_OK: return "ok";
    case SQ_E_ARG: return "invalid argument";
    case SQ_E_ALLOC: return "device allocation failed";
    case SQ_E_DEVICE: return "HIP runtime error";
    case SQ_E_BOUNDS: return "spectral bounds violated";
    case SQ_E_NOCONV: return "Fermi level not found";
    case SQ_E_STATE: return "call order violated";
  }
  return "unknown status";
}

// With a NULL plan: the message of the last failed sq_setup on this thread.
const char* sq_last_error(sq_plan plan) { return plan ? plan->err.c_str() : g_setup_err.c_str(); }

void sq_destroy(sq_plan plan) {
  if (!plan) return;
  if (plan->stream) (void)hipStreamSynchronize(plan->stream);
  for (int ph = 0; ph < PH_N; ++ph) {
    if (plan->ev0[ph]) (void)hipEventDestroy(plan->ev0[ph]);
    if (plan->ev1[ph]) (void)hipEventDestroy(plan->ev1[ph]);
  }
  for (void* a : plan->allocs) {
    if (plan->opt.dev_free) plan->opt.dev_free(a, plan->opt.alloc_ctx);
    else (void)hipFree(a);
  }
  delete plan;
}

sq_status sq_setup(const sq_cell* cells, int n_cells, const sq_options* opt, sq_plan* out) {
  if (!out) return fail(nullptr, SQ_E_ARG, "out is NULL");
  *out = nullptr;
  if (!cells || n_cells < 1 || !opt) return fail(nullptr, SQ_E_ARG, "cells / options missing");
  if (opt->precision != SQ_FP64 && opt->precision != SQ_MIXED && opt->precision != SQ_MIXED_STRESS)
    return fail(nullptr, SQ_E_ARG, "unknown precision");
  sq_plan p = new sq_plan_s();
  p->opt = *opt;
  p->stream = (hipStream_t)opt->hip_stream;
  sq_status st = SQ_OK;
  p->cells.resize(n_cells);
  int npl_max = 1;
  for (int i = 0; i < n_cells; ++i) {
    st = build_cell(p, cells[i], p->cells[i], i);
    if (st != SQ_OK) {
      sq_destroy(p);
      return st;
    }
    p->cells[i].node_base = p->Ntot;
    p->Ntot += p->cells[i].Nd;
    npl_max = std::max(npl_max, p->cells[i].npl);
  }
  const long long N = p->Ntot;
  PlanDev& P = p->P;
  P.mstride = npl_max + 2;
  auto A = [&](size_t bytes) { return dalloc(p, bytes); };
  P.lan = (double*)A(sizeof(double) * 2 * SQ_KL_MAX * N);
  P.lan_steps = (int*)A(sizeof(int) * N);
  P.bnd = (double*)A(sizeof(double) * 4 * N);
  P.mom = (double*)A(sizeof(double) * P.mstride * N);
  P.coef = (double*)A(sizeof(double) * P.mstride * N);
  P.rec = (double*)A(sizeof(double) * SQ_REC * N);
  P.nq = (double*)A(sizeof(double) * N);
  P.nqd = (double*)A(sizeof(double) * N);
  P.mus = (double*)A(sizeof(double) * SQ_MU_STRIDE * n_cells);
  P.sums = (double*)A(sizeof(double) * (SQ_REC + 4) * n_cells);
  P.err = (unsigned*)A(sizeof(unsigned) * 4);
  P.gval = (double*)A(sizeof(double) * SQ_GRAM_MAX * N);
  P.gidx = (unsigned*)A(sizeof(unsigned) * SQ_GRAM_MAX * N);
  P.gn = (int*)A(sizeof(int) * N);
  p->d_cells = (CellDev*)A(sizeof(CellDev) * n_cells);
  if (!P.lan || !P.lan_steps || !P.bnd || !P.mom || !P.coef || !P.rec || !P.nq || !P.nqd || !P.mus || !P.sums ||
      !P.err || !P.gval || !P.gidx || !P.gn || !p->d_cells) {
    sq_destroy(p);
    return fail(nullptr, SQ_E_ALLOC, "device allocation failed");
  }
  P.cells = p->d_cells;
  std::vector<CellDev> hc(n_cells);
  for (int i = 0; i < n_cells && st == SQ_OK; ++i) {
    CellHost& c = p->cells[i];
    c.d_vloc = (double*)A(sizeof(double) * c.Nd);
    if (!c.d_vloc) st = SQ_E_ALLOC;
    if (st == SQ_OK) c.d_img = upload(p, c.img, &st);
    if (st == SQ_OK) c.d_tile_ptr = upload(p, c.tile_ptr, &st);
    if (st == SQ_OK) c.d_tile_img = upload(p, c.tile_img, &st);
    CellDev& d = hc[i];
    std::memset(&d, 0, sizeof(d));
    for (int a = 0; a < 3; ++a) {
      d.n[a] = c.n[a];
      d.ntile[a] = c.ntile[a];
      d.L[a] = c.L[a];
    }
    d.m = c.m;
    d.nc = c.nc;
    d.npl = c.npl;
    d.K = c.K;
    d.nimg = (int)(c.img.size() / 4);
    d.nsp = (int)c.sp.size();
    d.mu_mode = c.mu_mode;
    d.Nd = c.Nd;
    d.node_base = c.node_base;
    d.h = c.h;
    d.dV = c.dV;
    d.kT = c.kT;
    d.ne = c.ne;
    d.vol = c.vol;
    d.mu0 = c.mu0;
    for (int k = 0; k <= SQ_FDM; ++k) {
      d.c2[k] = c.c2[k];
      d.c1[k] = c.c1[k];
      d.ck[k] = k == 0 ? 0.0 : -0.5 / (c.h * c.h) * c.c2[k];
      d.ckf[k] = (float)d.ck[k];
    }
    for (int s = 0; s < (int)c.sp.size(); ++s) {
      d.sp[s].v_amp = c.sp[s].v_amp;
      d.sp[s].v_sig = c.sp[s].v_sigma;
      d.sp[s].v_rc = c.sp[s].v_rcut;
      d.sp[s].p_sig = c.sp[s].p_sigma;
      d.sp[s].p_rc = c.sp[s].p_rcut;
      d.sp[s].gamma = c.sp[s].gamma;
    }
    d.vloc = c.d_vloc;
    d.img = c.d_img;
    d.tile_ptr = c.d_tile_ptr;
    d.tile_img = c.d_tile_img;
  }
  p->host_cells = hc;
  if (st == SQ_OK)
    st = check_hip(p, hipMemcpyAsync(p->d_cells, p->host_cells.data(), sizeof(CellDev) * n_cells,
                                     hipMemcpyHostToDevice, p->stream), "upload cells");
  if (st == SQ_OK) st = verify_cells(p, "after upload");
  for (int i = 0; i < n_cells && st == SQ_OK; ++i)
    st = check_hip(p, sq_launch_vloc(p->d_cells + i, hc[i], p->cells[i].d_vloc, p->stream), "vloc");
  // capacity census: images per cube, per z-column and at the node itself
  if (st == SQ_OK) {
    std::vector<int> all(n_cells);
    for (int i = 0; i < n_cells; ++i) all[i] = i;
    Selection pre;
    st = make_selection(p, all, pre);
    int* d_stats = (int*)A(sizeof(int) * 4 * n_cells);
    long long* d_pairs = (long long*)A(sizeof(long long) * n_cells);
    if (!d_stats || !d_pairs) st = SQ_E_ALLOC;
    if (st == SQ_OK) st = check_hip(p, hipMemsetAsync(d_stats, 0, sizeof(int) * 4 * n_cells, p->stream), "memset");
    if (st == SQ_OK) st = check_hip(p, hipMemsetAsync(d_pairs, 0, sizeof(long long) * n_cells, p->stream), "memset");
    if (st == SQ_OK) st = check_hip(p, hipMemsetAsync(P.err, 0, sizeof(unsigned), p->stream), "memset");
    for (const Group& g : pre.groups)
      if (st == SQ_OK)
        st = check_hip(p, sq_launch_census(g.nc, P, g.items, g.cell, g.n, d_stats, d_pairs, p->stream), "census");
    std::vector<int> stats(4 * n_cells);
    std::vector<long long> pairs(n_cells);
    if (st == SQ_OK)
      st = check_hip(p, hipMemcpyAsync(stats.data(), d_stats, sizeof(int) * stats.size(),
                                       hipMemcpyDeviceToHost, p->stream), "census copy");
    if (st == SQ_OK)
      st = check_hip(p, hipMemcpyAsync(pairs.data(), d_pairs, sizeof(long long) * pairs.size(),
                                       hipMemcpyDeviceToHost, p->stream), "census copy");
    if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(p->stream), "census");
    const bool fp64 = p->opt.precision == SQ_FP64;   // both passes FP64
    for (int i = 0; i < n_cells && st == SQ_OK; ++i) {
      CellHost& c = p->cells[i];
      c.census_img = stats[4 * i];
      c.census_col = std::max(1, stats[4 * i + 1]);
      c.census_near = stats[4 * i + 2];
      c.census_pairs = pairs[i];
      const std::string tag = "cell " + std::to_string(i) + ": ";
      // the FP64 Lanczos runs in every precision mode
      const int kc_lim = std::min(sq_kc_limit(true, c.nc), sq_kc_limit(fp64, c.nc));
      const int img_lim = sq_img_limit(c.nc);
      if (c.census_img > img_lim)
        st = fail(p, SQ_E_ARG, tag + std::to_string(c.census_img) +
                                   " atom images reach one cube (at most " +
                                   std::to_string(img_lim) + " supported)");
      else if (c.census_col > kc_lim)
        st = fail(p, SQ_E_ARG, tag + std::to_string(c.census_col) +
                                   " atom images cross one cube column (at most " +
                                   std::to_string(kc_lim) + " supported at this cube width)");
      else if (c.census_near > SQ_NEAR_MAX)
        st = fail(p, SQ_E_ARG, tag + "more than 32 projectors are nonzero at one node");
    }
  }
  // Gram matrices of every node's projectors (geometry only), then the node
  // groups, split by whether a node's Gram matrix fits
  if (st == SQ_OK) {
    std::vector<int> all(n_cells);
    for (int i = 0; i < n_cells; ++i) all[i] = i;
    Selection pre;
    st = make_selection(p, all, pre);
    for (const Group& g : pre.groups)
      if (st == SQ_OK) st = check_hip(p, sq_launch_gram(g.nc, g.kc, P, g.items, g.cell, g.n, p->stream), "gram");
    std::vector<int> gn(N);
    if (st == SQ_OK)
      st = check_hip(p, hipMemcpyAsync(gn.data(), P.gn, sizeof(int) * N, hipMemcpyDeviceToHost, p->stream),
                     "gram copy");
    if (st == SQ_OK) st = check_errors(p);
    if (st == SQ_OK) st = make_selection(p, all, p->all, &gn);
    p->per_cell.resize(n_cells);
    for (int i = 0; i < n_cells && st == SQ_OK; ++i) st = make_selection(p, {i}, p->per_cell[i], &gn);
  }
  if (st == SQ_OK) {
    st = check_hip(p, hipMemsetAsync(P.rec, 0, sizeof(double) * SQ_REC * N, p->stream), "memset");
    if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(p->stream), "setup");
    if (st == SQ_OK) st = verify_cells(p, "end of setup");
  }
  if (st != SQ_OK) {
    g_setup_err = p->err;
    sq_destroy(p);
    return st;
  }
  for (int ph = 0; ph < PH_N; ++ph) {
    if (hipEventCreate(&p->ev0[ph]) != hipSuccess) p->ev0[ph] = nullptr;
    if (hipEventCreate(&p->ev1[ph]) != hipSuccess) p->ev1[ph] = nullptr;
  }
  p->density_done.assign(n_cells, 0);
  p->stress_done.assign(n_cells, 0);
  *out = p;
  return SQ_OK;
}

sq_status sq_lanczos(sq_plan p, int cell, const int64_t* nodes, int64_t n, double* out) {
  if (!p || cell < 0 || cell >= (int)p->cells.size() || (n > 0 && (!nodes || !out))) return SQ_E_ARG;
  if (!p->density_done[cell]) return fail(p, SQ_E_STATE, "sq_lanczos before sq_density");
  const CellHost& c = p->cells[cell];
  const int W = 2 * SQ_KL_MAX;
  std::vector<double> lan((size_t)W * c.Nd);
  std::vector<int> steps(c.Nd);
  sq_status st = check_hip(p, hipMemcpyAsync(lan.data(), p->P.lan + c.node_base * W,
                                             sizeof(double) * lan.size(), hipMemcpyDeviceToHost,
                                             p->stream), "lanczos");
  if (st == SQ_OK)
    st = check_hip(p, hipMemcpyAsync(steps.data(), p->P.lan_steps + c.node_base,
                                     sizeof(int) * steps.size(), hipMemcpyDeviceToHost, p->stream),
                   "lanczos");
  if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(p->stream), "lanczos");
  if (st != SQ_OK) return st;
  const int K = c.K;
  for (int64_t i = 0; i < n; ++i) {
    if (nodes[i] < 0 || nodes[i] >= c.Nd) return fail(p, SQ_E_ARG, "node index out of range");
    double* o = out + (size_t)(2 * K + 1) * i;
    const int ns = steps[nodes[i]];
    o[0] = ns;
    for (int k = 0; k < K; ++k) {
      o[1 + k] = k < ns ? lan[(size_t)W * nodes[i] + k] : 0.0;
      o[1 + K + k] = k < ns ? lan[(size_t)W * nodes[i] + SQ_KL_MAX + k] : 0.0;
    }
  }
  return SQ_OK;
}

sq_status sq_cell_info(sq_plan p, int cell, int64_t* info) {
  if (!p || !info || cell < 0 || cell >= (int)p->cells.size()) return SQ_E_ARG;
  const CellHost& c = p->cells[cell];
  info[0] = c.Nd;
  info[1] = c.nc;
  info[2] = c.npl;
  info[3] = (int64_t)(c.img.size() / 4);
  info[4] = c.max_tile;
  info[5] = c.census_img;
  info[6] = c.census_col;
  info[7] = c.census_near;
  info[8] = c.census_pairs;
  return SQ_OK;
}

sq_status sq_phase_times(sq_plan p, int reset, double* ms, int64_t* count) {
  if (!p) return SQ_E_ARG;
  for (int ph = 0; ph < PH_N; ++ph) {
    if (ms) ms[ph] = p->phase_ms[ph];
    if (count) count[ph] = p->phase_n[ph];
    if (reset) {
      p->phase_ms[ph] = 0.0;
      p->phase_n[ph] = 0;
    }
  }
  return SQ_OK;
}

sq_status sq_density(sq_plan p, int cell, double* rho, double* mu) {
  if (!p) return SQ_E_ARG;
  Selection* S = nullptr;
  sq_status st = select(p, cell, &S);
  if (st != SQ_OK) return st;
  const bool fp64 = p->opt.precision != SQ_MIXED;   // precision of the moments pass
  hipStream_t s = p->stream;
  st = check_hip(p, hipMemsetAsync(p->P.err, 0, sizeof(unsigned), s), "memset");
  phase_begin(p, PH_LANCZOS);
  for (const Group& g : S->groups)
    if (st == SQ_OK)
      st = check_hip(p, sq_launch_lanczos(g.nc, g.kc, g.fused, p->P, g.items, g.cell, g.n, s), "lanczos");
  phase_end(p, PH_LANCZOS);
  phase_begin(p, PH_BOUNDS);
  if (st == SQ_OK) st = check_hip(p, sq_launch_bounds(p->P, S->items, S->item_cell, S->nall, s), "bounds");
  phase_end(p, PH_BOUNDS);
  phase_begin(p, PH_MOMENTS);
  for (const Group& g : S->groups)
    if (st == SQ_OK)
      st = check_hip(p, sq_launch_moments(g.nc, g.kc, fp64, g.fused, p->P, g.items, g.cell, g.n, s),
                     "moments");
  phase_end(p, PH_MOMENTS);
  const int nc = (int)S->cells.size();
  phase_begin(p, PH_MU);
  if (st == SQ_OK) st = check_hip(p, sq_launch_mu_init(p->P, S->d_cells, nc, S->d_fixed, s), "mu init");
  if (st != SQ_OK) return st;
  st = check_errors(p);
  if (st != SQ_OK) return st;
  // Fermi level: bracketed root search entirely on the device; the host
  // checks for completion after 10 evaluations, then every 4
  std::vector<double> mus(SQ_MU_STRIDE * p->cells.size());
  for (int it = 0, blk = 10; it < 210 && st == SQ_OK; it += blk, blk = 4) {
    for (int k = 0; k < blk && st == SQ_OK; ++k) {
      st = check_hip(p, sq_launch_mu_eval(p->P, S->items, S->item_cell, S->nall, s), "mu eval");
      if (st == SQ_OK) st = check_hip(p, sq_launch_mu_step(p->P, S->d_cells, nc, s), "mu step");
    }
    if (st != SQ_OK) break;
    st = check_hip(p, hipMemcpyAsync(mus.data(), p->P.mus, sizeof(double) * mus.size(),
                                     hipMemcpyDeviceToHost, s), "mu copy");
    if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(s), "mu sync");
    bool done = true;
    for (int ci : S->cells) done = done && mus[SQ_MU_STRIDE * ci + MU_DONE] != 0.0;
    if (done) break;
  }
  if (st != SQ_OK) return st;
  for (int ci : S->cells) {
    if (mus[SQ_MU_STRIDE * ci + MU_DONE] == 2.0)
      return fail(p, SQ_E_NOCONV, "cell " + std::to_string(ci) + ": N_e not bracketed");
    if (mus[SQ_MU_STRIDE * ci + MU_DONE] == 0.0)
      return fail(p, SQ_E_NOCONV, "cell " + std::to_string(ci) + ": Fermi-level search did not finish");
  }
  phase_end(p, PH_MU);
  phase_begin(p, PH_COEFFS);
  st = check_hip(p, sq_launch_coeffs(p->P, S->items, S->item_cell, S->nall, s), "coeffs");
  phase_end(p, PH_COEFFS);
  if (st == SQ_OK) st = check_errors(p);
  phase_collect(p);
  if (st != SQ_OK) return st;
  long long off = 0;
  for (int ci : S->cells) {
    const CellHost& c = p->cells[ci];
    if (rho) {
      const hipMemcpyKind k = p->opt.outputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
      st = check_hip(p, hipMemcpy2DAsync(rho + off, sizeof(double), p->P.rec + c.node_base * SQ_REC,
                                         sizeof(double) * SQ_REC, sizeof(double), c.Nd, k, s),
                     "rho copy");
      if (st != SQ_OK) return st;
    }
    off += c.Nd;
  }
  if (mu) {
    for (size_t i = 0; i < S->cells.size(); ++i) {
      const double v = mus[SQ_MU_STRIDE * S->cells[i] + MU_VAL];
      if (p->opt.outputs_on_device)
        st = check_hip(p, hipMemcpyAsync(mu + i, &v, sizeof(double), hipMemcpyHostToDevice, s), "mu");
      else
        mu[i] = v;
    }
  }
  if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(s), "density");
  if (st == SQ_OK) st = verify_cells(p, "end of density");
  if (st == SQ_OK)
    for (int ci : S->cells) {
      p->density_done[ci] = 1;
      p->stress_done[ci] = 0;
    }
  return st;
}

sq_status sq_energy(sq_plan p, int cell, double* e_band) {
  if (!p) return SQ_E_ARG;
  Selection* S = nullptr;
  sq_status st = select(p, cell, &S);
  if (st != SQ_OK) return st;
  for (int ci : S->cells)
    if (!p->density_done[ci]) return fail(p, SQ_E_STATE, "sq_energy before sq_density");
  hipStream_t s = p->stream;
  phase_begin(p, PH_REDUCE);
  st = check_hip(p, sq_launch_reduce(p->P, S->d_cells, (int)S->cells.size(), 1, 1, s), "reduce");
  phase_end(p, PH_REDUCE);
  std::vector<double> sums;
  if (st == SQ_OK) st = read_sums(p, sums);
  phase_collect(p);
  if (st != SQ_OK || !e_band) return st;
  for (size_t i = 0; i < S->cells.size() && st == SQ_OK; ++i)
    st = put_out(p, e_band + i, &sums[(SQ_REC + 4) * S->cells[i] + 1], sizeof(double));
  return st;
}

sq_status sq_stress(sq_plan p, int cell, double* sigma_voigt, double* parts) {
  if (!p) return SQ_E_ARG;
  Selection* S = nullptr;
  sq_status st = select(p, cell, &S);
  if (st != SQ_OK) return st;
  std::vector<double> sums;
  st = stress_pass(p, S, sums);
  if (st != SQ_OK) return st;
  for (size_t i = 0; i < S->cells.size(); ++i) {
    const int ci = S->cells[i];
    const double* pr = &sums[(SQ_REC + 4) * ci + 2];
    const double vol = p->cells[ci].vol;
    double sg[9];
    for (int t = 0; t < 9; ++t) sg[t] = (pr[t] + pr[9 + t]) / vol;
    double v6[6] = {sg[0], sg[4], sg[8], 0.5 * (sg[5] + sg[7]), 0.5 * (sg[2] + sg[6]),
                    0.5 * (sg[1] + sg[3])};
    if (sigma_voigt && st == SQ_OK) st = put_out(p, sigma_voigt + 6 * i, v6, sizeof(v6));
    if (parts && st == SQ_OK) st = put_out(p, parts + 18 * i, pr, sizeof(double) * 18);
  }
  return st;
}

sq_status sq_pressure(sq_plan p, int cell, double* p_direct, double* p_trace) {
  if (!p) return SQ_E_ARG;
  Selection* S = nullptr;
  sq_status st = select(p, cell, &S);
  if (st != SQ_OK) return st;
  bool need = false;
  for (int ci : S->cells) need = need || !p->stress_done[ci];
  std::vector<double> sums;
  if (need) {
    st = stress_pass(p, S, sums);
  } else {
    for (int ci : S->cells)
      if (!p->density_done[ci]) return fail(p, SQ_E_STATE, "sq_pressure before sq_density");
  }
  // band energy and local-potential energy columns (the stress columns are
  // reduced by the stress pass)
  hipStream_t s = p->stream;
  phase_begin(p, PH_REDUCE);
  if (st == SQ_OK)
    st = check_hip(p, sq_launch_reduce(p->P, S->d_cells, (int)S->cells.size(), 1, 1, s), "reduce");
  if (st == SQ_OK)
    st = check_hip(p, sq_launch_reduce(p->P, S->d_cells, (int)S->cells.size(), 21, 1, s), "reduce");
  phase_end(p, PH_REDUCE);
  if (st == SQ_OK) st = read_sums(p, sums);
  phase_collect(p);
  if (st != SQ_OK) return st;
  for (size_t i = 0; i < S->cells.size(); ++i) {
    const int ci = S->cells[i];
    const double* r = &sums[(SQ_REC + 4) * ci];
    const double vol3 = 3.0 * p->cells[ci].vol;
    const double trK = r[2] + r[6] + r[10], trN = r[11] + r[15] + r[19];
    const double pd = -(-2.0 * r[1] + 2.0 * r[21] + 2.0 * r[20] + trN) / vol3;
    const double pt = -(trK + trN) / vol3;
    if (p_direct && st == SQ_OK) st = put_out(p, p_direct + i, &pd, sizeof(double));
    if (p_trace && st == SQ_OK) st = put_out(p, p_trace + i, &pt, sizeof(double));
  }
  return st;
}

sq_status sq_xc(sq_plan p, int cell, double* e_xc, double* sigma_xc) {
  if (!p) return SQ_E_ARG;
  Selection* S = nullptr;
  sq_status st = select(p, cell, &S);
  if (st != SQ_OK) return st;
  for (int ci : S->cells)
    if (!p->density_done[ci]) return fail(p, SQ_E_STATE, "sq_xc before sq_density");
  hipStream_t s = p->stream;
  phase_begin(p, PH_REDUCE);
  st = check_hip(p, sq_launch_reduce(p->P, S->d_cells, (int)S->cells.size(), 22, 2, s), "reduce");
  phase_end(p, PH_REDUCE);
  std::vector<double> sums;
  if (st == SQ_OK) st = read_sums(p, sums);
  phase_collect(p);
  if (st != SQ_OK) return st;
  for (size_t i = 0; i < S->cells.size() && st == SQ_OK; ++i) {
    const int ci = S->cells[i];
    const double* r = &sums[(SQ_REC + 4) * ci];
    const double sg = r[23] / p->cells[ci].vol;
    if (e_xc) st = put_out(p, e_xc + i, &r[22], sizeof(double));
    if (sigma_xc && st == SQ_OK) st = put_out(p, sigma_xc + i, &sg, sizeof(double));
  }
  return st;
}

sq_status sq_nodes(sq_plan p, int cell, const int64_t* nodes, int64_t n, double* out) {
  if (!p || cell < 0 || cell >= (int)p->cells.size() || (n > 0 && (!nodes || !out))) return SQ_E_ARG;
  if (!p->density_done[cell]) return fail(p, SQ_E_STATE, "sq_nodes before sq_density");
  const CellHost& c = p->cells[cell];
  std::vector<double> all(SQ_REC * (size_t)c.Nd);
  sq_status st = check_hip(p, hipMemcpyAsync(all.data(), p->P.rec + c.node_base * SQ_REC,
                                             sizeof(double) * all.size(), hipMemcpyDeviceToHost,
                                             p->stream), "nodes");
  if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(p->stream), "nodes");
  if (st != SQ_OK) return st;
  for (int64_t i = 0; i < n; ++i) {
    if (nodes[i] < 0 || nodes[i] >= c.Nd) return fail(p, SQ_E_ARG, "node index out of range");
    std::memcpy(out + SQ_REC * i, &all[SQ_REC * nodes[i]], sizeof(double) * SQ_REC);
  }
  return SQ_OK;
}

sq_status sq_bounds(sq_plan p, int cell, double* lam_lo, double* lam_hi) {
  if (!p || cell < 0 || cell >= (int)p->cells.size()) return SQ_E_ARG;
  if (!p->density_done[cell]) return fail(p, SQ_E_STATE, "sq_bounds before sq_density");
  const CellHost& c = p->cells[cell];
  std::vector<double> b(4 * (size_t)c.Nd);
  sq_status st = check_hip(p, hipMemcpyAsync(b.data(), p->P.bnd + 4 * c.node_base,
                                             sizeof(double) * b.size(), hipMemcpyDeviceToHost,
                                             p->stream), "bounds");
  if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(p->stream), "bounds");
  if (st != SQ_OK) return st;
  for (long long q = 0; q < c.Nd; ++q) {
    if (lam_lo) lam_lo[q] = b[4 * q];
    if (lam_hi) lam_hi[q] = b[4 * q + 1];
  }
  return SQ_OK;
}

sq_status sq_moments(sq_plan p, int cell, const int64_t* nodes, int64_t n, double* out) {
  if (!p || cell < 0 || cell >= (int)p->cells.size() || (n > 0 && (!nodes || !out))) return SQ_E_ARG;
  if (!p->density_done[cell]) return fail(p, SQ_E_STATE, "sq_moments before sq_density");
  const CellHost& c = p->cells[cell];
  const int ms = p->P.mstride;
  std::vector<double> all((size_t)ms * c.Nd);
  sq_status st = check_hip(p, hipMemcpyAsync(all.data(), p->P.mom + c.node_base * ms,
                                             sizeof(double) * all.size(), hipMemcpyDeviceToHost,
                                             p->stream), "moments");
  if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(p->stream), "moments");
  if (st != SQ_OK) return st;
  for (int64_t i = 0; i < n; ++i) {
    if (nodes[i] < 0 || nodes[i] >= c.Nd) return fail(p, SQ_E_ARG, "node index out of range");
    std::memcpy(out + (size_t)(c.npl + 1) * i, &all[(size_t)ms * nodes[i]], sizeof(double) * (c.npl + 1));
  }
  return SQ_OK;
}

}  // extern "C"
