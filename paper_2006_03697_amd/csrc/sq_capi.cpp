// sq_capi.cpp -- the C ABI (include/sq.h): validation, per-cell tables
// (grid, atom images, per-tile image lists), device memory, node groups and
// their tile shapes (fixed or autotuned), and the order of kernel launches
// for density, band energy and stress, eager or replayed from captured HIP
// graphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "sq.h"
#include "sq_dev.h"

#include <rocprofiler-sdk-roctx/roctx.h>

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
  // measured capacities: images per cube, per z-column, nonzero at the
  // node; (node, projector) pairs
  int census_img = 0, census_col = 0, census_near = 0;
  long long census_pairs = 0;
  long long gram_entries = 0, gram_nodes = 0;   // stored Gram entries; nodes on the single-sweep form
  double c2[SQ_FDM + 1], c1[SQ_FDM + 1];
  double* d_vloc = nullptr;
  double* d_img = nullptr;
  int* d_tile_ptr = nullptr;
  int* d_tile_img = nullptr;
};

// Variant of one kernel family on a node group.
struct Tile {
  int kc = 0;           // slot capacity (16, 24: plane-0 weights in registers, 48: recomputed); 0: smallest
  int persistent = 0;   // persistent grid with a work counter
};

enum Fam { F_LAN = 0, F_MOM = 1, F_STR = 2, F_N = 3 };

struct Group {
  int nc = 0;
  bool fused = true;    // the nodes' Gram matrices fit: one sweep per recurrence step
  int kc1 = 0;          // slot need per z-column (measured)
  long long n = 0;
  long long* items = nullptr;   // device, longest first
  int* cell = nullptr;
  std::vector<long long> h_items;
  std::vector<int> h_cell;
  Tile tile[F_N];
  unsigned* counter = nullptr;   // work counter of persistent launches
};

struct Selection {
  std::vector<Group> groups;   // nodes grouped by (cube width, Gram form, slot needs)
  long long nall = 0;
  long long* items = nullptr;  // every node of the selection, in node order
  int* item_cell = nullptr;
  std::vector<int> cells;
  int* d_cells = nullptr;
  int* d_fixed = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};           // density, stress pass
  hipGraphExec_t exec[2] = {nullptr, nullptr};
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
  hipStream_t cap = nullptr;   // private stream the graphs are captured on
  bool recording = true;       // phase events are recorded (not while capturing)
  PlanDev P{};
  CellDev* d_cells = nullptr;
  std::vector<void*> allocs;
  Selection all;
  std::vector<Selection> per_cell;
  std::vector<int> density_done, stress_done;
  double* static_sums = nullptr;     // this device's static scratch (sq_stress_static)
  std::vector<double> host_sums;     // its host copy, sized at set-up
  long long Ntot = 0;
  std::vector<CellDev> host_cells;   // what was uploaded to d_cells
  std::map<std::string, Tile> tuned; // autotuned tiles by key
  // moments from the Lanczos tridiagonal (every cell: max(K, ceil(npl / 2))
  // Lanczos steps fit one wave's components), else from the recurrence pass
  bool qmom = false;
  std::string arch;
  std::string err;
};

namespace {

// A roctx range over one entry point (host wall time, with its final
// synchronisation): rocprofv3 --marker-trace shows the calls beside the
// kernels they launch.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// Fermi-level evaluations launched back to back in every sq_density before
// the host looks at the search state; a search still running after them
// continues in rounds of SQ_MU_MORE up to SQ_MU_MAX evaluations.
constexpr int SQ_MU_BUDGET = 48;
constexpr int SQ_MU_MORE = 32;
constexpr int SQ_MU_MAX = 240;

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

// Lanczos steps whose tridiagonal fixes the moments up to degree npl
// (degree <= 2k after k steps), and never fewer than the bounds use.
int qmom_steps(const CellHost& c) { return std::max(c.K, (c.npl + 1) / 2); }

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

sq_status check_hip(sq_plan p, hipError_t e, const char* what) {
  if (e != hipSuccess)
    return fail(p, SQ_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return SQ_OK;
}

// Key of a tuned tile: device, group shape, precision and kernel family.
std::string tune_key(sq_plan p, const Group& g, int fam) {
  const bool fp64 = fam == F_LAN || (fam == F_MOM && p->opt.precision != SQ_MIXED) ||
                    (fam == F_STR && p->opt.precision == SQ_FP64);
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s|nc=%d|fused=%d|kc=%d|%s|%s", p->arch.c_str(), g.nc,
                g.fused ? 1 : 0, g.kc1, fp64 ? "fp64" : "fp32",
                fam == F_LAN ? "lanczos" : (fam == F_MOM ? "moments" : "stress"));
  return buf;
}

// A tile serves a group when its slot capacity holds the group's need and
// the persistent form is compiled for it (16-slot single sweep only).
bool tile_ok(const Group& g, const Tile& t) {
  const int kc = t.kc ? t.kc : sq_kc_variant(g.fused, g.kc1);
  if (kc == 0 || kc < g.kc1 || sq_kc_variant(g.fused, kc) != kc) return false;
  return !t.persistent || (g.fused && kc == 16);
}

// Default tile of a group: the smallest slot capacity, the launch form of
// the options where compiled; a tuned choice overrides both.
void default_tiles(sq_plan p, Group& g) {
  for (int f = 0; f < F_N; ++f) {
    Tile t;
    t.kc = 0;
    t.persistent = p->opt.persistent ? 1 : 0;
    if (!tile_ok(g, t)) t.persistent = 0;
    auto it = p->tuned.find(tune_key(p, g, f));
    if (it != p->tuned.end() && tile_ok(g, it->second)) t = it->second;
    g.tile[f] = t;
  }
}

// Nodes grouped by (cube width, Gram matrix stored, slot needs); gn is the
// per-node Gram entry count (-1: over capacity), or NULL before it is known.
// Within a group the nodes are ordered longest first (decreasing Chebyshev
// degree, then node order), so that the last workgroups of a launch are the
// short ones.
sq_status make_selection(sq_plan p, const std::vector<int>& cells, Selection& S,
                         const std::vector<int>* gn = nullptr) {
  S.cells = cells;
  std::map<std::tuple<int, bool, int>, std::vector<std::pair<long long, int>>> by;
  std::vector<long long> all_items;
  std::vector<int> all_cells;
  for (int ci : cells) {
    const CellHost& c = p->cells[ci];
    for (long long q = 0; q < c.Nd; ++q) {
      const bool fused = !gn || (*gn)[c.node_base + q] >= 0;
      by[std::make_tuple(c.nc, fused, c.census_col)].emplace_back(c.node_base + q, ci);
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
  for (auto& kv : by) {
    auto& v = kv.second;
    std::stable_sort(v.begin(), v.end(), [&](const std::pair<long long, int>& a,
                                             const std::pair<long long, int>& b) {
      return p->cells[a.second].npl > p->cells[b.second].npl;
    });
    Group g;
    g.nc = std::get<0>(kv.first);
    g.fused = std::get<1>(kv.first);
    g.kc1 = std::get<2>(kv.first);
    g.n = (long long)v.size();
    for (auto& pr : v) {
      g.h_items.push_back(pr.first);
      g.h_cell.push_back(pr.second);
    }
    g.items = upload(p, g.h_items, &st);
    g.cell = upload(p, g.h_cell, &st);
    g.counter = (unsigned*)dalloc(p, sizeof(unsigned));
    if (!g.counter && st == SQ_OK) st = fail(p, SQ_E_ALLOC, "device allocation failed");
    default_tiles(p, g);
    S.groups.push_back(std::move(g));
  }
  return st;
}

RecLaunch rec_launch(const Group& g, int fam) {
  const Tile& t = g.tile[fam];
  RecLaunch R;
  R.nc = g.nc;
  R.kc = t.kc ? t.kc : g.kc1;
  R.fused = g.fused;
  R.counter = t.persistent ? g.counter : nullptr;
  R.grid = 0;   // persistent: the launcher sizes the grid to the resident capacity
  return R;
}

void phase_begin(sq_plan p, Phase ph, hipStream_t s) {
  if (p->recording && p->ev0[ph] && hipEventRecord(p->ev0[ph], s) == hipSuccess) p->ev_open[ph] = true;
}

void phase_end(sq_plan p, Phase ph, hipStream_t s) {
  if (p->recording && p->ev_open[ph]) (void)hipEventRecord(p->ev1[ph], s);
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

// The device copy of the cell table must equal the uploaded one (checked
// once, at the end of set-up).
sq_status verify_cells(sq_plan p, const char* where) {
  std::vector<CellDev> back(p->host_cells.size());
  hipError_t e = hipMemcpyAsync(back.data(), p->d_cells, sizeof(CellDev) * back.size(),
                                hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return check_hip(p, e, where);
  if (std::memcmp(back.data(), p->host_cells.data(), sizeof(CellDev) * back.size()) != 0)
    return fail(p, SQ_E_DEVICE, std::string(where) + ": device cell table differs from the uploaded one");
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

sq_status error_status(sq_plan p, unsigned h) {
  if (h & SQ_ERR_IMAGES) return fail(p, SQ_E_ARG, "more atom images reach a cube than supported");
  if (h & SQ_ERR_SLOTS) return fail(p, SQ_E_ARG, "more atom images cross a cube column than supported");
  if (h & SQ_ERR_NEAR) return fail(p, SQ_E_ARG, "more projectors are nonzero at one node than supported");
  if (h & SQ_ERR_RANGE)
    return fail(p, SQ_E_BOUNDS, "a projection left the range of the fixed-point sums (|<chi, v>| >= 2^20)");
  if (h & SQ_ERR_BOUNDS) return fail(p, SQ_E_BOUNDS, "a Chebyshev moment left [-1, 1]: spectral bounds too narrow");
  return SQ_OK;
}

sq_status check_errors(sq_plan p) {
  unsigned h = 0;
  hipError_t e = hipMemcpyAsync(&h, p->P.err, sizeof(unsigned), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return check_hip(p, e, "device");
  return error_status(p, h);
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

// ---- launch sequences (eager on the plan's stream, or captured) -----------

sq_status enqueue_mu_rounds(sq_plan p, Selection* S, int rounds, hipStream_t s) {
  const int nc = (int)S->cells.size();
  sq_status st = SQ_OK;
  for (int k = 0; k < rounds && st == SQ_OK; ++k) {
    st = check_hip(p, sq_launch_mu_eval(p->P, S->items, S->item_cell, S->nall, s), "mu eval");
    if (st == SQ_OK) st = check_hip(p, sq_launch_mu_step(p->P, S->d_cells, nc, s), "mu step");
  }
  return st;
}

// Bounds, moments, the Fermi level within its budget, coefficients and
// density: no host interaction.  The moments come from the Lanczos
// tridiagonal when the plan runs enough Lanczos steps (qmom), else from the
// recurrence pass on the cube.
sq_status enqueue_density(sq_plan p, Selection* S, hipStream_t s) {
  const bool fp64 = p->opt.precision != SQ_MIXED;   // precision of the moments pass
  sq_status st = check_hip(p, sq_launch_fill_u32(p->P.err, 0u, 1, s), "clear");
  phase_begin(p, PH_LANCZOS, s);
  for (const Group& g : S->groups)
    if (st == SQ_OK)
      st = check_hip(p, sq_launch_lanczos(rec_launch(g, F_LAN), p->P, g.items, g.cell, g.n, s), "lanczos");
  phase_end(p, PH_LANCZOS, s);
  phase_begin(p, PH_BOUNDS, s);
  if (st == SQ_OK) st = check_hip(p, sq_launch_bounds(p->P, S->items, S->item_cell, S->nall, s), "bounds");
  phase_end(p, PH_BOUNDS, s);
  phase_begin(p, PH_MOMENTS, s);
  if (p->qmom) {
    if (st == SQ_OK)
      st = check_hip(p, sq_launch_qmoments(p->P, S->items, S->item_cell, S->nall, s), "moments");
  } else {
    for (const Group& g : S->groups)
      if (st == SQ_OK)
        st = check_hip(p, sq_launch_moments(rec_launch(g, F_MOM), fp64, p->P, g.items, g.cell, g.n, s),
                       "moments");
  }
  phase_end(p, PH_MOMENTS, s);
  phase_begin(p, PH_MU, s);
  if (st == SQ_OK)
    st = check_hip(p, sq_launch_mu_init(p->P, S->d_cells, (int)S->cells.size(), S->d_fixed, s), "mu init");
  if (st == SQ_OK) st = enqueue_mu_rounds(p, S, SQ_MU_BUDGET, s);
  phase_end(p, PH_MU, s);
  phase_begin(p, PH_COEFFS, s);
  if (st == SQ_OK) st = check_hip(p, sq_launch_coeffs(p->P, S->items, S->item_cell, S->nall, s), "coeffs");
  phase_end(p, PH_COEFFS, s);
  return st;
}

// Density-matrix columns, their gradients, K and N per node, the nonlocal
// energy per node, and the node sums of those columns.
sq_status enqueue_stress(sq_plan p, Selection* S, hipStream_t s, double* sums = nullptr) {
  const bool fp64 = p->opt.precision == SQ_FP64;
  sq_status st = check_hip(p, sq_launch_fill_u32(p->P.err, 0u, 1, s), "clear");
  phase_begin(p, PH_STRESS, s);
  for (const Group& g : S->groups)
    if (st == SQ_OK)
      st = check_hip(p, sq_launch_stress(rec_launch(g, F_STR), fp64, p->P, g.items, g.cell, g.n, s),
                     "stress");
  phase_end(p, PH_STRESS, s);
  phase_begin(p, PH_REDUCE, s);
  PlanDev Pr = p->P;
  if (sums) Pr.sums = sums;   // the reduction's target (default: the plan's sums)
  if (st == SQ_OK)
    st = check_hip(p, sq_launch_reduce(Pr, S->d_cells, (int)S->cells.size(), 2, 19, s), "reduce");
  phase_end(p, PH_REDUCE, s);
  return st;
}

// Runs one of the two sequences: eagerly on the plan's stream, or (use_graph)
// by replaying its graph, captured on the private stream at the first call.
sq_status run_sequence(sq_plan p, Selection* S, int which) {
  auto enq = [&](hipStream_t s) { return which == 0 ? enqueue_density(p, S, s) : enqueue_stress(p, S, s); };
  if (!p->opt.use_graph) return enq(p->stream);
  if (!S->exec[which]) {
    p->recording = false;
    sq_status st = check_hip(p, hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal), "capture");
    if (st == SQ_OK) {
      const sq_status se = enq(p->cap);
      hipGraph_t graph = nullptr;
      const hipError_t ee = hipStreamEndCapture(p->cap, &graph);
      st = se != SQ_OK ? se : check_hip(p, ee, "end capture");
      if (st == SQ_OK && !graph) st = fail(p, SQ_E_DEVICE, "empty graph");
      if (st == SQ_OK) {
        hipGraphExec_t exec = nullptr;
        st = check_hip(p, hipGraphInstantiateWithFlags(&exec, graph, 0), "graph instantiate");
        if (st == SQ_OK) {
          S->graph[which] = graph;
          S->exec[which] = exec;
        } else {
          (void)hipGraphDestroy(graph);
        }
      } else if (graph) {
        (void)hipGraphDestroy(graph);
      }
    }
    p->recording = true;
    if (st != SQ_OK) return st;
  }
  return check_hip(p, hipGraphLaunch(S->exec[which], p->stream), "graph launch");
}

// The stress pass over a selection; marks the cells' stress as done.
sq_status stress_pass(sq_plan p, Selection* S, std::vector<double>& sums) {
  for (int ci : S->cells)
    if (!p->density_done[ci]) return fail(p, SQ_E_STATE, "sq_stress / sq_pressure before sq_density");
  sq_status st = run_sequence(p, S, 1);
  if (st == SQ_OK) st = check_errors(p);
  phase_collect(p);
  if (st == SQ_OK) st = read_sums(p, sums);
  if (st == SQ_OK)
    for (int ci : S->cells) p->stress_done[ci] = 1;
  return st;
}

// ---- autotuner ---------------------------------------------------------------

// Tiny JSON reader/writer for the tune cache: one object of
// "key": [slot_capacity, persistent] entries.
void tune_read(sq_plan p, const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, k);
  std::fclose(f);
  size_t pos = 0;
  while ((pos = text.find('"', pos)) != std::string::npos) {
    const size_t end = text.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string key = text.substr(pos + 1, end - pos - 1);
    const size_t lb = text.find('[', end), rb = text.find(']', end);
    if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
    int kc = 0, per = 0;
    if (std::sscanf(text.c_str() + lb + 1, "%d , %d", &kc, &per) == 2 && (kc == 16 || kc == 24 || kc == 48) &&
        (per == 0 || per == 1)) {
      Tile t;
      t.kc = kc;
      t.persistent = per;
      p->tuned[key] = t;
    }
    pos = rb + 1;
  }
}

void tune_write(sq_plan p, const char* path) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : p->tuned)
    std::fprintf(f, "  \"%s\": [%d, %d]%s\n", kv.first.c_str(), kv.second.kc, kv.second.persistent,
                 ++i < p->tuned.size() ? "," : "");
  std::fprintf(f, "}\n");
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}

// Device time (ms) of one launch of family fam with tile t on the sample.
sq_status time_tile(sq_plan p, const Group& g, int fam, const Tile& t, const long long* items,
                    const int* cells, long long n, float* ms) {
  Group gg;
  gg.nc = g.nc;
  gg.fused = g.fused;
  gg.kc1 = g.kc1;
  gg.counter = g.counter;
  gg.tile[fam] = t;
  const RecLaunch R = rec_launch(gg, fam);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  sq_status st = check_hip(p, hipEventCreate(&e0), "event");
  if (st == SQ_OK) st = check_hip(p, hipEventCreate(&e1), "event");
  float best = 1e30f;
  for (int rep = 0; rep < 2 && st == SQ_OK; ++rep) {
    st = check_hip(p, hipEventRecord(e0, p->stream), "event");
    hipError_t e = hipSuccess;
    if (fam == F_LAN) e = sq_launch_lanczos(R, p->P, items, cells, n, p->stream);
    else if (fam == F_MOM) e = sq_launch_moments(R, p->opt.precision != SQ_MIXED, p->P, items, cells, n, p->stream);
    else e = sq_launch_stress(R, p->opt.precision == SQ_FP64, p->P, items, cells, n, p->stream);
    if (st == SQ_OK) st = check_hip(p, e, "tune launch");
    if (st == SQ_OK) st = check_hip(p, hipEventRecord(e1, p->stream), "event");
    if (st == SQ_OK) st = check_hip(p, hipEventSynchronize(e1), "event");
    float v = 0.f;
    if (st == SQ_OK) st = check_hip(p, hipEventElapsedTime(&v, e0, e1), "event");
    if (st == SQ_OK) best = std::min(best, v);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  *ms = best;
  return st;
}

// Picks, per group of the whole-plan selection and kernel family, the
// fastest variant (slot capacity 16 or 24 with the plane-0 weights in
// registers, or 48 recomputing them; persistent or one workgroup per node) on a sample
// of the group's nodes (its first nodes: the
// longest).  The sample's bounds come from the tuned Lanczos, and its
// coefficients are zero for the stress timing (the operation count does not
// depend on them).  Every selection's groups then take the choices.
sq_status autotune(sq_plan p) {
  sq_status st = SQ_OK;
  bool dirty = false;
  for (Group& g : p->all.groups) {
    bool all_known = true;
    for (int f = 0; f < F_N; ++f)
      all_known = all_known && ((f == F_MOM && p->qmom) || p->tuned.count(tune_key(p, g, f)) > 0);
    if (all_known) continue;
    const long long n = std::min<long long>(g.n, 2048);
    std::vector<Tile> cand;
    for (int kc : {16, 24, 48})
      for (int per = 0; per <= 1; ++per) {
        Tile t;
        t.kc = kc;
        t.persistent = per;
        if (tile_ok(g, t)) cand.push_back(t);
      }
    if (cand.size() < 2) continue;   // nothing to choose
    for (int f = 0; f < F_N && st == SQ_OK; ++f) {
      if (f == F_MOM && p->qmom) continue;   // no recurrence pass for the moments
      if (f == F_STR)
        st = check_hip(p, sq_launch_fill_u32((unsigned*)p->P.coef, 0u,
                                             (long long)(2 * p->P.mstride) * p->Ntot, p->stream), "clear");
      float best = 1e30f;
      Tile bt = cand[0];
      for (const Tile& t : cand) {
        float ms = 0.f;
        if (st == SQ_OK) st = time_tile(p, g, f, t, g.items, g.cell, n, &ms);
        if (st == SQ_OK && ms < best) {
          best = ms;
          bt = t;
        }
      }
      if (st != SQ_OK) break;
      p->tuned[tune_key(p, g, f)] = bt;
      dirty = true;
      if (f == F_LAN) {   // bounds of the sample for the moments and stress timings
        Tile keep = g.tile[F_LAN];
        g.tile[F_LAN] = bt;
        st = check_hip(p, sq_launch_lanczos(rec_launch(g, F_LAN), p->P, g.items, g.cell, n, p->stream),
                       "tune lanczos");
        g.tile[F_LAN] = keep;
        if (st == SQ_OK) st = check_hip(p, sq_launch_bounds(p->P, g.items, g.cell, n, p->stream), "tune bounds");
      }
    }
  }
  if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(p->stream), "tune");
  if (st == SQ_OK) st = check_hip(p, sq_launch_fill_u32(p->P.err, 0u, 1, p->stream), "clear");
  if (st == SQ_OK && dirty && p->opt.tune_cache) tune_write(p, p->opt.tune_cache);
  if (st == SQ_OK) {
    for (Group& g : p->all.groups) default_tiles(p, g);
    for (Selection& S : p->per_cell)
      for (Group& g : S.groups) default_tiles(p, g);
  }
  return st;
}

}  // namespace

namespace {
// sigma (Voigt) and the K, N node sums of the selected cells from the
// reduced records (rows of SQ_REC + 4 per plan cell)
sq_status stress_outputs(sq_plan p, const Selection* S, const double* sums, double* sigma_voigt,
                         double* parts) {
  sq_status st = SQ_OK;
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
  auto drop = [](Selection& S) {
    for (int w = 0; w < 2; ++w) {
      if (S.exec[w]) (void)hipGraphExecDestroy(S.exec[w]);
      if (S.graph[w]) (void)hipGraphDestroy(S.graph[w]);
      S.exec[w] = nullptr;
      S.graph[w] = nullptr;
    }
  };
  drop(plan->all);
  for (Selection& S : plan->per_cell) drop(S);
  if (plan->cap) (void)hipStreamDestroy(plan->cap);
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
  Range range_("sq_setup");
  if (!out) return fail(nullptr, SQ_E_ARG, "out is NULL");
  *out = nullptr;
  if (!cells || n_cells < 1 || !opt) return fail(nullptr, SQ_E_ARG, "cells / options missing");
  if (opt->precision != SQ_FP64 && opt->precision != SQ_MIXED && opt->precision != SQ_MIXED_STRESS)
    return fail(nullptr, SQ_E_ARG, "unknown precision");
  if (opt->cheb_quad_points != 0 &&
      (opt->cheb_quad_points < 4 || (opt->cheb_quad_points & (opt->cheb_quad_points - 1)) != 0))
    return fail(nullptr, SQ_E_ARG, "cheb_quad_points must be 0 or a power of two");
  if (opt->inject & ~(SQ_INJECT_NARROW | SQ_INJECT_MU_CAP)) return fail(nullptr, SQ_E_ARG, "unknown inject bits");
  sq_plan p = new sq_plan_s();
  p->opt = *opt;
  p->stream = (hipStream_t)opt->hip_stream;
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      p->arch = prop.gcnArchName;
    const std::string::size_type c = p->arch.find(':');
    if (c != std::string::npos) p->arch = p->arch.substr(0, c);
  }
  if (opt->tune_cache) tune_read(p, opt->tune_cache);
  sq_status st = SQ_OK;
  p->cells.resize(n_cells);
  int npl_max = 1;
  for (int i = 0; i < n_cells; ++i) {
    st = build_cell(p, cells[i], p->cells[i], i);
    if (st == SQ_OK && opt->cheb_quad_points && opt->cheb_quad_points < 4 * (p->cells[i].npl + 2))
      st = fail(p, SQ_E_ARG, "cell " + std::to_string(i) + ": cheb_quad_points below 4 (npl + 2)");
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
  p->qmom = true;
  for (const CellHost& c : p->cells) p->qmom = p->qmom && qmom_steps(c) <= SQ_KL_MAX - 1;
  P.mstride = npl_max + 2;
  P.inject = opt->inject;
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
    if (!c.d_vloc) st = fail(p, SQ_E_ALLOC, "device allocation failed");
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
    d.krun = p->qmom ? qmom_steps(c) : c.K;
    d.nimg = (int)(c.img.size() / 4);
    d.nsp = (int)c.sp.size();
    d.mq = opt->cheb_quad_points;
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
  for (int i = 0; i < n_cells && st == SQ_OK; ++i)
    st = check_hip(p, sq_launch_vloc(p->d_cells + i, hc[i], p->cells[i].d_vloc, p->stream), "vloc");
  // capacity census: images per cube, per z-column, per half column and at
  // the node itself
  std::vector<int> all(n_cells);
  for (int i = 0; i < n_cells; ++i) all[i] = i;
  if (st == SQ_OK) {
    Selection pre;
    st = make_selection(p, all, pre);
    int* d_stats = (int*)A(sizeof(int) * SQ_CENSUS * n_cells);
    long long* d_pairs = (long long*)A(sizeof(long long) * n_cells);
    if (st == SQ_OK && (!d_stats || !d_pairs)) st = fail(p, SQ_E_ALLOC, "device allocation failed");
    if (st == SQ_OK) st = check_hip(p, hipMemsetAsync(d_stats, 0, sizeof(int) * SQ_CENSUS * n_cells, p->stream), "memset");
    if (st == SQ_OK) st = check_hip(p, hipMemsetAsync(d_pairs, 0, sizeof(long long) * n_cells, p->stream), "memset");
    if (st == SQ_OK) st = check_hip(p, hipMemsetAsync(P.err, 0, sizeof(unsigned), p->stream), "memset");
    for (const Group& g : pre.groups)
      if (st == SQ_OK)
        st = check_hip(p, sq_launch_census(g.nc, P, g.items, g.cell, g.n, d_stats, d_pairs, p->stream), "census");
    std::vector<int> stats(SQ_CENSUS * n_cells);
    std::vector<long long> pairs(n_cells);
    if (st == SQ_OK)
      st = check_hip(p, hipMemcpyAsync(stats.data(), d_stats, sizeof(int) * stats.size(),
                                       hipMemcpyDeviceToHost, p->stream), "census copy");
    if (st == SQ_OK)
      st = check_hip(p, hipMemcpyAsync(pairs.data(), d_pairs, sizeof(long long) * pairs.size(),
                                       hipMemcpyDeviceToHost, p->stream), "census copy");
    if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(p->stream), "census");
    for (int i = 0; i < n_cells && st == SQ_OK; ++i) {
      CellHost& c = p->cells[i];
      c.census_img = stats[SQ_CENSUS * i];
      c.census_col = std::max(1, stats[SQ_CENSUS * i + 1]);
      c.census_near = stats[SQ_CENSUS * i + 2];
      c.census_pairs = pairs[i];
      const std::string tag = "cell " + std::to_string(i) + ": ";
      const int kc_lim = 48;   // widest slot capacity (one thread per column)
      const int img_lim = sq_img_limit(c.nc);
      if (c.census_img > img_lim)
        st = fail(p, SQ_E_ARG, tag + std::to_string(c.census_img) +
                                   " atom images reach one cube (at most " +
                                   std::to_string(img_lim) + " supported)");
      else if (c.census_col > kc_lim)
        st = fail(p, SQ_E_ARG, tag + std::to_string(c.census_col) +
                                   " atom images cross one cube column (at most " +
                                   std::to_string(kc_lim) + " supported)");
      else if (c.census_near > SQ_NEAR_MAX)
        st = fail(p, SQ_E_ARG, tag + "more than 32 projectors are nonzero at one node");
    }
  }
  // Gram matrices of every node's projectors (geometry only), then the node
  // groups, split by whether a node's Gram matrix fits
  if (st == SQ_OK) {
    Selection pre;
    st = make_selection(p, all, pre);
    for (const Group& g : pre.groups)
      if (st == SQ_OK) st = check_hip(p, sq_launch_gram(g.nc, P, g.items, g.cell, g.n, p->stream), "gram");
    std::vector<int> gn(N);
    if (st == SQ_OK)
      st = check_hip(p, hipMemcpyAsync(gn.data(), P.gn, sizeof(int) * N, hipMemcpyDeviceToHost, p->stream),
                     "gram copy");
    if (st == SQ_OK) st = check_errors(p);
    for (int i = 0; i < n_cells && st == SQ_OK; ++i) {
      CellHost& c = p->cells[i];
      for (long long q = 0; q < c.Nd; ++q) {
        const int k = gn[c.node_base + q];
        if (k >= 0) {
          c.gram_entries += k;
          c.gram_nodes += 1;
        }
      }
    }
    if (st == SQ_OK) st = make_selection(p, all, p->all, &gn);
    p->per_cell.resize(n_cells);
    for (int i = 0; i < n_cells && st == SQ_OK; ++i) st = make_selection(p, {i}, p->per_cell[i], &gn);
  }
  if (st == SQ_OK && opt->use_graph)
    st = check_hip(p, hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking), "capture stream");
  if (st == SQ_OK && opt->autotune) st = autotune(p);
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
  // the library's static scratch on this device (sq_stress_static)
  if (n_cells <= SQ_STATIC_CELLS) {
    st = check_hip(p, sq_static_scratch(&p->static_sums), "static scratch");
    if (st != SQ_OK) {
      g_setup_err = p->err;
      sq_destroy(p);
      return st;
    }
    p->host_sums.assign((size_t)(SQ_REC + 4) * n_cells, 0.0);
  }
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
    const int ns = std::min(steps[nodes[i]], K);   // the steps the bounds use
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
  info[9] = c.K;
  info[10] = c.gram_entries;
  info[11] = c.gram_nodes;
  info[12] = p->qmom ? qmom_steps(c) : c.K;
  info[13] = p->qmom ? 1 : 0;
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
  Range range_("sq_density");
  if (!p) return SQ_E_ARG;
  Selection* S = nullptr;
  sq_status st = select(p, cell, &S);
  if (st != SQ_OK) return st;
  hipStream_t s = p->stream;
  st = run_sequence(p, S, 0);
  if (st != SQ_OK) return st;
  // one synchronisation: error flags and the search state of every cell
  std::vector<double> mus(SQ_MU_STRIDE * p->cells.size());
  unsigned eflags = 0;
  st = check_hip(p, hipMemcpyAsync(mus.data(), p->P.mus, sizeof(double) * mus.size(),
                                   hipMemcpyDeviceToHost, s), "mu copy");
  if (st == SQ_OK)
    st = check_hip(p, hipMemcpyAsync(&eflags, p->P.err, sizeof(unsigned), hipMemcpyDeviceToHost, s), "flags");
  if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(s), "density");
  phase_collect(p);
  if (st != SQ_OK) return st;
  st = error_status(p, eflags);
  if (st != SQ_OK) return st;
  auto running = [&]() {
    for (int ci : S->cells)
      if (mus[SQ_MU_STRIDE * ci + MU_DONE] == 0.0) return true;
    return false;
  };
  // a search still running after the budget: more rounds, then the
  // coefficients again
  if (running()) {
    for (int done_it = SQ_MU_BUDGET; done_it < SQ_MU_MAX && running() && st == SQ_OK; done_it += SQ_MU_MORE) {
      st = enqueue_mu_rounds(p, S, SQ_MU_MORE, s);
      if (st == SQ_OK)
        st = check_hip(p, hipMemcpyAsync(mus.data(), p->P.mus, sizeof(double) * mus.size(),
                                         hipMemcpyDeviceToHost, s), "mu copy");
      if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(s), "mu sync");
    }
    if (st == SQ_OK && !running())
      st = check_hip(p, sq_launch_coeffs(p->P, S->items, S->item_cell, S->nall, s), "coeffs");
    if (st != SQ_OK) return st;
  }
  for (int ci : S->cells) {
    const double d = mus[SQ_MU_STRIDE * ci + MU_DONE];
    if (d == 2.0) return fail(p, SQ_E_NOCONV, "cell " + std::to_string(ci) + ": N_e not bracketed");
    if (d == 0.0)
      return fail(p, SQ_E_NOCONV, "cell " + std::to_string(ci) + ": Fermi-level search did not finish");
    if (d == 3.0)
      return fail(p, SQ_E_NOCONV, "cell " + std::to_string(ci) +
                                      ": Fermi-level search reached its update cap without meeting |N - N_e| <= 1e-13 N_e");
  }
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
      if (st != SQ_OK) return st;
    }
  }
  if (rho || (mu && p->opt.outputs_on_device)) st = check_hip(p, hipStreamSynchronize(s), "density");
  if (st == SQ_OK)
    for (int ci : S->cells) {
      p->density_done[ci] = 1;
      p->stress_done[ci] = 0;
    }
  return st;
}

sq_status sq_energy(sq_plan p, int cell, double* e_band) {
  Range range_("sq_energy");
  if (!p) return SQ_E_ARG;
  Selection* S = nullptr;
  sq_status st = select(p, cell, &S);
  if (st != SQ_OK) return st;
  for (int ci : S->cells)
    if (!p->density_done[ci]) return fail(p, SQ_E_STATE, "sq_energy before sq_density");
  hipStream_t s = p->stream;
  phase_begin(p, PH_REDUCE, s);
  st = check_hip(p, sq_launch_reduce(p->P, S->d_cells, (int)S->cells.size(), 1, 1, s), "reduce");
  phase_end(p, PH_REDUCE, s);
  std::vector<double> sums;
  if (st == SQ_OK) st = read_sums(p, sums);
  phase_collect(p);
  if (st != SQ_OK || !e_band) return st;
  for (size_t i = 0; i < S->cells.size() && st == SQ_OK; ++i)
    st = put_out(p, e_band + i, &sums[(SQ_REC + 4) * S->cells[i] + 1], sizeof(double));
  return st;
}

sq_status sq_stress(sq_plan p, int cell, double* sigma_voigt, double* parts) {
  Range range_("sq_stress");
  if (!p) return SQ_E_ARG;
  Selection* S = nullptr;
  sq_status st = select(p, cell, &S);
  if (st != SQ_OK) return st;
  std::vector<double> sums;
  st = stress_pass(p, S, sums);
  if (st != SQ_OK) return st;
  return stress_outputs(p, S, sums.data(), sigma_voigt, parts);
}

sq_status sq_stress_static(sq_plan p, int cell, double* sigma_voigt, double* parts) {
  Range range_("sq_stress_static");
  if (!p) return SQ_E_ARG;
  if ((int)p->cells.size() > SQ_STATIC_CELLS)
    return fail(p, SQ_E_ARG, "sq_stress_static: the plan has " + std::to_string(p->cells.size()) +
                                 " cells; the static scratch holds " + std::to_string(SQ_STATIC_CELLS));
  if (!p->static_sums) return fail(p, SQ_E_DEVICE, "sq_stress_static: no static scratch on this device");
  Selection* S = nullptr;
  sq_status st = select(p, cell, &S);
  if (st != SQ_OK) return st;
  for (int ci : S->cells)
    if (!p->density_done[ci]) return fail(p, SQ_E_STATE, "sq_stress_static before sq_density");
  // always eager: a captured stress graph reduces into the plan's own sums.
  // The reduction writes every row it covers before it is read (nothing
  // needs clearing); rows of other cells keep an earlier call's contents
  // and are not read.
  st = enqueue_stress(p, S, p->stream, p->static_sums);
  if (st == SQ_OK) st = check_errors(p);
  phase_collect(p);
  if (st == SQ_OK)
    st = check_hip(p, hipMemcpyAsync(p->host_sums.data(), p->static_sums, sizeof(double) * p->host_sums.size(),
                                     hipMemcpyDeviceToHost, p->stream), "static sums");
  if (st == SQ_OK) st = check_hip(p, hipStreamSynchronize(p->stream), "static sums");
  if (st != SQ_OK) return st;
  // the plan's stress bookkeeping is left as it was: sq_pressure reads the
  // plan's own sums, which this call does not write
  return stress_outputs(p, S, p->host_sums.data(), sigma_voigt, parts);
}

sq_status sq_pressure(sq_plan p, int cell, double* p_direct, double* p_trace) {
  Range range_("sq_pressure");
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
  phase_begin(p, PH_REDUCE, s);
  if (st == SQ_OK)
    st = check_hip(p, sq_launch_reduce(p->P, S->d_cells, (int)S->cells.size(), 1, 1, s), "reduce");
  if (st == SQ_OK)
    st = check_hip(p, sq_launch_reduce(p->P, S->d_cells, (int)S->cells.size(), 21, 1, s), "reduce");
  phase_end(p, PH_REDUCE, s);
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
  Range range_("sq_xc");
  if (!p) return SQ_E_ARG;
  Selection* S = nullptr;
  sq_status st = select(p, cell, &S);
  if (st != SQ_OK) return st;
  for (int ci : S->cells)
    if (!p->density_done[ci]) return fail(p, SQ_E_STATE, "sq_xc before sq_density");
  hipStream_t s = p->stream;
  phase_begin(p, PH_REDUCE, s);
  st = check_hip(p, sq_launch_reduce(p->P, S->d_cells, (int)S->cells.size(), 22, 2, s), "reduce");
  phase_end(p, PH_REDUCE, s);
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
