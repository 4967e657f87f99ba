// sq_recur.hip -- gfx950 recurrence kernels of the infinite-cell
// Clenshaw-Curtis SQ hot path (arXiv 2006.03697, Sec. IV and App. A):
// spectral-bound Lanczos, Chebyshev moments, the stress pass, the projector
// Gram matrices and the capacity census.  Compiled once per cube width NC
// (SQ_ONE_NC).
//
// One workgroup owns one node q and its cube (region of influence) of
// NC^3 finite-difference nodes.  Thread (cx, cy) owns the z-column of the
// cube at (cx, cy): the current Chebyshev vector, the previous one and the
// diagonal of H_q on that column live in its registers; the current vector
// is mirrored in LDS so that x/y neighbours of the 12th-order stencil are
// LDS reads and z neighbours are register reads.  Atom-image projectors are
// separable Gaussians cut off at a sphere: per (column, image) the chord of
// the sphere on the column as a bit mask and the projector value at the
// column's first plane (registers, computed once per node); along the column
// the Gaussian factor follows from a two-multiply recurrence.  One sweep per
// operator application both adds the projector terms and takes the new
// projections (completed by the stored Gram matrix of the node's projectors).
#include "sq_devfn.h"

#ifndef SQ_ONE_NC
#error "sq_recur.hip is compiled once per cube width: define SQ_ONE_NC"
#endif

namespace {
// ---------------------------------------------------------------------------
// Cube layout in LDS and the thread <-> z-column map
//
// Thread (cx, cy) owns the z-column (cx, cy) of the cube: the current and
// previous Chebyshev vectors and the diagonal live in its registers, and the
// current vector is mirrored in LDS for the x and y neighbours of the
// stencil.  Padded layout: rows of RS >= NC + 6 elements (the tail zero) and
// planes of NC + 6 rows (the last 6 zero), after 6 zero rows and 6 zeros, so
// every neighbour outside the cube reads a zero and needs no predicate.
//
// LDS has 32 banks of 4 bytes: a 32-bit access by 32 lanes, or a 64-bit
// access by 16 lanes, is conflict-free when the element addresses are
// distinct modulo 32 (resp. 16).  With the padded row stride consecutive
// rows alias, so lanes are mapped to columns by address residue instead of
// row-major: lane 32 g + r owns the g-th column (in row-major order) whose
// row offset cy * RS + cx is congruent to r modulo 32.  Every access of a
// wave is then a constant shift of these offsets, hence conflict-free.  RS
// is the smallest stride for which no residue class has more columns than
// the block has 32-lane groups.
// ---------------------------------------------------------------------------
constexpr int sq_residue_max(int nc, int rs) {
  int cnt[32] = {};
  int mx = 0;
  for (int cy = 0; cy < nc; ++cy)
    for (int cx = 0; cx < nc; ++cx) {
      const int r = (cy * rs + cx) & 31;
      if (++cnt[r] > mx) mx = cnt[r];
    }
  return mx;
}

constexpr int sq_threads(int nc) { return ((nc * nc + 63) / 64) * 64; }

constexpr int sq_pick_rs(int nc) {
  for (int rs = nc + SQ_FDM; rs <= nc + SQ_FDM + 16; ++rs)
    if (sq_residue_max(nc, rs) * 32 <= sq_threads(nc)) return rs;
  return 0;
}

template <int NC, bool PAD>
struct Lay {
  static constexpr int NT = sq_threads(NC);
  static constexpr int NW = NT / 64;
  static constexpr int MH = NC / 2;
  static constexpr int RS = PAD ? sq_pick_rs(NC) : NC;              // row stride
  static constexpr int PL = PAD ? (NC + SQ_FDM) * RS : NC * NC;     // plane stride
  static constexpr int X0 = PAD ? SQ_FDM * RS + SQ_FDM : 0;         // offset of (0, 0, 0)
  static constexpr int SIZE = X0 + NC * PL;
  static_assert(!PAD || RS > 0, "no conflict-free row stride");
  __device__ static constexpr int at(int x, int y, int z) { return X0 + z * PL + y * RS + x; }

  // Column of thread tid (see above); inactive threads own no column.
  __device__ static void column(int tid, int& cx, int& cy, bool& active) {
    cx = 0;
    cy = 0;
    active = false;
    if constexpr (PAD) {
      const int r = tid & 31, g = tid >> 5;
      int seen = 0;
      for (int y = 0; y < NC; ++y) {
        const int x = (r - y * RS) & 31;   // the one column of row y with residue r
        if (x < NC) {
          if (seen == g) {
            cx = x;
            cy = y;
            active = true;
          }
          ++seen;
        }
      }
    } else {
      active = tid < NC * NC;
      cx = tid % NC;
      cy = tid / NC;
    }
  }
};

// A kernel variant: working precision T, cube width NC, KC projector slots
// per z-column, and whether each slot's weight on plane 0 is kept in a
// register (AREG) or recomputed at every use.  The padded LDS layout is used
// when the whole working set fits the 160 KiB of LDS.
template <typename T_, int NC_, int KC_, bool AREG_>
struct Var {
  using T = T_;
  static constexpr int NC = NC_;
  static constexpr int KC = KC_;
  static constexpr bool AREG = AREG_;
  // slot word: chord bits 31 .. 32 - NC, image index below
  static constexpr int IBITS = 32 - NC_;
  static constexpr int NIMG = (1 << IBITS) < 160 ? (1 << IBITS) : 160;
  static constexpr int NEAR = SQ_NEAR_MAX;
  static constexpr size_t OTHER = 8 * (size_t)NIMG * 11 + (size_t)NEAR * 11 * 8 + NEAR * 4 + 1024 +
                                  12 * (size_t)SQ_GRAM_MAX;
  // scratch of the Gram build (FP64 Lanczos pass only), in the cube buffer:
  // pair bitmap [NIMG][NWD], row starts [NIMG + 1], slot words [KC][NT]
  static constexpr int NWD = (NIMG + 31) / 32;
  static constexpr size_t GSCR = 4 * ((size_t)NIMG * NWD + NIMG + 1 + (size_t)KC * sq_threads(NC_));
#ifdef SQ_NO_PAD
  static constexpr bool PAD = false;
#else
  static constexpr bool PAD = sizeof(T_) * (size_t)Lay<NC_, true>::SIZE + OTHER <= 163840;
#endif
  using L = Lay<NC_, PAD>;
  // elements of the cube buffer: the padded or plain cube, or the Gram scratch
  static constexpr size_t TLN = (sizeof(T_) == 8 && (GSCR + 7) / 8 > (size_t)L::SIZE) ? (GSCR + 7) / 8
                                                                                   : (size_t)L::SIZE;
};

template <class Vr>
struct Smem {
  using T = typename Vr::T;
  static constexpr int NI = Vr::NIMG;
  T tl[Vr::TLN];
  double ix[NI], iy[NI], iz[NI];      // image positions (unwrapped)
  double rp2[NI], i2s[NI], gdv[NI];   // r_p^2, 1 / (2 sigma_p^2), gamma dV
  // z factor of each image on the cube planes: e(z) = exp(-u_z^2 i2s) with
  // u_z = u_0 + z h, generated as e(z + 1) = e(z) rr(z), rr(z + 1) = rr(z) cq
  double e0[NI], r0[NI], cq[NI];
  double pacc[2][NI];                 // projections, double-buffered over steps
  // Gram matrix <chi_I, chi_J> over the cube for I <= J with overlapping
  // supports: value and I | J << 16, ngram entries in (I, J) order
  double gval[SQ_GRAM_MAX];
  unsigned gidx[SQ_GRAM_MAX];
  int ngram;
  double red[2][2 * 16];              // block sums, double-buffered over steps
  double near_chi[Vr::NEAR];
  double nsum[Vr::NEAR][10];
  int near_img[Vr::NEAR];
  int wcnt[16];
  int nimg, nnear;
};

// Per-thread node context (registers).
template <class Vr>
struct Ctx {
  using T = typename Vr::T;
  int cx, cy, col;
  bool active;
  long long q0, q1, q2;
  int nslot;    // slots of this column
  int nsw;      // largest slot count in the wave (wave-uniform)
  // slot s: bit 31 - z set for the planes z of the chord of the image's
  // spherical support on this column; the image index in the low bits
  unsigned sid[Vr::KC];
  double a0[Vr::AREG ? Vr::KC : 1];   // projector value of slot s at (cx, cy, plane 0)
  T vd[Vr::NC];                       // diagonal of (H_q - shift) without the stencil centre
};

template <class Vr>
__device__ __forceinline__ double slot_start(const Smem<Vr>& S, const Ctx<Vr>& X, const CellDev& C,
                                             int s, int i) {
  if constexpr (Vr::AREG) {
    return X.a0[s];
  } else {
    constexpr int m = Vr::NC / 2;
    const double dx = node_coord(X.q0 + X.cx - m, C.h, S.ix[i]);
    const double dy = node_coord(X.q1 + X.cy - m, C.h, S.iy[i]);
    return exp(-sq_sum2(dx, dy) * S.i2s[i]) * S.e0[i];
  }
}

// Image list of the node's cube: the tile list filtered by distance to the
// cube's box, in tile-list order (deterministic).  Returns the count.
template <int NT, int NW, int CAP, class Store>
__device__ __forceinline__ int gather_images(const CellDev& C, long long q0, long long q1,
                                             long long q2, int m, int* cnt_lds, int* wcnt,
                                             Store store, unsigned* err) {
  const int tid = threadIdx.x;
  const double h = C.h;
  const int tx = (int)(q0 / SQ_TILE), ty = (int)(q1 / SQ_TILE), tz = (int)(q2 / SQ_TILE);
  const int tile = tx + C.ntile[0] * (ty + C.ntile[1] * tz);
  const int t0 = C.tile_ptr[tile], t1 = C.tile_ptr[tile + 1];
  if (tid == 0) *cnt_lds = 0;
  __syncthreads();
  const double lo0 = (double)(q0 - m) * h, hi0 = (double)(q0 + m) * h;
  const double lo1 = (double)(q1 - m) * h, hi1 = (double)(q1 + m) * h;
  const double lo2 = (double)(q2 - m) * h, hi2 = (double)(q2 + m) * h;
  int total = 0;
  for (int base = t0; base < t1; base += NT) {
    const int k = base + tid;
    bool pass = false;
    int I = 0;
    if (k < t1) {
      I = C.tile_img[k];
      const double R0 = C.img[4 * I], R1 = C.img[4 * I + 1], R2 = C.img[4 * I + 2];
      const int sp = (int)C.img[4 * I + 3];
      const double e0 = R0 < lo0 ? lo0 - R0 : (R0 > hi0 ? R0 - hi0 : 0.0);
      const double e1 = R1 < lo1 ? lo1 - R1 : (R1 > hi1 ? R1 - hi1 : 0.0);
      const double e2 = R2 < lo2 ? lo2 - R2 : (R2 > hi2 ? R2 - hi2 : 0.0);
      const double rp = C.sp[sp].p_rc;
      // conservative: an image that is kept but reaches no node adds zero
      pass = e0 * e0 + e1 * e1 + e2 * e2 < rp * rp * (1.0 + 1e-9) + 1e-12;
    }
    const unsigned long long mask = __ballot(pass);
    const int lane = tid & 63, w = tid >> 6;
    const int pre = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[w] = __popcll(mask);
    __syncthreads();
    int off = *cnt_lds;
    int chunk = 0;
    for (int i = 0; i < NW; ++i) {
      if (i < w) off += wcnt[i];
      chunk += wcnt[i];
    }
    if (pass) {
      const int pos = off + pre;
      if (pos < CAP) store(pos, I);
      else atomicOr(err, SQ_ERR_IMAGES);
    }
    __syncthreads();
    if (tid == 0) *cnt_lds += chunk;
    total += chunk;
    __syncthreads();
  }
  return total;   // may exceed CAP (then only CAP were stored and err is set)
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return __builtin_amdgcn_readfirstlane(v);
}

// Node prologue: image list of the cube, z-factor constants, per-column
// chords and projector weights, diagonal.  shift is subtracted from the
// diagonal.
template <class Vr>
__device__ __forceinline__ void node_prologue(const CellDev& C, long long q, double shift,
                                              Smem<Vr>& S, Ctx<Vr>& X, unsigned* err) {
  using T = typename Vr::T;
  using L = typename Vr::L;
  constexpr int NC = Vr::NC;
  constexpr int m = L::MH;
  const int tid = threadIdx.x;
  L::column(tid, X.cx, X.cy, X.active);
  X.col = X.cx + NC * X.cy;
  X.q0 = q % C.n[0];
  X.q1 = (q / C.n[0]) % C.n[1];
  X.q2 = q / ((long long)C.n[0] * C.n[1]);
  const double h = C.h;

  // ---- images whose projector may reach this cube ----
  auto store = [&](int pos, int I) {
    const SpecDev& s = C.sp[(int)C.img[4 * I + 3]];
    S.ix[pos] = C.img[4 * I];
    S.iy[pos] = C.img[4 * I + 1];
    S.iz[pos] = C.img[4 * I + 2];
    S.rp2[pos] = s.p_rc * s.p_rc;
    S.i2s[pos] = 1.0 / (2.0 * s.p_sig * s.p_sig);
    S.gdv[pos] = s.gamma * C.dV;
  };
  const int found = gather_images<L::NT, L::NW, Vr::NIMG>(C, X.q0, X.q1, X.q2, m, &S.nimg,
                                                           S.wcnt, store, err);
  const int nimg = found < Vr::NIMG ? found : Vr::NIMG;
  if (tid == 0) S.nimg = nimg;

  // ---- z-factor constants of every image; projection accumulators ----
  for (int i = tid; i < Vr::NIMG; i += L::NT) {
    double e0 = 0.0, r0 = 0.0, cq = 0.0;
    if (i < nimg) {
      const double u0 = node_coord(X.q2 - m, h, S.iz[i]);
      const double is = S.i2s[i];
      e0 = exp(-(u0 * u0) * is);
      r0 = exp(-(2.0 * u0 * h + h * h) * is);
      cq = exp(-2.0 * h * h * is);
    }
    S.e0[i] = e0;
    S.r0[i] = r0;
    S.cq[i] = cq;
    S.pacc[0][i] = 0.0;
    S.pacc[1][i] = 0.0;
  }
  for (int i = tid; i < L::SIZE; i += L::NT) S.tl[i] = (T)0;
  if (tid == 0) S.nnear = 0;
  __syncthreads();

  // ---- per-column chords of every image's spherical support ----
  X.nslot = 0;
#pragma unroll
  for (int s = 0; s < Vr::KC; ++s) X.sid[s] = 0u;
  if constexpr (Vr::AREG) {
#pragma unroll
    for (int s = 0; s < Vr::KC; ++s) X.a0[s] = 0.0;
  }
  if (X.active) {
    for (int i = 0; i < nimg; ++i) {
      const double dx = node_coord(X.q0 + X.cx - m, h, S.ix[i]);
      const double dy = node_coord(X.q1 + X.cy - m, h, S.iy[i]);
      const double dxy2 = sq_sum2(dx, dy);
      const double rp2 = S.rp2[i];
      if (!(dxy2 < rp2)) continue;
      unsigned bits = 0u;
      for (int z = 0; z < NC; ++z) {
        const double dz = node_coord(X.q2 + z - m, h, S.iz[i]);
        if (sq_add(dxy2, dz) < rp2) bits |= 0x80000000u >> z;
      }
      if (bits == 0u) continue;
      if (X.nslot >= Vr::KC) {
        atomicOr(err, SQ_ERR_SLOTS);
        continue;
      }
      const unsigned word = bits | (unsigned)i;
#pragma unroll
      for (int s = 0; s < Vr::KC; ++s) {
        if (s == X.nslot) {
          X.sid[s] = word;
          if constexpr (Vr::AREG) X.a0[s] = exp(-dxy2 * S.i2s[i]) * S.e0[i];
        }
      }
      ++X.nslot;
    }
  }
  X.nsw = wave_max(X.nslot);

  // ---- diagonal: local potential (periodic) + stencil centre - shift ----
  const double cdiag = -0.5 / (h * h) * 3.0 * C.c2[0];
  const long long ix = wrapll(X.q0 + X.cx - m, C.n[0]);
  const long long iy = wrapll(X.q1 + X.cy - m, C.n[1]);
#pragma unroll
  for (int z = 0; z < NC; ++z) {
    double v = 0.0;
    if (X.active) {
      const long long iz = wrapll(X.q2 + z - m, C.n[2]);
      v = C.vloc[ix + (long long)C.n[0] * (iy + (long long)C.n[1] * iz)];
    }
    X.vd[z] = (T)(v + cdiag - shift);
  }
}

// Weight of a slot on one plane in the working precision: a on the chord,
// zero off it.  In FP64 only the high word is selected (one select instead of
// two): off the chord the weight is the subnormal made of a's low word, below
// 2^-1042 in magnitude, which changes no sum or product it enters by more
// than that (the vectors and projections it meets are of order one, the
// results are compared at 1e-10).
template <typename T>
__device__ __forceinline__ T chord_weight(bool on, double a);
template <>
__device__ __forceinline__ float chord_weight<float>(bool on, double a) {
  return on ? (float)a : 0.0f;
}
template <>
__device__ __forceinline__ double chord_weight<double>(bool on, double a) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(a);
  const unsigned long long hi = on ? (b >> 32) : 0ull;
  return __longlong_as_double((long long)((hi << 32) | (b & 0xffffffffull)));
}

// Projector weights of one slot along the column: w(z) = a e(z)/e(0) on the
// planes of the chord, zero elsewhere.  f(z, w) is called for every plane.
template <int NC, class F>
__device__ __forceinline__ void slot_sweep(unsigned mk, double a, double rr, double cq, F f) {
#pragma unroll
  for (int z = 0; z < NC; ++z) {
    unsigned nm;
    const bool on = __builtin_add_overflow(mk, mk, &nm);   // bit 31 - z
    mk = nm;
    const double an = a * rr;   // before the use: a's registers then hold the weight
    rr *= cq;
    f(z, on, a);
    a = an;
  }
}

// Projections <chi_I, v> of the vector v held in registers into S.pacc[buf]
// (the caller places a barrier before they are read).
template <class Vr>
__device__ __forceinline__ void project(Smem<Vr>& S, const Ctx<Vr>& X, const CellDev& C,
                                        const typename Vr::T (&v)[Vr::NC], int buf) {
  using T = typename Vr::T;
  constexpr int NC = Vr::NC;
  constexpr unsigned IMASK = (1u << Vr::IBITS) - 1u;
#pragma unroll
  for (int s = 0; s < Vr::KC; ++s) {
    if (s < X.nsw) {
      const unsigned mk = X.sid[s];
      const int i = (int)(mk & IMASK);
      T part = (T)0;
      slot_sweep<NC>(mk, slot_start<Vr>(S, X, C, s, i), S.r0[i], S.cq[i],
                     [&](int z, bool on, double a) { part += chord_weight<T>(on, a) * v[z]; });
      if (s < X.nslot) atomicAdd(&S.pacc[buf][i], (double)part);
    }
  }
}

// One application of the nodal operator to the vector held in registers
// (cur) and mirrored in S.tl:
//   io <- sc * ((H_q - shift) cur) - pm * io + cw w_q
// io holds the previous vector on entry and the new one on exit (registers
// only; the caller mirrors it).
//
// Projections: S.pacc[par] holds <chi_I, cur> on entry and S.pacc[par ^ 1]
// is zero; on exit S.pacc[par ^ 1] holds <chi_I, io>.  FUSED: they come out
// of the same sweep that adds the projector terms c_I chi_I, c_I = sc gamma
// dV <chi_I, cur>: every column visits its images in increasing index, and
// the projection onto chi_I is taken before the column adds c_I chi_I, so the
// sweep yields <chi_I, u> + sum_{J < I} c_J G_IJ (u the stencil part of io,
// G the Gram matrix of the projectors over the cube); the missing
// sum_{J >= I} G_IJ c_J is added from the stored upper triangle.  Otherwise
// (a cube whose Gram matrix exceeds its capacity) a second sweep projects
// the finished io.  The caller clears S.pacc[par] before the next step.
// Ends after one block barrier.
template <class Vr, bool FUSED>
__device__ __forceinline__ void apply_step(Smem<Vr>& S, Ctx<Vr>& X, const CellDev& C,
                                           const typename Vr::T (&cur)[Vr::NC],
                                           typename Vr::T (&io)[Vr::NC], const typename Vr::T* ck,
                                           double sc, typename Vr::T pm, int par, double cw = 0.0) {
  using T = typename Vr::T;
  using L = typename Vr::L;
  constexpr int NC = Vr::NC;
  constexpr unsigned IMASK = (1u << Vr::IBITS) - 1u;
  const int nsw = X.nsw;
  // keep the per-slot data opaque so that nothing derived from it is hoisted
  // across steps (register pressure)
#pragma unroll
  for (int s = 0; s < Vr::KC; ++s) opaque(X.sid[s]);
  if constexpr (Vr::AREG) {
#pragma unroll
    for (int s = 0; s < Vr::KC; ++s) opaque(X.a0[s]);
  }
  if constexpr (FUSED) {
    // (1) the upper-triangle Gram terms of the new projections
    const int ngram = S.ngram;
    for (int e = threadIdx.x; e < ngram; e += L::NT) {
      const unsigned ij = S.gidx[e];
      const int i = (int)(ij & 0xffffu), j = (int)(ij >> 16);
      atomicAdd(&S.pacc[par ^ 1][i], S.gval[e] * (sc * S.gdv[j] * S.pacc[par][j]));
    }
  }
  // (2) stencil + diagonal on the own column (x/y neighbours from LDS)
  if (X.active) {
    const int cx = X.cx, cy = X.cy;
    const int base = L::at(cx, cy, 0);
    const T tsc = (T)sc;
#pragma unroll
    for (int z = 0; z < NC; ++z) {
      T acc = X.vd[z] * cur[z];
      const T* pc = S.tl + base + z * L::PL;
#pragma unroll
      for (int k = 1; k <= SQ_FDM; ++k) {
        T s = (T)0;
        if (z + k < NC) s += cur[z + k];
        if (z - k >= 0) s += cur[z - k];
        if constexpr (L::RS > NC) {
          s += (pc[k] + pc[-k]) + (pc[k * L::RS] + pc[-k * L::RS]);
        } else {
          if (cx + k < NC) s += pc[k];
          if (cx - k >= 0) s += pc[-k];
          if (cy + k < NC) s += pc[k * L::RS];
          if (cy - k >= 0) s += pc[-k * L::RS];
        }
        acc += ck[k] * s;
      }
      io[z] = tsc * acc - pm * io[z];
    }
    // optional cw w_q (the unit vector at the node): part of the vector the
    // projector terms are added to, and of its projections
    if (X.cx == Vr::NC / 2 && X.cy == Vr::NC / 2) io[Vr::NC / 2] += (T)cw;
  }
  if constexpr (FUSED) {
    // (3) one sweep per image: projection of io, then the projector term
#pragma unroll
    for (int s = 0; s < Vr::KC; ++s) {
      if (s < nsw) {
        const unsigned mk = X.sid[s];
        const int i = (int)(mk & IMASK);
        const T coef = (T)(s < X.nslot ? sc * S.gdv[i] * S.pacc[par][i] : 0.0);
        T part = (T)0;
        slot_sweep<NC>(mk, slot_start<Vr>(S, X, C, s, i), S.r0[i], S.cq[i],
                       [&](int z, bool on, double a) {
                         const T w = chord_weight<T>(on, a);
                         part += w * io[z];
                         io[z] += w * coef;
                       });
        if (s < X.nslot) atomicAdd(&S.pacc[par ^ 1][i], (double)part);
      }
    }
  } else {
    // (3') the projector terms, then the projections of the finished io
#pragma unroll
    for (int s = 0; s < Vr::KC; ++s) {
      if (s < nsw) {
        const unsigned mk = X.sid[s];
        const int i = (int)(mk & IMASK);
        const double coef = s < X.nslot ? sc * S.gdv[i] * S.pacc[par][i] : 0.0;
        slot_sweep<NC>(mk, coef * slot_start<Vr>(S, X, C, s, i), S.r0[i], S.cq[i],
                       [&](int z, bool on, double a) { io[z] += chord_weight<T>(on, a); });
      }
    }
    project<Vr>(S, X, C, io, par ^ 1);
  }
  __syncthreads();
}

template <class Vr>
__device__ __forceinline__ void clear_proj(Smem<Vr>& S, int buf) {
  for (int i = threadIdx.x; i < Vr::NIMG; i += Vr::L::NT) S.pacc[buf][i] = 0.0;
}

// Mirror the column into LDS (the caller places a barrier before it is read).
template <class Vr>
__device__ __forceinline__ void mirror(Smem<Vr>& S, const Ctx<Vr>& X, const typename Vr::T (&v)[Vr::NC]) {
  using L = typename Vr::L;
  if (X.active) {
    const int base = L::at(X.cx, X.cy, 0);
#pragma unroll
    for (int z = 0; z < Vr::NC; ++z) S.tl[base + z * L::PL] = v[z];
  }
}

template <class Vr>
__device__ __forceinline__ void load_unit(Smem<Vr>& S, Ctx<Vr>& X, typename Vr::T (&cur)[Vr::NC],
                                          typename Vr::T (&prv)[Vr::NC]) {
  using T = typename Vr::T;
  constexpr int NC = Vr::NC;
  constexpr int m = NC / 2;
#pragma unroll
  for (int z = 0; z < NC; ++z) {
    cur[z] = (X.active && X.cx == m && X.cy == m && z == m) ? (T)1 : (T)0;
    prv[z] = (T)0;
  }
  mirror<Vr>(S, X, cur);
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ void stencil_coefs(const CellDev& C, T* ck) {
  // read from the cell table (uniform: the values stay in scalar registers)
#pragma unroll
  for (int k = 0; k <= SQ_FDM; ++k) ck[k] = sizeof(T) == 8 ? (T)C.ck[k] : (T)C.ckf[k];
}

// Block sums of two values; red is double-buffered by the caller (the next
// use of the same buffer is separated by at least one more barrier).
template <int NW>
__device__ __forceinline__ void block_sum2_db(double& a, double& b, double* red) {
  a = warp_sum(a);
  b = warp_sum(b);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) {
    red[w] = a;
    red[NW + w] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    sa += red[i];
    sb += red[NW + i];
  }
  a = sa;
  b = sb;
}

// ---------------------------------------------------------------------------
// Gram matrix of the projectors over the cube, G_IJ = <chi_I, chi_J> for
// I <= J, restricted to the pairs whose chords share a plane on some column
// (every other entry is zero).  Built once per node by the Lanczos pass from
// the same per-column chords and weights the sweeps use, and stored for the
// moments and stress passes.  A cube with more than SQ_GRAM_MAX such pairs
// gets the count -1, and its steps take two sweeps (projector terms, then
// projections).  Uses the cube buffer as scratch; the caller clears it
// afterwards.
// ---------------------------------------------------------------------------
template <class Vr>
__device__ void gram_build(Smem<Vr>& S, const Ctx<Vr>& X, const CellDev& C) {
  using L = typename Vr::L;
  constexpr int NC = Vr::NC;
  constexpr int NI = Vr::NIMG;
  constexpr int NWD = Vr::NWD;
  constexpr int NT = L::NT;
  constexpr unsigned IMASK = (1u << Vr::IBITS) - 1u;
  static_assert(sizeof(S.tl) >= Vr::GSCR, "Gram scratch");
  unsigned* bm = reinterpret_cast<unsigned*>(S.tl);   // [NI][NWD] pairs present
  int* rs = reinterpret_cast<int*>(bm + NI * NWD);     // [NI + 1] first entry of each row
  unsigned* sl = reinterpret_cast<unsigned*>(rs + NI + 1);   // [KC][NT] slot words
  const int tid = threadIdx.x;
  for (int k = tid; k < NI * NWD; k += NT) bm[k] = 0u;
#pragma unroll
  for (int s = 0; s < Vr::KC; ++s) sl[s * NT + tid] = X.sid[s];
  __syncthreads();
  // pairs of this column's slots (image indices increase with the slot)
  if (X.active) {
    for (int s = 0; s < X.nslot; ++s) {
      const unsigned a = sl[s * NT + tid];
      const int i = (int)(a & IMASK);
      for (int s2 = s; s2 < X.nslot; ++s2) {
        const unsigned b = sl[s2 * NT + tid];
        if ((a & b & ~IMASK) == 0u) continue;
        const int j = (int)(b & IMASK);
        atomicOr(&bm[i * NWD + (j >> 5)], 1u << (j & 31));
      }
    }
  }
  __syncthreads();
  if (tid < NI) {
    int c = 0;
#pragma unroll
    for (int w = 0; w < NWD; ++w) c += __popc(bm[tid * NWD + w]);
    rs[tid] = c;
  }
  __syncthreads();
  if (tid < 64) {   // exclusive scan of the row counts by wave 0
    constexpr int PER = (NI + 63) / 64;
    int loc[PER];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int r = tid * PER + k;
      loc[k] = r < NI ? rs[r] : 0;
      sum += loc[k];
    }
    int inc = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int v = __shfl_up(inc, o);
      if (tid >= o) inc += v;
    }
    int ex = inc - sum;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int r = tid * PER + k;
      if (r < NI) rs[r] = ex;
      ex += loc[k];
    }
    if (tid == 63) S.ngram = inc;
  }
  __syncthreads();
  const int total = S.ngram;
  const bool fits = total <= SQ_GRAM_MAX;
  if (fits)
    for (int e = tid; e < total; e += NT) S.gval[e] = 0.0;
  __syncthreads();
  // column sums of chi_I chi_J over the shared planes
  if (X.active && fits) {
    constexpr int m = NC / 2;
    const double h = C.h;
    for (int s = 0; s < X.nslot; ++s) {
      const unsigned a = sl[s * NT + tid];
      const int i = (int)(a & IMASK);
      const double wi = exp(-sq_sum2(node_coord(X.q0 + X.cx - m, h, S.ix[i]),
                                     node_coord(X.q1 + X.cy - m, h, S.iy[i])) * S.i2s[i]) * S.e0[i];
      for (int s2 = s; s2 < X.nslot; ++s2) {
        const unsigned b = sl[s2 * NT + tid];
        if ((a & b & ~IMASK) == 0u) continue;
        const int j = (int)(b & IMASK);
        const double wj = exp(-sq_sum2(node_coord(X.q0 + X.cx - m, h, S.ix[j]),
                                       node_coord(X.q1 + X.cy - m, h, S.iy[j])) * S.i2s[j]) * S.e0[j];
        double ai = wi, ri = S.r0[i], aj = wj, rj = S.r0[j], sum = 0.0;
        const double qi = S.cq[i], qj = S.cq[j];
        unsigned mk = a & b;
#pragma unroll
        for (int z = 0; z < NC; ++z) {
          unsigned nm;
          const bool on = __builtin_add_overflow(mk, mk, &nm);
          mk = nm;
          sum += on ? ai * aj : 0.0;
          ai *= ri;
          ri *= qi;
          aj *= rj;
          rj *= qj;
        }
        const int jw = j >> 5;
        int idx = rs[i] + __popc(bm[i * NWD + jw] & ((1u << (j & 31)) - 1u));
        for (int w = 0; w < jw; ++w) idx += __popc(bm[i * NWD + w]);
        atomicAdd(&S.gval[idx], sum);
        S.gidx[idx] = (unsigned)i | ((unsigned)j << 16);
      }
    }
  }
  if (!fits && tid == 0) S.ngram = -1;   // the steps then take two sweeps
  __syncthreads();
}

template <class Vr>
__device__ __forceinline__ void gram_store(const Smem<Vr>& S, const PlanDev& P, long long g) {
  const int ng = S.ngram;
  for (int e = threadIdx.x; e < ng; e += Vr::L::NT) {
    P.gval[g * SQ_GRAM_MAX + e] = S.gval[e];
    P.gidx[g * SQ_GRAM_MAX + e] = S.gidx[e];
  }
  if (threadIdx.x == 0) P.gn[g] = ng;
}

// (the caller places a barrier before the entries are read)
template <class Vr>
__device__ __forceinline__ void gram_load(Smem<Vr>& S, const PlanDev& P, long long g) {
  const int ng = min(max(P.gn[g], -1), SQ_GRAM_MAX);
  for (int e = threadIdx.x; e < ng; e += Vr::L::NT) {
    S.gval[e] = P.gval[g * SQ_GRAM_MAX + e];
    S.gidx[e] = P.gidx[g * SQ_GRAM_MAX + e];
  }
  if (threadIdx.x == 0) S.ngram = ng;
}

// ---------------------------------------------------------------------------
// Spectral bounds: K-step FP64 Lanczos on H_q from the unit vector w_q
// (chi_q and zeta_q come from the extreme eigenvalues of H_q, Sec. IV)
// ---------------------------------------------------------------------------
// One Lanczos step with v_k in A (and S.tl), v_{k-1} in B on entry; on exit
// v_{k+1} is in B (and S.tl) unless the recursion stopped.
template <class Vr, bool FUSED>
__device__ __forceinline__ bool lanczos_step(Smem<Vr>& S, Ctx<Vr>& X, const CellDev& C,
                                             const double (&A)[Vr::NC], double (&B)[Vr::NC],
                                             const double* ck, int k, double& bprev, double& tol,
                                             double* lan) {
  constexpr int NC = Vr::NC;
  constexpr int NW = Vr::L::NW;
  apply_step<Vr, FUSED>(S, X, C, A, B, ck, 1.0, bprev, k & 1);   // B = H v_k - beta v_{k-1}
  double a = 0.0, dum = 0.0;
#pragma unroll
  for (int z = 0; z < NC; ++z) a += A[z] * B[z];
  block_sum2_db<NW>(a, dum, S.red[0]);
  double b = 0.0;
#pragma unroll
  for (int z = 0; z < NC; ++z) {
    B[z] -= a * A[z];
    b += B[z] * B[z];
  }
  block_sum2_db<NW>(b, dum, S.red[1]);
  b = sqrt(b);
  if (threadIdx.x == 0) {
    lan[k] = a;
    lan[SQ_KL_MAX + k] = b;
  }
  if (k == 0) tol = 1e-14 * (fabs(a) + b);
  if (b < tol) return false;
  const double ib = 1.0 / b;
#pragma unroll
  for (int z = 0; z < NC; ++z) B[z] *= ib;
  mirror<Vr>(S, X, B);
  // projections of v_{k+1} = (H v_k - beta v_{k-1} - a v_k) / b
  const int par = k & 1;
  for (int i = threadIdx.x; i < Vr::NIMG; i += Vr::L::NT) {
    S.pacc[par ^ 1][i] = (S.pacc[par ^ 1][i] - a * S.pacc[par][i]) * ib;
    S.pacc[par][i] = 0.0;
  }
  bprev = b;
  __syncthreads();
  return true;
}

template <class Vr, bool FUSED>
__global__ void __launch_bounds__(Vr::L::NT) k_lanczos(PlanDev P, const long long* items,
                                                        const int* item_cell) {
  static_assert(sizeof(typename Vr::T) == 8, "Lanczos runs in FP64");
  constexpr int NC = Vr::NC;
  __shared__ Smem<Vr> S;
  const long long g = items[blockIdx.x];
  const CellDev& C = P.cells[item_cell[blockIdx.x]];
  const long long q = g - C.node_base;
  Ctx<Vr> X;
  node_prologue<Vr>(C, q, 0.0, S, X, P.err);
  if constexpr (FUSED) gram_load<Vr>(S, P, g);
  double ck[SQ_FDM + 1];
  stencil_coefs<double>(C, ck);
  double A[NC], B[NC];
  load_unit<Vr>(S, X, A, B);
  project<Vr>(S, X, C, A, 0);
  __syncthreads();
  double bprev = 0.0, tol = 0.0;
  int steps = 0;
  double* lan = P.lan + g * (2 * SQ_KL_MAX);
  for (int k = 0; k < C.K; k += 2) {
    steps = k + 1;
    if (!lanczos_step<Vr, FUSED>(S, X, C, A, B, ck, k, bprev, tol, lan)) break;
    if (k + 1 >= C.K) break;
    steps = k + 2;
    if (!lanczos_step<Vr, FUSED>(S, X, C, B, A, ck, k + 1, bprev, tol, lan)) break;
  }
  if (threadIdx.x == 0) P.lan_steps[g] = steps;
}

// Set-up pass: the Gram matrix of every node's projectors (count -1 when it
// exceeds SQ_GRAM_MAX entries; such nodes are launched with FUSED = false).
template <class Vr>
__global__ void __launch_bounds__(Vr::L::NT) k_gram(PlanDev P, const long long* items,
                                                     const int* item_cell) {
  static_assert(sizeof(typename Vr::T) == 8, "the Gram build runs in FP64");
  __shared__ Smem<Vr> S;
  const long long g = items[blockIdx.x];
  const CellDev& C = P.cells[item_cell[blockIdx.x]];
  const long long q = g - C.node_base;
  Ctx<Vr> X;
  node_prologue<Vr>(C, q, 0.0, S, X, P.err);
  gram_build<Vr>(S, X, C);
  gram_store<Vr>(S, P, g);
}

// ---------------------------------------------------------------------------
// Chebyshev moments rho_q^j = w_q^T T_j(Hhat_q) w_q, j = 0..npl, from the
// three-term recurrence (Sec. IV) taken to degree ceil(npl/2) with
//   rho^{2k} = 2 <t^k, t^k> - rho^0,  rho^{2k+1} = 2 <t^{k+1}, t^k> - rho^1
// (Hhat_q is symmetric, T_{a+b} + T_{|a-b|} = 2 T_a T_b).
// ---------------------------------------------------------------------------
template <class Vr, bool FUSED>
__global__ void __launch_bounds__(Vr::L::NT) k_moments(PlanDev P, const long long* items,
                                                        const int* item_cell) {
  using T = typename Vr::T;
  constexpr int NC = Vr::NC;
  constexpr int NW = Vr::L::NW;
  __shared__ Smem<Vr> S;
  const long long g = items[blockIdx.x];
  const CellDev& C = P.cells[item_cell[blockIdx.x]];
  const long long q = g - C.node_base;
  const double chi = P.bnd[4 * g + 2], zeta = P.bnd[4 * g + 3];
  Ctx<Vr> X;
  node_prologue<Vr>(C, q, chi, S, X, P.err);
  if constexpr (FUSED) gram_load<Vr>(S, P, g);
  T ck[SQ_FDM + 1];
  stencil_coefs<T>(C, ck);
  T A[NC], B[NC];
  load_unit<Vr>(S, X, A, B);
  project<Vr>(S, X, C, A, 0);
  __syncthreads();
  double* mom = P.mom + g * P.mstride;
  const int npl = C.npl;
  const int kmax = (npl + 1) / 2;
  double rho1 = 0.0;
  bool bad = false;
  if (threadIdx.x == 0) mom[0] = 1.0;
  // t^{k+1} from t^k (cur) and t^{k-1} (io); then rho^{2k+1}, rho^{2k+2}
  auto step = [&](const T (&cur)[NC], T (&io)[NC], int k) {
    apply_step<Vr, FUSED>(S, X, C, cur, io, ck, k == 0 ? 1.0 / zeta : 2.0 / zeta, k == 0 ? (T)0 : (T)1,
                   k & 1);
    double sq = 0.0, cr = 0.0;
#pragma unroll
    for (int z = 0; z < NC; ++z) {
      const double a = (double)io[z], b = (double)cur[z];
      sq += a * a;
      cr += a * b;
    }
    mirror<Vr>(S, X, io);
    clear_proj<Vr>(S, k & 1);
    block_sum2_db<NW>(sq, cr, S.red[k & 1]);
    if (k == 0) rho1 = cr;
    const int j1 = 2 * k + 1, j2 = 2 * k + 2;
    const double r1 = (k == 0) ? cr : 2.0 * cr - rho1;
    const double r2 = 2.0 * sq - 1.0;
    if (fabs(r1) > 1.0 + 1e-4 || (j2 <= npl && fabs(r2) > 1.0 + 1e-4) || !(r1 == r1)) bad = true;
    if (threadIdx.x == 0) {
      mom[j1] = r1;
      if (j2 <= npl) mom[j2] = r2;
    }
  };
  for (int k = 0; k < kmax; k += 2) {
    step(A, B, k);
    if (k + 1 < kmax) step(B, A, k + 1);
  }
  if (bad && threadIdx.x == 0) atomicOr(P.err, SQ_ERR_BOUNDS);
}

// ---------------------------------------------------------------------------
// Stress pass: recurrence again with the coefficients known, the DM column
// d_q = sum'_j c_q^j t^j accumulated in FP64, then the kinetic functional
// K_ab = 2 (grad_a grad_b d_q)_q and the nonlocal functional
// N_ab = -2 sum_I gamma dV chi_I(x_q) [delta_ab chi_I^T d_q
//        + 2 sum_y chi_I(y) (y_b - R_Ib) (grad_a d_q)(y)]   (Sec. IV)
// ---------------------------------------------------------------------------
template <class Vr>
__device__ __forceinline__ void grad_xy_round(Smem<Vr>& S, Ctx<Vr>& X,
                                              const typename Vr::T (&part)[Vr::NC],
                                              double (&gx)[Vr::NC], double (&gy)[Vr::NC],
                                              const double* w) {
  constexpr int NC = Vr::NC;
  using T = typename Vr::T;
  using L = typename Vr::L;
  const int base = L::at(X.cx, X.cy, 0);
  mirror<Vr>(S, X, part);
  __syncthreads();
  if (X.active) {
    const int cx = X.cx, cy = X.cy;
#pragma unroll
    for (int z = 0; z < NC; ++z) {
      const T* pc = S.tl + base + z * L::PL;
      double ax = 0.0, ay = 0.0;
#pragma unroll
      for (int k = 1; k <= SQ_FDM; ++k) {
        if constexpr (L::RS > NC) {
          ax += w[k] * ((double)pc[k] - (double)pc[-k]);
          ay += w[k] * ((double)pc[k * L::RS] - (double)pc[-k * L::RS]);
        } else {
          if (cx + k < NC) ax += w[k] * (double)pc[k];
          if (cx - k >= 0) ax -= w[k] * (double)pc[-k];
          if (cy + k < NC) ay += w[k] * (double)pc[k * L::RS];
          if (cy - k >= 0) ay -= w[k] * (double)pc[-k * L::RS];
        }
      }
      gx[z] += ax;
      gy[z] += ay;
    }
  }
  __syncthreads();
}

template <class Vr, bool FUSED>
__global__ void __launch_bounds__(Vr::L::NT) k_stress(PlanDev P, const long long* items,
                                                       const int* item_cell) {
  using T = typename Vr::T;
  using L = typename Vr::L;
  constexpr int NC = Vr::NC;
  constexpr int NC2 = NC * NC;
  constexpr int m = L::MH;
  constexpr unsigned IMASK = (1u << Vr::IBITS) - 1u;
  __shared__ Smem<Vr> S;
  const long long g = items[blockIdx.x];
  const CellDev& C = P.cells[item_cell[blockIdx.x]];
  const long long q = g - C.node_base;
  const double chi = P.bnd[4 * g + 2], zeta = P.bnd[4 * g + 3];
  const double* coef = P.coef + g * P.mstride;
  Ctx<Vr> X;
  node_prologue<Vr>(C, q, chi, S, X, P.err);
  if constexpr (FUSED) gram_load<Vr>(S, P, g);
  T ck[SQ_FDM + 1];
  stencil_coefs<T>(C, ck);
  T A[NC], B[NC];
  double d[NC];
  const int npl = C.npl;
  if constexpr (sizeof(T) == 8) {
    // FP64: Clenshaw's recurrence for d_q = sum'_j c_j T_j(Hhat) w_q,
    //   b_k = c_k w + 2 Hhat b_{k+1} - b_{k+2},  k = npl-1 .. 1,
    //   b_npl = c_npl w,  b_{npl+1} = 0,  d_q = c_0 w / 2 + Hhat b_1 - b_2,
    // the same npl applications as the forward recurrence but no separate
    // accumulator for d_q (registers)
    load_unit<Vr>(S, X, A, B);
    const T cn = (T)coef[npl];
#pragma unroll
    for (int z = 0; z < NC; ++z) A[z] *= cn;
    mirror<Vr>(S, X, A);
    __syncthreads();
    project<Vr>(S, X, C, A, 0);
    __syncthreads();
    // step j computes b_k, k = npl - 1 - j, from b_{k+1} (cur) and b_{k+2}
    // (io); the last one (k = 0) forms d_q
    auto step = [&](const T (&cur)[NC], T (&io)[NC], int j) {
      const int k = npl - 1 - j;
      apply_step<Vr, FUSED>(S, X, C, cur, io, ck, k == 0 ? 1.0 / zeta : 2.0 / zeta, (T)1, j & 1,
                            k == 0 ? 0.5 * coef[0] : coef[k]);
      mirror<Vr>(S, X, io);
      clear_proj<Vr>(S, j & 1);
      __syncthreads();
    };
    for (int j = 0; j < npl; j += 2) {
      step(A, B, j);
      if (j + 1 < npl) step(B, A, j + 1);
    }
    const bool in_b = (npl & 1) != 0;
#pragma unroll
    for (int z = 0; z < NC; ++z) d[z] = (double)(in_b ? B[z] : A[z]);
  } else {
    // FP32 vectors: forward recurrence t^{j+1} = 2 Hhat t^j - t^{j-1} with
    // d_q = sum'_j c_j t^j accumulated in FP64
    load_unit<Vr>(S, X, A, B);
    project<Vr>(S, X, C, A, 0);
    __syncthreads();
    const double c0h = 0.5 * coef[0];
#pragma unroll
    for (int z = 0; z < NC; ++z) d[z] = c0h * (double)A[z];
    auto step = [&](const T (&cur)[NC], T (&io)[NC], int j) {
      apply_step<Vr, FUSED>(S, X, C, cur, io, ck, j == 0 ? 1.0 / zeta : 2.0 / zeta,
                            j == 0 ? (T)0 : (T)1, j & 1);
      const double cj = coef[j + 1];
#pragma unroll
      for (int z = 0; z < NC; ++z) d[z] += cj * (double)io[z];
      mirror<Vr>(S, X, io);
      clear_proj<Vr>(S, j & 1);
      __syncthreads();
    };
    for (int j = 0; j < npl; j += 2) {
      step(A, B, j);
      if (j + 1 < npl) step(B, A, j + 1);
    }
  }

  // ---- gradients of d along x, y (LDS, FP64 via hi/lo rounds) and z ----
  const double ih = 1.0 / C.h;
  double w[SQ_FDM + 1];
#pragma unroll
  for (int k = 0; k <= SQ_FDM; ++k) w[k] = C.c1[k];
  double gx[NC], gy[NC], gz[NC];
#pragma unroll
  for (int z = 0; z < NC; ++z) {
    gx[z] = 0.0;
    gy[z] = 0.0;
    double a = 0.0;
#pragma unroll
    for (int k = 1; k <= SQ_FDM; ++k) {
      if (z + k < NC) a += w[k] * d[z + k];
      if (z - k >= 0) a -= w[k] * d[z - k];
    }
    gz[z] = a * ih;
  }
  {
    T hi[NC];
#pragma unroll
    for (int z = 0; z < NC; ++z) hi[z] = (T)d[z];
    grad_xy_round<Vr>(S, X, hi, gx, gy, w);
    if constexpr (sizeof(T) < sizeof(double)) {
#pragma unroll
      for (int z = 0; z < NC; ++z) hi[z] = (T)(d[z] - (double)hi[z]);
      grad_xy_round<Vr>(S, X, hi, gx, gy, w);
    }
#pragma unroll
    for (int z = 0; z < NC; ++z) {
      gx[z] *= ih;
      gy[z] *= ih;
    }
  }

  // ---- kinetic functional from the plane z = m and the centre column ----
  double* plane = reinterpret_cast<double*>(S.tl);   // 3 * NC2 + 3 * NC doubles
  static_assert(sizeof(T) * L::SIZE >= sizeof(double) * (3 * NC2 + 3 * NC), "plane");
  if (X.active) {
    plane[X.col] = gx[m];
    plane[NC2 + X.col] = gy[m];
    plane[2 * NC2 + X.col] = gz[m];
    if (X.cx == m && X.cy == m) {
#pragma unroll
      for (int z = 0; z < NC; ++z) {
        plane[3 * NC2 + z] = gx[z];
        plane[3 * NC2 + NC + z] = gy[z];
        plane[3 * NC2 + 2 * NC + z] = gz[z];
      }
    }
  }
  // ---- near images: projector nonzero at the node itself ----
  if (X.active && X.cx == m && X.cy == m) {
    int nn = 0;
#pragma unroll
    for (int s = 0; s < Vr::KC; ++s) {
      if (s < X.nslot) {
        const unsigned mk = X.sid[s];
        const int i = (int)(mk & IMASK);
        if (mk & (0x80000000u >> m)) {
          if (nn < Vr::NEAR) {
            S.near_img[nn] = i;
            const double dx = node_coord(X.q0, C.h, S.ix[i]);
            const double dy = node_coord(X.q1, C.h, S.iy[i]);
            const double dz = node_coord(X.q2, C.h, S.iz[i]);
            S.near_chi[nn] = exp(-sq_add(sq_sum2(dx, dy), dz) * S.i2s[i]);
          } else {
            atomicOr(P.err, SQ_ERR_NEAR);
          }
          ++nn;
        }
      }
    }
    S.nnear = nn < Vr::NEAR ? nn : Vr::NEAR;
  }
  for (int i = threadIdx.x; i < Vr::NEAR * 10; i += L::NT) (&S.nsum[0][0])[i] = 0.0;
  __syncthreads();

  double* rec = P.rec + g * SQ_REC;
  if (threadIdx.x == 0) {
    const double* px = plane;
    const double* py = plane + NC2;
    const double* pz = plane + 2 * NC2;
    const double* cxg = plane + 3 * NC2;
    // (grad_a G_b)(c) = (1/h) sum_k w_k (G_b(c + k e_a) - G_b(c - k e_a))
    for (int b = 0; b < 3; ++b) {
      const double* pb = b == 0 ? px : (b == 1 ? py : pz);
      const double* cb = cxg + b * NC;
      double kx = 0.0, ky = 0.0, kz = 0.0;
      for (int k = 1; k <= SQ_FDM; ++k) {
        if (k > m) break;
        kx += w[k] * (pb[m * NC + m + k] - pb[m * NC + m - k]);
        ky += w[k] * (pb[(m + k) * NC + m] - pb[(m - k) * NC + m]);
        kz += w[k] * (cb[m + k] - cb[m - k]);
      }
      rec[2 + 0 * 3 + b] = 2.0 * kx * ih;
      rec[2 + 1 * 3 + b] = 2.0 * ky * ih;
      rec[2 + 2 * 3 + b] = 2.0 * kz * ih;
    }
  }

  // ---- nonlocal sums over the support of every near image ----
  const int nnear = S.nnear;
  if (X.active && nnear > 0) {
    const double xc = (double)(X.q0 + X.cx - m) * C.h;
    const double yc = (double)(X.q1 + X.cy - m) * C.h;
#pragma unroll
    for (int s = 0; s < Vr::KC; ++s) {
      if (s < X.nslot) {
        const unsigned mk = X.sid[s];
        const int i = (int)(mk & IMASK);
        int nidx = -1;
        for (int n = 0; n < nnear; ++n)
          if (S.near_img[n] == i) nidx = n;
        if (nidx >= 0) {
          const double rx = xc - S.ix[i], ry = yc - S.iy[i];
          double acc[10];
#pragma unroll
          for (int t = 0; t < 10; ++t) acc[t] = 0.0;
          slot_sweep<NC>(mk, slot_start<Vr>(S, X, C, s, i), S.r0[i], S.cq[i],
                         [&](int z, bool on, double chiv) {
                           if (on) {
                             const double rz = (double)(X.q2 + z - m) * C.h - S.iz[i];
                             acc[0] += chiv * d[z];
                             const double ga[3] = {gx[z], gy[z], gz[z]};
                             const double rb[3] = {rx, ry, rz};
#pragma unroll
                             for (int a = 0; a < 3; ++a)
#pragma unroll
                               for (int b = 0; b < 3; ++b) acc[1 + 3 * a + b] += chiv * rb[b] * ga[a];
                           }
                         });
#pragma unroll
          for (int t = 0; t < 10; ++t) atomicAdd(&S.nsum[nidx][t], acc[t]);
        }
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double N[9], enl = 0.0;
    for (int t = 0; t < 9; ++t) N[t] = 0.0;
    for (int n = 0; n < nnear; ++n) {
      const int i = S.near_img[n];
      const double f = -2.0 * S.gdv[i] * S.near_chi[n];
      enl -= f * S.nsum[n][0];   // 2 gamma dV chi_I(x_q) chi_I^T d_q
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          N[3 * a + b] += f * ((a == b ? S.nsum[n][0] : 0.0) + 2.0 * S.nsum[n][1 + 3 * a + b]);
    }
    for (int t = 0; t < 9; ++t) rec[11 + t] = N[t];
    rec[20] = enl;
  }
}

// ---------------------------------------------------------------------------
// Capacity census (set-up time): per node the number of atom images reaching
// its cube, the largest number crossing one z-column, and the number whose
// projector is nonzero at the node.  Maxima per cell go to stats[4 * cell].
// ---------------------------------------------------------------------------
template <int NC>
__global__ void __launch_bounds__(sq_threads(NC)) k_census(PlanDev P, const long long* items,
                                                            const int* item_cell, int* stats,
                                                            long long* pair_total) {
  constexpr int NT = sq_threads(NC);
  constexpr int CAP = 512;
  __shared__ double sx[CAP], sy[CAP], sz[CAP], srp2[CAP];
  __shared__ int wcnt[16], cnt, colmax, nnear;
  __shared__ unsigned long long npairs;
  const long long g = items[blockIdx.x];
  const int ci = item_cell[blockIdx.x];
  const CellDev& C = P.cells[ci];
  const long long q = g - C.node_base;
  const int m = NC / 2;
  const long long q0 = q % C.n[0], q1 = (q / C.n[0]) % C.n[1], q2 = q / ((long long)C.n[0] * C.n[1]);
  auto store = [&](int pos, int I) {
    sx[pos] = C.img[4 * I];
    sy[pos] = C.img[4 * I + 1];
    sz[pos] = C.img[4 * I + 2];
    const double rp = C.sp[(int)C.img[4 * I + 3]].p_rc;
    srp2[pos] = rp * rp;
  };
  const int found = gather_images<NT, NT / 64, CAP>(C, q0, q1, q2, m, &cnt, wcnt, store, P.err);
  const int nimg = found < CAP ? found : CAP;
  if (threadIdx.x == 0) {
    colmax = 0;
    nnear = 0;
    npairs = 0;
  }
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid < NC * NC) {
    const int cx = tid % NC, cy = tid / NC;
    int count = 0, near = 0, pairs = 0;
    for (int i = 0; i < nimg; ++i) {
      const double dx = node_coord(q0 + cx - m, C.h, sx[i]);
      const double dy = node_coord(q1 + cy - m, C.h, sy[i]);
      const double dxy2 = sq_sum2(dx, dy);
      if (!(dxy2 < srp2[i])) continue;
      bool any = false;
      for (int z = 0; z < NC; ++z) {
        const double dz = node_coord(q2 + z - m, C.h, sz[i]);
        if (sq_add(dxy2, dz) < srp2[i]) {
          any = true;
          ++pairs;
          if (cx == m && cy == m && z == m) ++near;
        }
      }
      if (any) ++count;
    }
    atomicMax(&colmax, count);
    if (near) atomicAdd(&nnear, near);
    if (pairs) atomicAdd(&npairs, (unsigned long long)pairs);
  }
  __syncthreads();
  if (tid == 0) {
    atomicMax(&stats[4 * ci + 0], found);
    atomicMax(&stats[4 * ci + 1], colmax);
    atomicMax(&stats[4 * ci + 2], nnear);
    atomicAdd(reinterpret_cast<unsigned long long*>(pair_total) + ci, npairs);
  }
}

}  // namespace

#define SQ_CAT2(a, b) a##b
#define SQ_CAT(a, b) SQ_CAT2(a, b)
// Everything below that depends on the width has internal linkage: the
// units of the other widths define templates of the same names, and weak
// (COMDAT) instantiations would otherwise be merged across widths.
namespace {
constexpr int SQN = SQ_ONE_NC;

enum Fam { FAM_LAN, FAM_MOM, FAM_STR, FAM_GRAM };

template <class Vr, int F, bool FUSED>
hipError_t launch_var(const PlanDev& P, const long long* items, const int* ic, long long n,
                      hipStream_t s) {
  const dim3 grid((unsigned)n), block(Vr::L::NT);
  if constexpr (F == FAM_LAN)
    hipLaunchKernelGGL((k_lanczos<Vr, FUSED>), grid, block, 0, s, P, items, ic);
  else if constexpr (F == FAM_MOM)
    hipLaunchKernelGGL((k_moments<Vr, FUSED>), grid, block, 0, s, P, items, ic);
  else if constexpr (F == FAM_STR)
    hipLaunchKernelGGL((k_stress<Vr, FUSED>), grid, block, 0, s, P, items, ic);
  else
    hipLaunchKernelGGL(k_gram<Vr>, grid, block, 0, s, P, items, ic);
  return hipGetLastError();
}

// Nodes without a stored Gram matrix (rare: dense projector overlap) all use
// the widest slot capacity, so only one two-sweep variant per precision is
// compiled.
template <int F, bool FUSED>
hipError_t launch_fp64(int kc, const PlanDev& P, const long long* items, const int* ic, long long n,
                       hipStream_t s) {
  if constexpr (!FUSED) {
    if (kc <= 48) return launch_var<Var<double, SQN, 48, false>, F, FUSED>(P, items, ic, n, s);
  } else {
    if (kc <= 14) return launch_var<Var<double, SQN, 14, true>, F, FUSED>(P, items, ic, n, s);
    if (kc <= 16) return launch_var<Var<double, SQN, 16, true>, F, FUSED>(P, items, ic, n, s);
    if (kc <= 32) return launch_var<Var<double, SQN, 32, false>, F, FUSED>(P, items, ic, n, s);
    if (kc <= 48) return launch_var<Var<double, SQN, 48, false>, F, FUSED>(P, items, ic, n, s);
  }
  return hipErrorInvalidValue;
}

template <int F, bool FUSED>
hipError_t launch_fp32(int kc, const PlanDev& P, const long long* items, const int* ic, long long n,
                       hipStream_t s) {
  if constexpr (!FUSED) {
    if (kc <= 48) return launch_var<Var<float, SQN, 48, false>, F, FUSED>(P, items, ic, n, s);
  } else {
    if (kc <= 14) return launch_var<Var<float, SQN, 14, true>, F, FUSED>(P, items, ic, n, s);
    if (kc <= 16) return launch_var<Var<float, SQN, 16, true>, F, FUSED>(P, items, ic, n, s);
    if (kc <= 32) return launch_var<Var<float, SQN, 32, true>, F, FUSED>(P, items, ic, n, s);
    if (kc <= 48) return launch_var<Var<float, SQN, 48, false>, F, FUSED>(P, items, ic, n, s);
  }
  return hipErrorInvalidValue;
}

template <int F>
hipError_t launch_prec(bool fp64, bool fused, int kc, const PlanDev& P, const long long* items,
                       const int* ic, long long n, hipStream_t s) {
  if (fp64)
    return fused ? launch_fp64<F, true>(kc, P, items, ic, n, s) : launch_fp64<F, false>(kc, P, items, ic, n, s);
  return fused ? launch_fp32<F, true>(kc, P, items, ic, n, s) : launch_fp32<F, false>(kc, P, items, ic, n, s);
}
}  // namespace

hipError_t SQ_CAT(sq_launch_lanczos_, SQ_ONE_NC)(int kc, bool fused, const PlanDev& P,
                                                const long long* items, const int* ic, long long n,
                                                hipStream_t s) {
  return fused ? launch_fp64<FAM_LAN, true>(kc, P, items, ic, n, s)
               : launch_fp64<FAM_LAN, false>(kc, P, items, ic, n, s);
}

hipError_t SQ_CAT(sq_launch_moments_, SQ_ONE_NC)(bool fp64, int kc, bool fused, const PlanDev& P,
                                                const long long* items, const int* ic, long long n,
                                                hipStream_t s) {
  return launch_prec<FAM_MOM>(fp64, fused, kc, P, items, ic, n, s);
}

hipError_t SQ_CAT(sq_launch_stress_, SQ_ONE_NC)(bool fp64, int kc, bool fused, const PlanDev& P,
                                               const long long* items, const int* ic, long long n,
                                               hipStream_t s) {
  return launch_prec<FAM_STR>(fp64, fused, kc, P, items, ic, n, s);
}

hipError_t SQ_CAT(sq_launch_gram_, SQ_ONE_NC)(int kc, const PlanDev& P, const long long* items,
                                             const int* ic, long long n, hipStream_t s) {
  return launch_fp64<FAM_GRAM, true>(kc, P, items, ic, n, s);
}

hipError_t SQ_CAT(sq_launch_census_, SQ_ONE_NC)(const PlanDev& P, const long long* items,
                                               const int* ic, long long n, int* stats,
                                               long long* pairs, hipStream_t s) {
  hipLaunchKernelGGL(k_census<SQN>, dim3((unsigned)n), dim3(sq_threads(SQN)), 0, s, P, items, ic, stats,
                     pairs);
  return hipGetLastError();
}
