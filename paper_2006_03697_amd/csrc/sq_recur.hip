// sq_recur.hip -- gfx950 recurrence kernels of the infinite-cell
// Clenshaw-Curtis SQ hot path (arXiv 2006.03697, Sec. IV and App. A):
// spectral-bound Lanczos, Chebyshev moments, the stress pass, the projector
// Gram matrices and the capacity census.  Compiled once per cube width NC
// (SQ_ONE_NC).
//
// One workgroup owns one node q and its cube (region of influence) of
// NC^3 finite-difference nodes.  Thread (cx, cy) owns the z-column (cx, cy)
// of the cube: the current Chebyshev vector, the previous one and the
// diagonal of H_q on that column live in its registers; the current vector
// is mirrored in LDS so that x/y neighbours of the 12th-order stencil are LDS
// reads and z neighbours register reads.  Atom-image projectors are
// separable Gaussians cut off at a sphere: per (column, image) the chord of
// the sphere on the column as a bit mask and the projector value at the
// column's first plane (registers, computed once per node); along the column
// the Gaussian factor follows from a two-multiply recurrence.  One sweep per operator application both adds
// the projector terms and takes the new projections (completed by the stored
// Gram matrix of the node's projectors).  Projections are summed exactly in
// two-word integers, so every result is reproducible bit for bit.
#include "sq_devfn.h"

#ifndef SQ_ONE_NC
#error "sq_recur.hip is compiled once per cube width: define SQ_ONE_NC"
#endif

namespace {
// ---------------------------------------------------------------------------
// Cube layout in LDS and the thread <-> z-column map
//
// The mirror holds G consecutive planes of a column in one element (FP64:
// two planes, 16 bytes; FP32: two planes, 8 bytes), so every x/y neighbour
// read of the stencil serves G planes: FP64 reads are ds_read_b128, which
// run at about 1.85x the bytes per clock of 8-byte reads on gfx950.  (Four
// FP32 planes per 16-byte element would halve the FP32 reads again, but the
// register tuples of the 16-byte loads then push the FP32 kernels into
// kilobytes of spills.)
//
// Padded layout: rows of RS >= NC + 6 elements (the tail zero) and plane
// groups of NC + 6 rows (the last 6 zero), after 6 zero rows and 6 zeros,
// so every x/y neighbour outside the cube reads a zero and needs no
// predicate; the zero rows and columns are shared by consecutive rows and
// plane groups.
//
// LDS has 64 banks of 4 bytes: M = 256 / E lanes reading E bytes each
// (E = 16: M = 16; E = 8: M = 32) are conflict-free when their element
// indices are distinct modulo M.  With the padded row stride consecutive
// rows alias, so lanes are mapped to columns by address residue instead of
// row-major: lane M g + r owns the g-th column (in row-major order) whose
// row offset cy * RS + cx is congruent to r modulo M.  Every access of an
// M-lane group is then a constant shift of these offsets, hence
// conflict-free.  RS is the smallest stride for which no residue class has
// more columns than the block has M-lane groups.
// ---------------------------------------------------------------------------
constexpr int sq_residue_max(int nc, int rs, int mod) {
  int cnt[32] = {};
  int mx = 0;
  for (int cy = 0; cy < nc; ++cy)
    for (int cx = 0; cx < nc; ++cx) {
      const int r = (cy * rs + cx) & (mod - 1);
      if (++cnt[r] > mx) mx = cnt[r];
    }
  return mx;
}

constexpr int sq_pick_rs(int nc, int mod) {
  for (int rs = nc + SQ_FDM; rs <= nc + SQ_FDM + 32; ++rs)
    if (sq_residue_max(nc, rs, mod) * mod <= sq_threads(nc)) return rs;
  return 0;
}

// vectors of two values: the mirror element of both precisions, and the
// packed (rr(0), cq) pair of an image
template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec2<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};

template <int NC, int G, int M, bool PAD>
struct Lay {
  static constexpr int NTC = sq_threads(NC);   // threads (one per column)
  static constexpr int MH = NC / 2;
  static constexpr int NZG = (NC + G - 1) / G;                      // plane groups
  static constexpr int RS = PAD ? sq_pick_rs(NC, M) : NC;           // row stride
  static constexpr int PL = PAD ? (NC + SQ_FDM) * RS : NC * NC;     // plane-group stride
  static constexpr int X0 = PAD ? SQ_FDM * RS + SQ_FDM : 0;         // offset of (0, 0, 0)
  static constexpr int SIZE = X0 + NZG * PL;                        // elements
  static_assert(!PAD || RS > 0, "no conflict-free row stride");
  __device__ static constexpr int at(int x, int y, int zg) { return X0 + zg * PL + y * RS + x; }

  // Column of local thread t (see above); inactive threads own no column.
  __device__ static void column(int t, int& cx, int& cy, bool& active) {
    cx = 0;
    cy = 0;
    active = false;
    if constexpr (PAD) {
      const int r = t & (M - 1), g = t / M;
      int seen = 0;
      for (int y = 0; y < NC; ++y) {
        // the columns of row y with residue r (x0, x0 + M, ...)
        for (int x = (r - y * RS) & (M - 1); x < NC; x += M) {
          if (seen == g) {
            cx = x;
            cy = y;
            active = true;
          }
          ++seen;
        }
      }
    } else {
      active = t < NC * NC;
      cx = t % NC;
      cy = t / NC;
    }
  }
};

// A kernel variant: working precision T, cube width NC, KC projector slots
// per z-column, and whether each slot's weight on plane 0 is kept in a
// register (AREG) or recomputed at every use.  The padded LDS layout is used
// when the working set fits the 160 KiB of LDS.
template <typename T_, int NC_, int KC_, bool AREG_>
struct Var {
  using T = T_;
  static constexpr int NC = NC_;
  static constexpr int KC = KC_;
  static constexpr bool AREG = AREG_;
  static constexpr int ZH = NC_;   // planes per thread (the whole column)
  static constexpr int NTC = sq_threads(NC_);
  static constexpr int NT = NTC;
  static constexpr int NW = NT / 64;
  // slot word: chord bits 31 .. 32 - ZH, image index below
  static constexpr int IBITS = 32 - ZH;
  static constexpr int NIMG = sq_img_max(NC_);
  static constexpr int NEAR = SQ_NEAR_MAX;
  static constexpr int GCAP = sq_gram_cap(NC_);
  static constexpr int GPT = (GCAP + NT - 1) / NT;   // Gram entries per thread (registers)
  static_assert(NIMG <= (1 << IBITS) && NIMG <= 65536, "image index width");
  static_assert(NT <= 1024, "workgroup size");
  // The planes of a column are split into NSEG segments.  Per slot, a wave
  // visits only the segments from the first to the last that the chord of
  // some lane touches (images are sorted by z, so a slot holds images of
  // similar height on every lane); the sweep then starts from the slot's
  // weight at the first visited plane.  Only with the weights in registers.
  static constexpr int NSEG = AREG_ && KC_ <= 16 && NC_ >= 13 ? 4 : 1;
  __host__ __device__ static constexpr int seg_lo(int k) { return k * NC_ / NSEG; }
  // LDS besides the cube buffer: per-image tables, near images, block sums,
  // and a union of the projection sums (steps) with the stress pass's
  // near-image sums and line buffer (after the last step)
  static constexpr size_t OTHER = 8 * (size_t)NIMG * 9 + 8 * 4 * (size_t)NIMG + (size_t)NEAR * 12 +
                                  2 * 2 * 16 * 8 + 256 + 8 * (size_t)(NSEG - 1) * NIMG;
  static constexpr size_t EPB = 16 * (size_t)NEAR * 10 + 8 * 9 * (2 * SQ_FDM + 1);
  static constexpr size_t uni(int copies) {
    return 16 * (size_t)NIMG * copies > EPB ? 16 * (size_t)NIMG * copies : EPB;
  }
  // scratch of the Gram build in the cube buffer: pair bitmap [NIMG][NWD],
  // row starts [NIMG + 1], slot words [KC][NT], two-word sums [GCAP][2]
  static constexpr int NWD = (NIMG + 31) / 32;
  static constexpr size_t GSCR = 4 * ((size_t)NIMG * NWD + NIMG + 1 + (size_t)KC * NT) + 8 +
                                 16 * (size_t)GCAP;
  using V = typename Vec2<T_>::type;   // mirror element: two planes
  static constexpr int G = 2;
  static constexpr int M = 256 / (int)sizeof(V);   // lanes per conflict-free group
#ifdef SQ_NO_PAD
  static constexpr bool PAD = false;
#else
  static constexpr bool PAD = sizeof(V) * (size_t)Lay<NC_, G, M, true>::SIZE + OTHER + uni(1) <= 163840;
#endif
  using L = Lay<NC_, G, M, PAD>;
  static constexpr int MH = NC_ / 2;
  // elements of the cube buffer: the mirror, or the Gram scratch
  static constexpr size_t GEL = (GSCR + sizeof(V) - 1) / sizeof(V);
  static constexpr size_t TLN = GEL > (size_t)L::SIZE ? GEL : (size_t)L::SIZE;
  // copies of the projection sums: lanes of a wave that add to the same
  // image serialise on its LDS words, so lane l adds to copy l mod NCOPY
  // (copies of one image are adjacent, in distinct banks) and the copies
  // are summed after the step; as many as the LDS left over holds (1..8)
  static constexpr size_t USED = sizeof(V) * (size_t)TLN + OTHER;
  static constexpr int NCOPY = USED + uni(8) <= 163840   ? 8
                               : USED + uni(4) <= 163840 ? 4
                               : USED + uni(2) <= 163840 ? 2
                                                         : 1;
  static_assert(USED + uni(NCOPY) <= 163840, "LDS");
};

template <class Vr>
struct Smem {
  using T = typename Vr::T;
  static constexpr int NI = Vr::NIMG;
  typename Vr::V tl[Vr::TLN];          // the mirror (G planes per element), or scratch
  double ix[NI], iy[NI], iz[NI];      // image positions (unwrapped), sorted by z
  double rp2[NI], i2s[NI], gdv[NI];   // r_p^2, 1 / (2 sigma_p^2), gamma dV
  // z factor of each image on the cube planes: e(z) = exp(-u_z^2 i2s) with
  // u_z = u_0 + z h, generated as e(z + 1) = e(z) rr(z), rr(z + 1) = rr(z) cq;
  // rq = (rr(0), cq) (one 16-byte read per slot and step)
  double e0[NI];
  typename Vec2<double>::type rq[NI];
  // rr at the first plane of segments 1 .. NSEG - 1
  double rrs[Vr::NSEG > 1 ? Vr::NSEG - 1 : 1][Vr::NSEG > 1 ? NI : 1];
  double pf[2][NI];                   // projections <chi_I, v>, double-buffered over steps
  double gpf[2][NI];                  // gamma dV <chi_I, v>
  union {
    unsigned long long pint[NI][Vr::NCOPY][2];   // projection sums being formed (copies, two words)
    struct {   // stress pass, after the last step
      unsigned long long nsum[Vr::NEAR][10][2];  // sums over the near images' supports
      double kl[3][3][2 * SQ_FDM + 1];           // G_b = grad_b d on the line through the node along a
    } ep;
  };
  double red[2][2 * 16];              // block sums, double-buffered over steps
  double near_chi[Vr::NEAR];
  int near_img[Vr::NEAR];
  int wcnt[16];
  int nimg, nnear, ngram;
  unsigned item;
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
  int bown;     // LDS element of the column's plane group 0
  // slot s: bit 31 - z set for the planes z of the chord of the image's
  // spherical support on this column; the image index in the low bits
  unsigned sid[Vr::KC];
  // projector value of slot s at (cx, cy) on the first plane the wave visits
  double a0[Vr::AREG ? Vr::KC : 1];
  // wave-uniform segment range of slot s in bits 4(s % 8) of word s / 8:
  // first segment in the low two bits, last segment in the next two
  unsigned segw[Vr::NSEG > 1 ? (Vr::KC + 7) / 8 : 1];
  T vd[Vr::ZH];                       // diagonal of (H_q - shift) without the stencil centre
  // the node's stored Gram entries (global memory, read at every step)
  const double* gvp;
  const unsigned* gip;
  int ngram;
  bool bad;     // a fixed-point term was out of range
};

template <class Vr>
__device__ __forceinline__ double plane0_weight(const Smem<Vr>& S, const Ctx<Vr>& X, const CellDev& C,
                                                int i) {
  constexpr int m = Vr::MH;
  const double dx = node_coord(X.q0 + X.cx - m, C.h, S.ix[i]);
  const double dy = node_coord(X.q1 + X.cy - m, C.h, S.iy[i]);
  return exp(-sq_sum2(dx, dy) * S.i2s[i]) * S.e0[i];
}

template <class Vr>
__device__ __forceinline__ double slot_start(const Smem<Vr>& S, const Ctx<Vr>& X, const CellDev& C,
                                             int s, int i) {
  if constexpr (Vr::AREG) {
    return X.a0[s];
  } else {
    return plane0_weight<Vr>(S, X, C, i);
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

__device__ __forceinline__ unsigned wave_or(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= (unsigned)__shfl_xor((int)v, o);
  return (unsigned)__builtin_amdgcn_readfirstlane((int)v);
}

// Stencil centre of the kinetic operator -1/2 Laplacian (three axes).
__device__ __forceinline__ double node_diag_kinetic(const CellDev& C) {
  return -0.5 / (C.h * C.h) * 3.0 * C.c2[0];
}

// Node prologue: image list of the cube (sorted by z, ties in gather order),
// z-factor constants, per-column chords and projector weights, diagonal,
// projection buffers.  shift is subtracted from the diagonal.
template <class Vr>
__device__ __forceinline__ void node_prologue(const CellDev& C, long long q, double shift,
                                              Smem<Vr>& S, Ctx<Vr>& X, unsigned* err) {
  using T = typename Vr::T;
  using L = typename Vr::L;
  constexpr int NC = Vr::NC;
  constexpr int ZH = Vr::ZH;
  constexpr int NT = Vr::NT;
  constexpr int NI = Vr::NIMG;
  constexpr int m = Vr::MH;
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
  const int found = gather_images<NT, Vr::NW, NI>(C, X.q0, X.q1, X.q2, m, &S.nimg, S.wcnt, store, err);
  const int nimg = found < NI ? found : NI;
  if (tid == 0) S.nimg = nimg;

  // ---- sort by z (rank by (z, gather position)); scratch in the cube buffer ----
  {
    double* scr = reinterpret_cast<double*>(S.tl);   // [6][NI]
    static_assert(sizeof(S.tl) >= 6 * sizeof(double) * NI, "sort scratch");
    for (int t = tid; t < nimg; t += NT) {
      const double zt = S.iz[t];
      int r = 0;
      for (int j = 0; j < nimg; ++j) {
        const double zj = S.iz[j];
        r += (zj < zt || (zj == zt && j < t)) ? 1 : 0;
      }
      scr[r] = S.ix[t];
      scr[NI + r] = S.iy[t];
      scr[2 * NI + r] = zt;
      scr[3 * NI + r] = S.rp2[t];
      scr[4 * NI + r] = S.i2s[t];
      scr[5 * NI + r] = S.gdv[t];
    }
    __syncthreads();
    for (int t = tid; t < nimg; t += NT) {
      S.ix[t] = scr[t];
      S.iy[t] = scr[NI + t];
      S.iz[t] = scr[2 * NI + t];
      S.rp2[t] = scr[3 * NI + t];
      S.i2s[t] = scr[4 * NI + t];
      S.gdv[t] = scr[5 * NI + t];
    }
    __syncthreads();
  }

  // ---- z-factor constants of every image; projections ----
  for (int i = tid; i < NI; i += NT) {
    double e0 = 0.0, r0 = 0.0, cq = 0.0;
    if (i < nimg) {
      const double is = S.i2s[i];
      const double u0 = node_coord(X.q2 - m, h, S.iz[i]);
      e0 = exp(-(u0 * u0) * is);
      r0 = exp(-(2.0 * u0 * h + h * h) * is);
      cq = exp(-2.0 * h * h * is);
    }
    S.e0[i] = e0;
    S.rq[i] = typename Vec2<double>::type{r0, cq};
    if constexpr (Vr::NSEG > 1) {
#pragma unroll
      for (int k = 1; k < Vr::NSEG; ++k) {
        double rk = 0.0;
        if (i < nimg) {
          const double uk = node_coord(X.q2 + Vr::seg_lo(k) - m, h, S.iz[i]);
          rk = exp(-(2.0 * uk * h + h * h) * S.i2s[i]);
        }
        S.rrs[k - 1][i] = rk;
      }
    }
    S.pf[0][i] = 0.0;
    S.pf[1][i] = 0.0;
    S.gpf[0][i] = 0.0;
    S.gpf[1][i] = 0.0;
#pragma unroll
    for (int c = 0; c < Vr::NCOPY; ++c) {
      S.pint[i][c][0] = 0ull;
      S.pint[i][c][1] = 0ull;
    }
  }
  for (int i = tid; i < (int)Vr::TLN; i += NT) S.tl[i] = typename Vr::V{};
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
          if constexpr (Vr::AREG) {
            // with segments: the xy factor here, the z factor below
            X.a0[s] = Vr::NSEG > 1 ? exp(-dxy2 * S.i2s[i]) : exp(-dxy2 * S.i2s[i]) * S.e0[i];
          }
        }
      }
      ++X.nslot;
    }
  }
  X.nsw = wave_max(X.nslot);
  if constexpr (Vr::NSEG > 1) {
    constexpr unsigned IMASK = (1u << Vr::IBITS) - 1u;
#pragma unroll
    for (int w = 0; w < (Vr::KC + 7) / 8; ++w) X.segw[w] = 0u;
#pragma unroll
    for (int s = 0; s < Vr::KC; ++s) {
      // planes touched by slot s on any lane of the wave (bit 31 - z)
      const unsigned u = wave_or(X.sid[s] & ~IMASK);
      int kf = 0, kl = 0;
      if (u != 0u) {
        const int zf = __clz((int)u), zl = 31 - __builtin_ctz(u);
#pragma unroll
        for (int k = 1; k < Vr::NSEG; ++k) {
          if (zf >= Vr::seg_lo(k)) kf = k;
          if (zl >= Vr::seg_lo(k)) kl = k;
        }
      }
      X.segw[s / 8] |= (unsigned)(kf | (kl << 2)) << (4 * (s % 8));
      if (s < X.nslot) {
        const int i = (int)(X.sid[s] & IMASK);
        double e = S.e0[i];
        if (kf > 0) {
          const double uk = node_coord(X.q2 + Vr::seg_lo(kf) - m, h, S.iz[i]);
          e = exp(-(uk * uk) * S.i2s[i]);
        }
        X.a0[s] *= e;
      }
    }
  }

  // ---- diagonal: local potential (periodic) + stencil centre - shift ----
  const double cdiag = node_diag_kinetic(C);
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
  X.bown = L::at(X.cx, X.cy, 0);
  X.gvp = nullptr;
  X.gip = nullptr;
  X.ngram = 0;
  X.bad = false;
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

// Projector weights of one slot along the column: w(z) = a e(z)/e(0)
// on the planes of the chord, zero elsewhere.  f(z, on, w) is called for
// every plane.
template <int ZH, class F>
__device__ __forceinline__ void slot_sweep(unsigned mk, double a, typename Vec2<double>::type rq, F f) {
  double rr = rq.x;
  const double cq = rq.y;
#pragma unroll
  for (int z = 0; z < ZH; ++z) {
    unsigned nm;
    const bool on = __builtin_add_overflow(mk, mk, &nm);   // bit 31 - z
    mk = nm;
    const double an = a * rr;   // before the use: a's registers then hold the weight
    rr *= cq;
    f(z, on, a);
    a = an;
  }
}

// Weights of slot s (image i, slot word mk, weight a on the first plane
// visited) along the column, over the segments the wave visits for it:
// f(z, on, w) is called for every plane of those segments.
template <class Vr, class F>
__device__ __forceinline__ void sweep(const Smem<Vr>& S, const Ctx<Vr>& X, int s, int i, unsigned mk,
                                      double a, F f) {
  const typename Vec2<double>::type rq = S.rq[i];
  if constexpr (Vr::NSEG == 1) {
    slot_sweep<Vr::ZH>(mk, a, rq, f);
  } else {
    const unsigned code = (X.segw[s / 8] >> (4 * (s % 8))) & 15u;   // uniform
    const int kf = (int)(code & 3u), kl = (int)(code >> 2);
    double rr = rq.x;
    const double cq = rq.y;
    if (kf > 0) {
      rr = S.rrs[kf - 1][i];
      mk <<= Vr::seg_lo(kf);
    }
#pragma unroll
    for (int k = 0; k < Vr::NSEG; ++k) {
      if (k >= kf && k <= kl) {
#pragma unroll
        for (int z = Vr::seg_lo(k); z < Vr::seg_lo(k + 1); ++z) {
          unsigned nm;
          const bool on = __builtin_add_overflow(mk, mk, &nm);   // bit 31 - z
          mk = nm;
          const double an = a * rr;
          rr *= cq;
          f(z, on, a);
          a = an;
        }
      }
    }
  }
}

// Projections <chi_I, v> of the vector v held in registers, added to
// S.pint (the caller places a barrier before they are read).
template <class Vr>
__device__ __forceinline__ void project(Smem<Vr>& S, Ctx<Vr>& X, const CellDev& C,
                                        const typename Vr::T (&v)[Vr::ZH]) {
  using T = typename Vr::T;
  constexpr unsigned IMASK = (1u << Vr::IBITS) - 1u;
  slot_for<Vr::KC>([&](auto si) __attribute__((always_inline)) {
    const int s = si;
    if (s < X.nsw) {
      const unsigned mk = X.sid[s];
      const int i = (int)(mk & IMASK);
      T part = (T)0;
      sweep<Vr>(S, X, s, i, mk, slot_start<Vr>(S, X, C, s, i),
                [&](int z, bool on, double a) { part += chord_weight<T>(on, a) * v[z]; });
      // a slot past the thread's count has sid 0 and weight zero: it adds 0 to image 0
      fx_add(S.pint[i][threadIdx.x & (Vr::NCOPY - 1)], (double)part, X.bad);
    }
  });
}

// After the barrier that ends a step: the new projections
// pf[par ^ 1] = (sum - alpha pf[par]) * ib from the integer sums, which are
// cleared for the next step (the caller places a barrier before either is
// used again).
template <class Vr>
__device__ __forceinline__ void finish_proj(Smem<Vr>& S, int par, double alpha = 0.0, double ib = 1.0) {
  for (int i = threadIdx.x; i < Vr::NIMG; i += Vr::NT) {
    unsigned long long hi = 0ull, lo = 0ull;
#pragma unroll
    for (int c = 0; c < Vr::NCOPY; ++c) {
      hi += S.pint[i][c][0];
      lo += S.pint[i][c][1];
      S.pint[i][c][0] = 0ull;
      S.pint[i][c][1] = 0ull;
    }
    double v = fx_join((long long)hi, (long long)lo);
    if (alpha != 0.0) v -= alpha * S.pf[par][i];
    v *= ib;
    S.pf[par ^ 1][i] = v;
    S.gpf[par ^ 1][i] = S.gdv[i] * v;
  }
}

// One application of the nodal operator to the vector held in registers
// (cur) and mirrored in S.tl:
//   io <- sc * ((H_q - shift) cur) - pm * io + cw w_q
// io holds the previous vector on entry and the new one on exit (registers
// only; the caller mirrors it).
//
// Projections: S.pf[par] holds <chi_I, cur> on entry and S.pint is zero; on
// exit S.pint holds the integer sums of <chi_I, io>.  FUSED: they come out
// of the same sweep that adds the projector terms c_I chi_I, c_I = sc gamma
// dV <chi_I, cur>: every thread visits its images in increasing index, and
// the projection onto chi_I is taken before the thread adds c_I chi_I, so
// the sweep yields <chi_I, u> + sum_{J < I} c_J G_IJ (u the stencil part of
// io, G the Gram matrix of the projectors over the cube); the missing
// sum_{J >= I} G_IJ c_J is added from the stored upper triangle.  Otherwise
// (a cube whose Gram matrix exceeds its capacity) a second sweep projects
// the finished io.  Ends after one block barrier; the caller then forms
// S.pf[par ^ 1] with finish_proj.
template <class Vr, bool FUSED>
__device__ __forceinline__ void apply_step(Smem<Vr>& S, Ctx<Vr>& X, const CellDev& C,
                                           const typename Vr::T (&cur)[Vr::ZH],
                                           typename Vr::T (&io)[Vr::ZH], const typename Vr::T* ck,
                                           double sc, typename Vr::T pm, int par, double cw = 0.0) {
  using T = typename Vr::T;
  using L = typename Vr::L;
  constexpr int ZH = Vr::ZH;
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
    // (1) the upper-triangle Gram terms of the new projections (entries from
    // global memory, cached: the same few kilobytes at every step); a
    // thread past the count adds zero to image 0
    const int ng = X.ngram;
    if (ng > 0) {
#pragma unroll
      for (int e = 0; e < Vr::GPT; ++e) {
        const int k = threadIdx.x + e * Vr::NT;
        if (e * Vr::NT < ng) {   // uniform
          const bool in = k < ng;
          const int kk = in ? k : ng - 1;
          const double gval = X.gvp[kk];
          const unsigned ij = in ? X.gip[kk] : 0u;
          const int i = (int)(ij & 0xffffu), j = (int)(ij >> 16);
          fx_add(S.pint[i][threadIdx.x & (Vr::NCOPY - 1)], in ? gval * (sc * S.gpf[par][j]) : 0.0, X.bad);
        }
      }
    }
  }
  // (2) stencil + diagonal on the own planes (x/y neighbours from LDS, G
  // planes per read; z neighbours from registers)
  if (X.active) {
    using V = typename Vr::V;
    constexpr int G = Vr::G;
    const T tsc = (T)sc;
#pragma unroll
    for (int zg = 0; zg < L::NZG; ++zg) {
      T acc[G];
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int z = zg * G + u;
        acc[u] = z < ZH ? X.vd[z] * cur[z] : (T)0;
      }
      const V* pc = S.tl + X.bown + zg * L::PL;
#pragma unroll
      for (int k = 1; k <= SQ_FDM; ++k) {
        V h;
        if constexpr (L::RS > Vr::NC) {
          h = (pc[k] + pc[-k]) + (pc[k * L::RS] + pc[-k * L::RS]);
        } else {
          h = V{};
          if (X.cx + k < Vr::NC) h += pc[k];
          if (X.cx - k >= 0) h += pc[-k];
          if (X.cy + k < Vr::NC) h += pc[k * L::RS];
          if (X.cy - k >= 0) h += pc[-k * L::RS];
        }
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const int z = zg * G + u;
          if (z < ZH) {
            T s = (T)0;
            if (z + k < ZH) s += cur[z + k];
            if (z - k >= 0) s += cur[z - k];
            s += h[u];
            acc[u] += ck[k] * s;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int z = zg * G + u;
        if (z < ZH) io[z] = tsc * acc[u] - pm * io[z];
      }
    }
    // optional cw w_q (the unit vector at the node): part of the vector the
    // projector terms are added to, and of its projections
    if (X.cx == Vr::MH && X.cy == Vr::MH) io[Vr::MH] += (T)cw;
  }
  if constexpr (FUSED) {
    // (3) one sweep per image: projection of io, then the projector term
    // (a slot past the thread's count has sid 0: weight zero, image 0)
    slot_for<Vr::KC>([&](auto si) __attribute__((always_inline)) {
      const int s = si;
      if (s < nsw) {
        const unsigned mk = X.sid[s];
        const int i = (int)(mk & IMASK);
        const T coef = (T)(sc * S.gpf[par][i]);
        T part = (T)0;
        sweep<Vr>(S, X, s, i, mk, slot_start<Vr>(S, X, C, s, i), [&](int z, bool on, double a) {
          const T w = chord_weight<T>(on, a);
          part += w * io[z];
          io[z] += w * coef;
        });
        fx_add(S.pint[i][threadIdx.x & (Vr::NCOPY - 1)], (double)part, X.bad);
      }
    });
  } else {
    // (3') the projector terms, then the projections of the finished io
    slot_for<Vr::KC>([&](auto si) __attribute__((always_inline)) {
      const int s = si;
      if (s < nsw) {
        const unsigned mk = X.sid[s];
        const int i = (int)(mk & IMASK);
        const double coef = s < X.nslot ? sc * S.gpf[par][i] : 0.0;
        sweep<Vr>(S, X, s, i, mk, coef * slot_start<Vr>(S, X, C, s, i),
                  [&](int z, bool on, double a) { io[z] += chord_weight<T>(on, a); });
      }
    });
    project<Vr>(S, X, C, io);
  }
  __syncthreads();
}

// Mirror the thread's planes into LDS (the caller places a barrier before
// they are read).
template <class Vr>
__device__ __forceinline__ void mirror(Smem<Vr>& S, const Ctx<Vr>& X, const typename Vr::T (&v)[Vr::ZH]) {
  using L = typename Vr::L;
  using V = typename Vr::V;
  constexpr int G = Vr::G;
  if (X.active) {
#pragma unroll
    for (int zg = 0; zg < L::NZG; ++zg) {
      V e;
#pragma unroll
      for (int u = 0; u < G; ++u) e[u] = zg * G + u < Vr::ZH ? v[zg * G + u] : (typename Vr::T)0;
      S.tl[X.bown + zg * L::PL] = e;
    }
  }
}

// cur = cw w_q (the unit vector at the node scaled by cw), prv = 0; mirrored;
// its projections in S.pf[0].
template <class Vr>
__device__ __forceinline__ void load_unit(Smem<Vr>& S, Ctx<Vr>& X, const CellDev& C,
                                          typename Vr::T (&cur)[Vr::ZH], typename Vr::T (&prv)[Vr::ZH],
                                          double cw = 1.0) {
  using T = typename Vr::T;
  constexpr int m = Vr::MH;
#pragma unroll
  for (int z = 0; z < Vr::ZH; ++z) {
    cur[z] = (X.active && X.cx == m && X.cy == m && z == m) ? (T)cw : (T)0;
    prv[z] = (T)0;
  }
  mirror<Vr>(S, X, cur);
  project<Vr>(S, X, C, cur);
  __syncthreads();
  finish_proj<Vr>(S, 1);   // S.pf[0]
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ void stencil_coefs(const CellDev& C, T* ck) {
  // read from the cell table (uniform: the values stay in scalar registers)
#pragma unroll
  for (int k = 0; k <= SQ_FDM; ++k) ck[k] = sizeof(T) == 8 ? (T)C.ck[k] : (T)C.ckf[k];
}

// Block sums of two values in a fixed order; red is double-buffered by the
// caller (the next use of the same buffer is separated by at least one more
// barrier).
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

// Nodes of one launch: one workgroup per node, or (PERSIST) a persistent
// grid whose workgroups take node indices from the counter until the list
// is exhausted.  f(g, cell) processes the node (one call site, so that the
// node body is inlined: a called function would keep its arrays in scratch
// memory); the loop places a barrier before the next node's prologue.
// (a template parameter: a loop around the node body changes the register
// allocation of the whole kernel, so the one-node form has no loop)
template <class Vr, bool PERSIST, class F>
__device__ __forceinline__ void for_nodes(Smem<Vr>& S, const long long* items, const int* item_cell,
                                          long long nitems, unsigned* counter, F f) {
  if constexpr (!PERSIST) {
    f(items[blockIdx.x], item_cell[blockIdx.x]);
  } else {
    for (;;) {
      __syncthreads();
      if (threadIdx.x == 0) S.item = atomicAdd(counter, 1u);
      __syncthreads();
      const long long it = (long long)S.item;
      if (it >= nitems) break;
      f(items[it], item_cell[it]);
    }
  }
}

// ---------------------------------------------------------------------------
// Gram matrix of the projectors over the cube, G_IJ = <chi_I, chi_J> for
// I <= J, restricted to the pairs whose chords share a plane on some column
// (every other entry is zero).  Built once per node at set-up from the same
// chords and weights the sweeps use, and stored for the recurrence kernels,
// which hold the entries in registers.  A cube with more than GCAP such
// pairs gets the count -1, and its steps take two sweeps (projector terms,
// then projections).  The entries are exact integer sums of the per-point
// products (rounded to 2^-81), so they do not depend on how the cube is
// split among threads.  Uses the cube buffer as scratch; the caller clears it
// afterwards.
// ---------------------------------------------------------------------------
template <class Vr>
__device__ void gram_build(Smem<Vr>& S, const Ctx<Vr>& X, const CellDev& C, unsigned* err) {
  constexpr int ZH = Vr::ZH;
  constexpr int NI = Vr::NIMG;
  constexpr int NWD = Vr::NWD;
  constexpr int NT = Vr::NT;
  constexpr int CAP = Vr::GCAP;
  constexpr unsigned IMASK = (1u << Vr::IBITS) - 1u;
  static_assert(sizeof(S.tl) >= Vr::GSCR, "Gram scratch");
  unsigned* bm = reinterpret_cast<unsigned*>(S.tl);            // [NI][NWD] pairs present
  int* rs = reinterpret_cast<int*>(bm + NI * NWD);              // [NI + 1] first entry of each row
  unsigned* sl = reinterpret_cast<unsigned*>(rs + NI + 1);      // [KC][NT] slot words
  unsigned long long* ga = reinterpret_cast<unsigned long long*>(
      reinterpret_cast<char*>(S.tl) + ((4 * ((size_t)NI * NWD + NI + 1 + (size_t)Vr::KC * NT) + 15) & ~(size_t)15));
  const int tid = threadIdx.x;
  for (int k = tid; k < NI * NWD; k += NT) bm[k] = 0u;
#pragma unroll
  for (int s = 0; s < Vr::KC; ++s) sl[s * NT + tid] = X.sid[s];
  __syncthreads();
  // pairs of this thread's slots (image indices increase with the slot)
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
  for (int r = tid; r < NI; r += NT) {   // row counts (every row, whatever the block size)
    int c = 0;
#pragma unroll
    for (int w = 0; w < NWD; ++w) c += __popc(bm[r * NWD + w]);
    rs[r] = c;
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
  const bool fits = total <= CAP;
  if (fits)
    for (int e = tid; e < 2 * total; e += NT) ga[e] = 0ull;
  __syncthreads();
  // column sums of chi_I chi_J over the shared planes, point by point
  if (X.active && fits) {
    constexpr int m = Vr::MH;
    const double h = C.h;
    for (int s = 0; s < X.nslot; ++s) {
      const unsigned a = sl[s * NT + tid];
      const int i = (int)(a & IMASK);
      const double wi = exp(-sq_sum2(node_coord(X.q0 + X.cx - m, h, S.ix[i]),
                                     node_coord(X.q1 + X.cy - m, h, S.iy[i])) * S.i2s[i]) *
                        S.e0[i];
      for (int s2 = s; s2 < X.nslot; ++s2) {
        const unsigned b = sl[s2 * NT + tid];
        if ((a & b & ~IMASK) == 0u) continue;
        const int j = (int)(b & IMASK);
        const double wj = exp(-sq_sum2(node_coord(X.q0 + X.cx - m, h, S.ix[j]),
                                       node_coord(X.q1 + X.cy - m, h, S.iy[j])) * S.i2s[j]) *
                          S.e0[j];
        double ai = wi, ri = S.rq[i].x, aj = wj, rj = S.rq[j].x;
        const double qi = S.rq[i].y, qj = S.rq[j].y;
        long long shi = 0, slo = 0;
        unsigned mk = a & b & ~IMASK;
#pragma unroll
        for (int z = 0; z < ZH; ++z) {
          unsigned nm;
          const bool on = __builtin_add_overflow(mk, mk, &nm);
          mk = nm;
          if (on) {
            long long th, tlw;
            fx_split(ai * aj, th, tlw);
            shi += th;
            slo += tlw;
          }
          ai *= ri;
          ri *= qi;
          aj *= rj;
          rj *= qj;
        }
        const int jw = j >> 5;
        int idx = rs[i] + __popc(bm[i * NWD + jw] & ((1u << (j & 31)) - 1u));
        for (int w = 0; w < jw; ++w) idx += __popc(bm[i * NWD + w]);
        if (idx >= 0 && idx < total) {
          atomicAdd(&ga[2 * idx], (unsigned long long)shi);
          atomicAdd(&ga[2 * idx + 1], (unsigned long long)slo);
        } else {
          atomicOr(err, SQ_ERR_IMAGES);
        }
      }
    }
  }
  __syncthreads();
  // entry order (I, J): rows in order, J increasing within a row
  if (fits) {
    unsigned* gidx = reinterpret_cast<unsigned*>(rs + NI + 1);   // reuses the slot words
    for (int r = tid; r < NI; r += NT) {
      int e = rs[r];
      for (int w = 0; w < NWD; ++w) {
        unsigned bits = bm[r * NWD + w];
        while (bits) {
          const int b = __ffs(bits) - 1;
          bits &= bits - 1u;
          if (e < total) gidx[e] = (unsigned)r | ((unsigned)(32 * w + b) << 16);
          ++e;
        }
      }
    }
  }
  if (!fits && tid == 0) S.ngram = -1;   // the steps then take two sweeps
  __syncthreads();
}

template <class Vr>
__device__ __forceinline__ void gram_store(Smem<Vr>& S, const PlanDev& P, long long g) {
  constexpr int NI = Vr::NIMG;
  constexpr int NWD = Vr::NWD;
  const int ng = min(max(S.ngram, -1), Vr::GCAP);
  const int* rs = reinterpret_cast<const int*>(reinterpret_cast<const unsigned*>(S.tl) + NI * NWD);
  const unsigned* gidx = reinterpret_cast<const unsigned*>(rs + NI + 1);
  const unsigned long long* ga = reinterpret_cast<const unsigned long long*>(
      reinterpret_cast<const char*>(S.tl) +
      ((4 * ((size_t)NI * NWD + NI + 1 + (size_t)Vr::KC * Vr::NT) + 15) & ~(size_t)15));
  for (int e = threadIdx.x; e < ng; e += Vr::NT) {
    P.gval[g * SQ_GRAM_MAX + e] = fx_join((long long)ga[2 * e], (long long)ga[2 * e + 1]);
    P.gidx[g * SQ_GRAM_MAX + e] = gidx[e];
  }
  if (threadIdx.x == 0) P.gn[g] = ng;
}

// The node's stored Gram entries: thread t uses entries t + e NT at every
// step.  A count over the variant's capacity (the host never launches such
// a node on the single-sweep form) uses none.
template <class Vr>
__device__ __forceinline__ void gram_load(Ctx<Vr>& X, const PlanDev& P, long long g) {
  const int ng = P.gn[g];
  X.ngram = (ng >= 0 && ng <= Vr::GCAP) ? ng : 0;
  X.gvp = P.gval + g * SQ_GRAM_MAX;
  X.gip = P.gidx + g * SQ_GRAM_MAX;
}

// End of a node: report fixed-point terms that were out of range.
template <class Vr>
__device__ __forceinline__ void node_epilogue(const Ctx<Vr>& X, unsigned* err) {
  if (X.bad) atomicOr(err, SQ_ERR_RANGE);
}

// ---------------------------------------------------------------------------
// Spectral bounds: K-step FP64 Lanczos on H_q from the unit vector w_q
// (chi_q and zeta_q come from the extreme eigenvalues of H_q, Sec. IV)
// ---------------------------------------------------------------------------
// One Lanczos step with v_k in A (and S.tl), v_{k-1} in B on entry; on exit
// v_{k+1} is in B (and S.tl) unless the recursion stopped.  The operator is
// H_q - sigma (the node's diagonal entry, sigma = alpha_1): the same Krylov
// space and couplings, alpha shifted by sigma, which is added back.  The
// projections of v_{k+1} are (proj(H v_k - beta v_{k-1}) - alpha_k
// proj(v_k)) / beta_k, so an error in proj(v_k) returns multiplied by
// alpha_k / beta_k; unshifted that factor is about 2 at every step (errors
// grow 1e5-fold in 20 steps, 1e11-fold in 40), shifted it stays below one.
template <class Vr, bool FUSED>
__device__ __forceinline__ bool lanczos_step(Smem<Vr>& S, Ctx<Vr>& X, const CellDev& C,
                                             const double (&A)[Vr::ZH], double (&B)[Vr::ZH],
                                             const double* ck, int k, double& bprev, double& tol,
                                             double* lan, double sigma) {
  constexpr int ZH = Vr::ZH;
  constexpr int NW = Vr::NW;
  apply_step<Vr, FUSED>(S, X, C, A, B, ck, 1.0, bprev, k & 1);   // B = (H - sigma) v_k - beta v_{k-1}
  // alpha = <v_k, B> and |B|^2 in one block sum: |B - alpha v_k|^2 =
  // |B|^2 - alpha^2 for a unit v_k.  With the shift alpha is not large
  // against beta, so the difference keeps its accuracy; where it cancels
  // (beta^2 < 1e-4 |B|^2, near an invariant subspace) the residual's norm
  // is summed directly.
  double a = 0.0, bb = 0.0;
#pragma unroll
  for (int z = 0; z < ZH; ++z) {
    a += A[z] * B[z];
    bb += B[z] * B[z];
  }
  block_sum2_db<NW>(a, bb, S.red[0]);
  double b = bb - a * a;
#pragma unroll
  for (int z = 0; z < ZH; ++z) B[z] -= a * A[z];
  if (!(b > 1e-4 * bb)) {   // uniform
    double dum = 0.0;
    b = 0.0;
#pragma unroll
    for (int z = 0; z < ZH; ++z) b += B[z] * B[z];
    block_sum2_db<NW>(b, dum, S.red[1]);
  }
  b = sqrt(b);
  if (threadIdx.x == 0) {
    lan[k] = a + sigma;
    lan[SQ_KL_MAX + k] = b;
  }
  if (k == 0) tol = 1e-14 * (fabs(a + sigma) + b);
  if (b < tol) return false;
  const double ib = 1.0 / b;
#pragma unroll
  for (int z = 0; z < ZH; ++z) B[z] *= ib;
  mirror<Vr>(S, X, B);
  // projections of v_{k+1} = (H v_k - beta v_{k-1} - a v_k) / b
  finish_proj<Vr>(S, k & 1, a, ib);
  bprev = b;
  __syncthreads();
  return true;
}

template <class Vr, bool FUSED, bool PERSIST>
__global__ void __launch_bounds__(Vr::NT) k_lanczos(PlanDev P, const long long* items,
                                                     const int* item_cell, long long nitems,
                                                     unsigned* counter) {
  static_assert(sizeof(typename Vr::T) == 8, "Lanczos runs in FP64");
  constexpr int ZH = Vr::ZH;
  __shared__ Smem<Vr> S;
  for_nodes<Vr, PERSIST>(S, items, item_cell, nitems, counter, [&](long long g, int ci) __attribute__((always_inline)) {
    const CellDev& C = P.cells[ci];
    const long long q = g - C.node_base;
    // the diagonal entry of H_q at the node (the prologue's diagonal there)
    const double sigma = C.vloc[q] + node_diag_kinetic(C);
    Ctx<Vr> X;
    node_prologue<Vr>(C, q, sigma, S, X, P.err);
    if constexpr (FUSED) gram_load<Vr>(X, P, g);
    double ck[SQ_FDM + 1];
    stencil_coefs<double>(C, ck);
    double A[ZH], B[ZH];
    load_unit<Vr>(S, X, C, A, B);
    double bprev = 0.0, tol = 0.0;
    int steps = 0;
    double* lan = P.lan + g * (2 * SQ_KL_MAX);
    for (int k = 0; k < C.krun; k += 2) {
      steps = k + 1;
      if (!lanczos_step<Vr, FUSED>(S, X, C, A, B, ck, k, bprev, tol, lan, sigma)) break;
      if (k + 1 >= C.krun) break;
      steps = k + 2;
      if (!lanczos_step<Vr, FUSED>(S, X, C, B, A, ck, k + 1, bprev, tol, lan, sigma)) break;
    }
    if (threadIdx.x == 0) P.lan_steps[g] = steps;
    node_epilogue<Vr>(X, P.err);
  });
}

// Set-up pass: the Gram matrix of every node's projectors (count -1 when it
// exceeds the capacity; such nodes are launched with FUSED = false).
template <class Vr>
__global__ void __launch_bounds__(Vr::NT) k_gram(PlanDev P, const long long* items,
                                                  const int* item_cell) {
  static_assert(sizeof(typename Vr::T) == 8, "the Gram build runs in FP64");
  __shared__ Smem<Vr> S;
  const long long g = items[blockIdx.x];
  const CellDev& C = P.cells[item_cell[blockIdx.x]];
  const long long q = g - C.node_base;
  Ctx<Vr> X;
  node_prologue<Vr>(C, q, 0.0, S, X, P.err);
  gram_build<Vr>(S, X, C, P.err);
  gram_store<Vr>(S, P, g);
}

// ---------------------------------------------------------------------------
// Chebyshev moments rho_q^j = w_q^T T_j(Hhat_q) w_q, j = 0..npl, from the
// three-term recurrence (Sec. IV) taken to degree ceil(npl/2) with
//   rho^{2k} = 2 <t^k, t^k> - rho^0,  rho^{2k+1} = 2 <t^{k+1}, t^k> - rho^1
// (Hhat_q is symmetric, T_{a+b} + T_{|a-b|} = 2 T_a T_b).
// ---------------------------------------------------------------------------
template <class Vr, bool FUSED, bool PERSIST>
__global__ void __launch_bounds__(Vr::NT) k_moments(PlanDev P, const long long* items,
                                                     const int* item_cell, long long nitems,
                                                     unsigned* counter) {
  using T = typename Vr::T;
  constexpr int ZH = Vr::ZH;
  constexpr int NW = Vr::NW;
  __shared__ Smem<Vr> S;
  for_nodes<Vr, PERSIST>(S, items, item_cell, nitems, counter, [&](long long g, int ci) __attribute__((always_inline)) {
    const CellDev& C = P.cells[ci];
    const long long q = g - C.node_base;
    const double chi = P.bnd[4 * g + 2], zeta = P.bnd[4 * g + 3];
    Ctx<Vr> X;
    node_prologue<Vr>(C, q, chi, S, X, P.err);
    if constexpr (FUSED) gram_load<Vr>(X, P, g);
    T ck[SQ_FDM + 1];
    stencil_coefs<T>(C, ck);
    T A[ZH], B[ZH];
    load_unit<Vr>(S, X, C, A, B);
    double* mom = P.mom + g * P.mstride;
    const int npl = C.npl;
    const int kmax = (npl + 1) / 2;
    double rho1 = 0.0;
    bool bad = false;
    if (threadIdx.x == 0) mom[0] = 1.0;
    // t^{k+1} from t^k (cur) and t^{k-1} (io); then rho^{2k+1}, rho^{2k+2}
    auto step = [&](const T (&cur)[ZH], T (&io)[ZH], int k) {
      apply_step<Vr, FUSED>(S, X, C, cur, io, ck, k == 0 ? 1.0 / zeta : 2.0 / zeta,
                            k == 0 ? (T)0 : (T)1, k & 1);
      double sq = 0.0, cr = 0.0;
#pragma unroll
      for (int z = 0; z < ZH; ++z) {
        const double a = (double)io[z], b = (double)cur[z];
        sq += a * a;
        cr += a * b;
      }
      mirror<Vr>(S, X, io);
      finish_proj<Vr>(S, k & 1);
      block_sum2_db<NW>(sq, cr, S.red[k & 1]);
      if (k == 0) rho1 = cr;
      const int j1 = 2 * k + 1, j2 = 2 * k + 2;
      const double r1 = (k == 0) ? cr : 2.0 * cr - rho1;
      const double r2 = 2.0 * sq - 1.0;
      // |rho^j| <= 1 when the bounds hold: 1e-6 slack for FP64 rounding, 1e-4
      // for FP32 vectors (their rounding reaches 1e-6 near |rho^j| = 1)
      constexpr double btol = sizeof(T) == 8 ? 1e-6 : 1e-4;
      if (!(fabs(r1) <= 1.0 + btol) || (j2 <= npl && !(fabs(r2) <= 1.0 + btol))) bad = true;
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
    node_epilogue<Vr>(X, P.err);
  });
}

// ---------------------------------------------------------------------------
// Stress pass: recurrence again with the coefficients known, the DM column
// d_q = sum'_j c_q^j t^j, then the kinetic functional
// K_ab = 2 (grad_a grad_b d_q)_q and the nonlocal functional
// N_ab = -2 sum_I gamma dV chi_I(x_q) [delta_ab chi_I^T d_q
//        + 2 sum_y chi_I(y) (y_b - R_Ib) (grad_a d_q)(y)]   (Sec. IV)
// ---------------------------------------------------------------------------
// One round of the gradient along x (dir 0) or y (dir 1) of the vector
// part, mirrored in LDS: g[z] += sum_k w_k (part(+k) - part(-k)) on the own
// planes (unscaled by 1/h).  Two barriers.
template <class Vr>
__device__ __forceinline__ void grad_round(Smem<Vr>& S, Ctx<Vr>& X, const typename Vr::T (&part)[Vr::ZH],
                                           double (&g)[Vr::ZH], const double* w, int dir) {
  using T = typename Vr::T;
  using L = typename Vr::L;
  using V = typename Vr::V;
  constexpr int G = Vr::G;
  mirror<Vr>(S, X, part);
  __syncthreads();
  if (X.active) {
    const int st = dir == 0 ? 1 : L::RS;
    const int pos = dir == 0 ? X.cx : X.cy;
#pragma unroll
    for (int zg = 0; zg < L::NZG; ++zg) {
      const V* pc = S.tl + X.bown + zg * L::PL;
      double a[G];
#pragma unroll
      for (int u = 0; u < G; ++u) a[u] = 0.0;
#pragma unroll
      for (int k = 1; k <= SQ_FDM; ++k) {
        if constexpr (L::RS > Vr::NC) {
          const V p = pc[k * st], q = pc[-k * st];
#pragma unroll
          for (int u = 0; u < G; ++u) a[u] += w[k] * ((double)p[u] - (double)q[u]);
        } else {
          if (pos + k < Vr::NC) {
            const V p = pc[k * st];
#pragma unroll
            for (int u = 0; u < G; ++u) a[u] += w[k] * (double)p[u];
          }
          if (pos - k >= 0) {
            const V q = pc[-k * st];
#pragma unroll
            for (int u = 0; u < G; ++u) a[u] -= w[k] * (double)q[u];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < G; ++u)
        if (zg * G + u < Vr::ZH) g[zg * G + u] += a[u];
    }
  }
  __syncthreads();
}

// Gradient along z of the FP64 column d (registers; neighbours outside the
// cube dropped).
template <class Vr>
__device__ __forceinline__ void grad_z(const Ctx<Vr>& X, const double (&d)[Vr::ZH], double (&g)[Vr::ZH],
                                       const double* w, double ih) {
  constexpr int ZH = Vr::ZH;
#pragma unroll
  for (int z = 0; z < ZH; ++z) {
    double a = 0.0;
#pragma unroll
    for (int k = 1; k <= SQ_FDM; ++k) {
      double up = 0.0, dn = 0.0;
      if (z + k < ZH) up = d[z + k];
      if (z - k >= 0) dn = d[z - k];
      a += w[k] * (up - dn);
    }
    g[z] = X.active ? a * ih : 0.0;
  }
}

// Nonlocal sums over the supports of the near images, for the thread's
// slots whose image is near: DIR = -1: sum chi d (into term 0); DIR = a:
// sum chi (y_b - R_b) (grad_a d) for b = 0..2 (terms 1 + 3a + b).
template <class Vr, int DIR>
__device__ __forceinline__ void near_sums(Smem<Vr>& S, Ctx<Vr>& X, const CellDev& C,
                                          const double (&v)[Vr::ZH]) {
  constexpr int m = Vr::MH;
  constexpr unsigned IMASK = (1u << Vr::IBITS) - 1u;
  const int nnear = S.nnear;
  if (!X.active || nnear == 0) return;
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
        double acc[3] = {0.0, 0.0, 0.0};
        // once per node: the whole column from plane 0
        slot_sweep<Vr::ZH>(mk, plane0_weight<Vr>(S, X, C, i), S.rq[i],
                           [&](int z, bool on, double chiv) {
                             if (on) {
                               if constexpr (DIR < 0) {
                                 acc[0] += chiv * v[z];
                               } else {
                                 const double rz = (double)(X.q2 + z - m) * C.h - S.iz[i];
                                 const double cg = chiv * v[z];
                                 acc[0] += cg * rx;
                                 acc[1] += cg * ry;
                                 acc[2] += cg * rz;
                               }
                             }
                           });
        if constexpr (DIR < 0) {
          fx_add(S.ep.nsum[nidx][0], acc[0], X.bad);
        } else {
#pragma unroll
          for (int b = 0; b < 3; ++b) fx_add(S.ep.nsum[nidx][1 + 3 * DIR + b], acc[b], X.bad);
        }
      }
    }
  }
}

template <class Vr, bool FUSED, bool PERSIST>
__global__ void __launch_bounds__(Vr::NT) k_stress(PlanDev P, const long long* items,
                                                    const int* item_cell, long long nitems,
                                                    unsigned* counter) {
  using T = typename Vr::T;
  constexpr int NC = Vr::NC;
  constexpr int ZH = Vr::ZH;
  constexpr int NC2 = NC * NC;
  constexpr int m = Vr::MH;
  constexpr unsigned IMASK = (1u << Vr::IBITS) - 1u;
  __shared__ Smem<Vr> S;
  for_nodes<Vr, PERSIST>(S, items, item_cell, nitems, counter, [&](long long g, int ci) __attribute__((always_inline)) {
    const CellDev& C = P.cells[ci];
    const long long q = g - C.node_base;
    const double chi = P.bnd[4 * g + 2], zeta = P.bnd[4 * g + 3];
    const double* coef = P.coef + g * P.mstride;
    Ctx<Vr> X;
    node_prologue<Vr>(C, q, chi, S, X, P.err);
    if constexpr (FUSED) gram_load<Vr>(X, P, g);
    T ck[SQ_FDM + 1];
    stencil_coefs<T>(C, ck);
    T A[ZH], B[ZH];
    double d[ZH];
    const int npl = C.npl;
    if constexpr (sizeof(T) == 8) {
      // FP64: Clenshaw's recurrence for d_q = sum'_j c_j T_j(Hhat) w_q,
      //   b_k = c_k w + 2 Hhat b_{k+1} - b_{k+2},  k = npl-1 .. 1,
      //   b_npl = c_npl w,  b_{npl+1} = 0,  d_q = c_0 w / 2 + Hhat b_1 - b_2,
      // the same npl applications as the forward recurrence but no separate
      // accumulator for d_q (registers)
      load_unit<Vr>(S, X, C, A, B, coef[npl]);
      // step j computes b_k, k = npl - 1 - j, from b_{k+1} (cur) and b_{k+2}
      // (io); the last one (k = 0) forms d_q
      auto step = [&](const T (&cur)[ZH], T (&io)[ZH], int j) {
        const int k = npl - 1 - j;
        apply_step<Vr, FUSED>(S, X, C, cur, io, ck, k == 0 ? 1.0 / zeta : 2.0 / zeta, (T)1, j & 1,
                              k == 0 ? 0.5 * coef[0] : coef[k]);
        mirror<Vr>(S, X, io);
        finish_proj<Vr>(S, j & 1);
        __syncthreads();
      };
      for (int j = 0; j < npl; j += 2) {
        step(A, B, j);
        if (j + 1 < npl) step(B, A, j + 1);
      }
      const bool in_b = (npl & 1) != 0;
#pragma unroll
      for (int z = 0; z < ZH; ++z) d[z] = (double)(in_b ? B[z] : A[z]);
    } else {
      // FP32 vectors: forward recurrence t^{j+1} = 2 Hhat t^j - t^{j-1} with
      // d_q = sum'_j c_j t^j accumulated in FP64
      load_unit<Vr>(S, X, C, A, B);
      const double c0h = 0.5 * coef[0];
#pragma unroll
      for (int z = 0; z < ZH; ++z) d[z] = c0h * (double)A[z];
      auto step = [&](const T (&cur)[ZH], T (&io)[ZH], int j) {
        apply_step<Vr, FUSED>(S, X, C, cur, io, ck, j == 0 ? 1.0 / zeta : 2.0 / zeta,
                              j == 0 ? (T)0 : (T)1, j & 1);
        const double cj = coef[j + 1];
#pragma unroll
        for (int z = 0; z < ZH; ++z) d[z] += cj * (double)io[z];
        mirror<Vr>(S, X, io);
        finish_proj<Vr>(S, j & 1);
        __syncthreads();
      };
      for (int j = 0; j < npl; j += 2) {
        step(A, B, j);
        if (j + 1 < npl) step(B, A, j + 1);
      }
    }

    // ---- gradients, one direction at a time (registers: d and one
    // gradient), the kinetic inputs on the three lines through the node,
    // and the nonlocal sums over the near images' supports ----
    const double ih = 1.0 / C.h;
    double w[SQ_FDM + 1];
#pragma unroll
    for (int k = 0; k <= SQ_FDM; ++k) w[k] = C.c1[k];
    // near images: projector nonzero at the node itself (found by the thread
    // that owns the node)
    if (X.active && X.cx == m && X.cy == m) {
      const unsigned bit = 0x80000000u >> m;
      int nn = 0;
#pragma unroll
      for (int s = 0; s < Vr::KC; ++s) {
        if (s < X.nslot) {
          const unsigned mk = X.sid[s];
          const int i = (int)(mk & IMASK);
          if (mk & bit) {
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
    for (int i = threadIdx.x; i < Vr::NEAR * 10 * 2; i += Vr::NT) (&S.ep.nsum[0][0][0])[i] = 0ull;
    for (int i = threadIdx.x; i < 3 * 3 * (2 * SQ_FDM + 1); i += Vr::NT) (&S.ep.kl[0][0][0])[i] = 0.0;
    __syncthreads();
    near_sums<Vr, -1>(S, X, C, d);   // chi^T d
#pragma unroll
    for (int dir = 0; dir < 3; ++dir) {
      double gr[ZH];
      if (dir < 2) {
#pragma unroll
        for (int z = 0; z < ZH; ++z) gr[z] = 0.0;
        T part[ZH];
#pragma unroll
        for (int z = 0; z < ZH; ++z) part[z] = (T)d[z];
        grad_round<Vr>(S, X, part, gr, w, dir);
        if constexpr (sizeof(T) < sizeof(double)) {   // FP32 mirror: the remainder in a second round
#pragma unroll
          for (int z = 0; z < ZH; ++z) part[z] = (T)(d[z] - (double)part[z]);
          grad_round<Vr>(S, X, part, gr, w, dir);
        }
#pragma unroll
        for (int z = 0; z < ZH; ++z) gr[z] *= ih;
      } else {
        grad_z<Vr>(X, d, gr, w, ih);
      }
      // G_dir on the x, y and z lines through the node (offsets -6 .. 6)
      if (X.active) {
#pragma unroll
        for (int z = 0; z < ZH; ++z) {
          const int ox = X.cx - m, oy = X.cy - m, oz = z - m;
          if (oy == 0 && oz == 0 && ox >= -SQ_FDM && ox <= SQ_FDM) S.ep.kl[0][dir][ox + SQ_FDM] = gr[z];
          if (ox == 0 && oz == 0 && oy >= -SQ_FDM && oy <= SQ_FDM) S.ep.kl[1][dir][oy + SQ_FDM] = gr[z];
          if (ox == 0 && oy == 0 && oz >= -SQ_FDM && oz <= SQ_FDM) S.ep.kl[2][dir][oz + SQ_FDM] = gr[z];
        }
      }
      if (dir == 0) near_sums<Vr, 0>(S, X, C, gr);
      else if (dir == 1) near_sums<Vr, 1>(S, X, C, gr);
      else near_sums<Vr, 2>(S, X, C, gr);
    }
    __syncthreads();
    double* rec = P.rec + g * SQ_REC;
    if (threadIdx.x == 0) {
      // K_ab = 2 (grad_a G_b)(node), (grad_a G_b) = (1/h) sum_k w_k
      // (G_b(+k e_a) - G_b(-k e_a)); points outside the cube hold zero
      for (int a = 0; a < 3; ++a)
        for (int bb = 0; bb < 3; ++bb) {
          double acc = 0.0;
          for (int k = 1; k <= SQ_FDM; ++k) acc += w[k] * (S.ep.kl[a][bb][SQ_FDM + k] - S.ep.kl[a][bb][SQ_FDM - k]);
          rec[2 + 3 * a + bb] = 2.0 * acc * ih;
        }
      double N[9], enl = 0.0;
      for (int t = 0; t < 9; ++t) N[t] = 0.0;
      const int nnear = S.nnear;
      for (int n = 0; n < nnear; ++n) {
        const int i = S.near_img[n];
        const double f = -2.0 * S.gdv[i] * S.near_chi[n];
        double ns[10];
        for (int t = 0; t < 10; ++t) ns[t] = fx_load(S.ep.nsum[n][t]);
        enl -= f * ns[0];   // 2 gamma dV chi_I(x_q) chi_I^T d_q
        for (int a = 0; a < 3; ++a)
          for (int bb = 0; bb < 3; ++bb) N[3 * a + bb] += f * ((a == bb ? ns[0] : 0.0) + 2.0 * ns[1 + 3 * a + bb]);
      }
      for (int t = 0; t < 9; ++t) rec[11 + t] = N[t];
      rec[20] = enl;
    }
    node_epilogue<Vr>(X, P.err);
  });
}

// ---------------------------------------------------------------------------
// Capacity census (set-up time): per node the number of atom images reaching
// its cube, the largest number crossing one z-column, and the number whose
// projector is nonzero at the node.  Maxima per cell go to
// stats[SQ_CENSUS * cell + 0..2].
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
    atomicMax(&stats[SQ_CENSUS * ci + 0], found);
    atomicMax(&stats[SQ_CENSUS * ci + 1], colmax);
    atomicMax(&stats[SQ_CENSUS * ci + 2], nnear);
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

enum Fam { FAM_LAN, FAM_MOM, FAM_STR };

template <class Vr, int F, bool FUSED, bool PERSIST>
auto kernel_of() {
  if constexpr (F == FAM_LAN) return &k_lanczos<Vr, FUSED, PERSIST>;
  else if constexpr (F == FAM_MOM) return &k_moments<Vr, FUSED, PERSIST>;
  else return &k_stress<Vr, FUSED, PERSIST>;
}

// One workgroup per node; or, PERSIST, as many workgroups as the device
// holds at once (occupancy of the kernel times the number of CUs), each
// taking nodes from the work counter, cleared first by a fill kernel (also
// inside a captured graph).
template <class Vr, int F, bool FUSED, bool PERSIST>
hipError_t launch_one(const RecLaunch& R, const PlanDev& P, const long long* items, const int* ic,
                      long long n, hipStream_t s) {
  auto kern = kernel_of<Vr, F, FUSED, PERSIST>();
  unsigned grid = (unsigned)n;
  if constexpr (PERSIST) {
    static int per_cu = 0;   // occupancy of this kernel (a property of the code object)
    if (per_cu <= 0) {
      int v = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kern, Vr::NT, 0) != hipSuccess || v < 1) v = 1;
      per_cu = v;
    }
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const long long want = R.grid > 0 ? (long long)R.grid : (long long)per_cu * cus;
    grid = (unsigned)(want < n ? want : n);
    e = sq_launch_fill_u32(R.counter, 0u, 1, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(grid), dim3(Vr::NT), 0, s, P, items, ic, n, R.counter);
  return hipGetLastError();
}

template <class Vr, int F, bool FUSED, bool WITH_PERSIST>
hipError_t launch_var(const RecLaunch& R, const PlanDev& P, const long long* items, const int* ic,
                      long long n, hipStream_t s) {
  if constexpr (WITH_PERSIST) {
    if (R.counter) return launch_one<Vr, F, FUSED, true>(R, P, items, ic, n, s);
  }
  return launch_one<Vr, F, FUSED, false>(R, P, items, ic, n, s);
}

// The compiled variants per precision: sq_kc_pick gives the slot capacity
// (16 or 24 with the plane weights in registers, or 48); nodes without a stored
// Gram matrix (rare: dense projector overlap) all use the 48-slot two-sweep
// form.  The persistent form is compiled for the 16-slot single-sweep
// variant; the others run one workgroup per node.
template <typename T, int F>
hipError_t launch_t(const RecLaunch& R, const PlanDev& P, const long long* items, const int* ic,
                    long long n, hipStream_t s) {
  const int kc = sq_kc_pick(R.fused, R.kc);
  if (!R.fused) {
    if (kc == 48) return launch_var<Var<T, SQN, 48, false>, F, false, false>(R, P, items, ic, n, s);
    return hipErrorInvalidValue;
  }
  if (kc == 16) return launch_var<Var<T, SQN, 16, true>, F, true, true>(R, P, items, ic, n, s);
  if (kc == 24) return launch_var<Var<T, SQN, 24, true>, F, true, false>(R, P, items, ic, n, s);
  if (kc == 48) return launch_var<Var<T, SQN, 48, false>, F, true, false>(R, P, items, ic, n, s);
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t SQ_CAT(sq_launch_lanczos_, SQ_ONE_NC)(const RecLaunch& R, const PlanDev& P,
                                                const long long* items, const int* ic, long long n,
                                                hipStream_t s) {
  return launch_t<double, FAM_LAN>(R, P, items, ic, n, s);
}

hipError_t SQ_CAT(sq_launch_moments_, SQ_ONE_NC)(const RecLaunch& R, bool fp64, const PlanDev& P,
                                                const long long* items, const int* ic, long long n,
                                                hipStream_t s) {
  return fp64 ? launch_t<double, FAM_MOM>(R, P, items, ic, n, s) : launch_t<float, FAM_MOM>(R, P, items, ic, n, s);
}

hipError_t SQ_CAT(sq_launch_stress_, SQ_ONE_NC)(const RecLaunch& R, bool fp64, const PlanDev& P,
                                               const long long* items, const int* ic, long long n,
                                               hipStream_t s) {
  return fp64 ? launch_t<double, FAM_STR>(R, P, items, ic, n, s) : launch_t<float, FAM_STR>(R, P, items, ic, n, s);
}

// The Gram build always runs the widest FP64 variant (the entries do not
// depend on the variant that reads them).
hipError_t SQ_CAT(sq_launch_gram_, SQ_ONE_NC)(const PlanDev& P, const long long* items,
                                             const int* ic, long long n, hipStream_t s) {
  using Vr = Var<double, SQN, 48, false>;
  hipLaunchKernelGGL(k_gram<Vr>, dim3((unsigned)n), dim3(Vr::NT), 0, s, P, items, ic);
  return hipGetLastError();
}

hipError_t SQ_CAT(sq_launch_census_, SQ_ONE_NC)(const PlanDev& P, const long long* items,
                                               const int* ic, long long n, int* stats,
                                               long long* pairs, hipStream_t s) {
  hipLaunchKernelGGL(k_census<SQN>, dim3((unsigned)n), dim3(sq_threads(SQN)), 0, s, P, items, ic, stats,
                     pairs);
  return hipGetLastError();
}
