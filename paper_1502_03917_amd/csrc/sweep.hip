// One fused kernel per LSGS sweep (Alg. 2 of Takacs, arXiv 1502.03917, with
// the unknowns ordered by the colours c(i,j) = (i + 2j) mod 7) for gfx950,
// and the same kernel for a sweep of the collective point smoother (section
// 2: a 2x2 solve of (y_v, lambda_v) per vertex, in the same 7 colours).
//
// A colour phase updates the vertices of one colour; each of them reads and
// writes r on its closed neighbourhood, so after 7 phases the residual at a
// vertex depends on the initial residual up to 14 lattice steps away.  Each
// workgroup owns a TW x TW tile of vertices.  It loads the residual (both
// fields) of the tile plus a 14-vertex halo into LDS once, then runs the 7
// phases in LDS with one barrier after each: phase c visits the vertices of
// colour c within Chebyshev distance 13 - 2c of the tile, exactly the set
// whose updates reach the tile, and all of those are computed from correct
// inputs.  At the end the tile's residual is written to r_out and its x,
// loaded into registers at the start, is written back with the accumulated
// corrections.  r is read from r_in and written to r_out (distinct buffers),
// so no tile sees a neighbour's finished values.
//
// Global traffic per owned vertex: x read and written once, r written once,
// r read once plus the halo share (neighbouring tiles re-read each other's
// borders, mostly from L2 because consecutive tiles run on the same XCD).
//
// The collective smoother reads only its own vertex's residual and scatters
// to the closed neighbourhood, so a phase widens the dependence by one step
// instead of two: a 7-vertex halo per sweep, and phase c visits the vertices
// of colour c within distance 7 - c of the tile.  Its scatters from the
// outermost window reach the guard ring, which nothing reads.
#include <type_traits>

#include "mg_internal.hpp"

namespace mgk {

namespace {

constexpr int kHalo = 14;     // LSGS: halo of one sweep
constexpr int kHaloCgs = 7;   // collective smoother: halo of one sweep

// transfers folded into a launch (SweepIO): none, the prolongation with the
// new residual before the sweeps, the restriction of the residual after them
constexpr int kIoNone = 0, kIoProlong = 1, kIoRestrict = 2;

// Workgroup barrier that orders LDS accesses only; global memory needs no
// ordering inside a sweep (r_in is read-only, r_out and x are per owned vertex).
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Global accesses go through buffer instructions and are issued
// unconditionally: a masked-off access uses an offset past the end of the
// buffer, which the hardware turns into a zero load / dropped store.  With a
// fixed number of memory operations the compiler waits only for the data it
// is about to use.
constexpr unsigned kOff = 0x80000000u;  // past the end of every buffer (< 2 GiB each)
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* p, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}
__device__ inline double bload(__amdgpu_buffer_rsrc_t r, unsigned off, double*) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ inline float bload(__amdgpu_buffer_rsrc_t r, unsigned off, float*) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ inline void bstore(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
__device__ inline void bstore(__amdgpu_buffer_rsrc_t r, unsigned off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}

// Row pitch of the LDS region beyond its RMAX + 2 cells (a guard cell each
// side).  A 16-byte (FP64) or 8-byte (FP32) access is served a few lanes at a
// time, and the lanes of a phase step through a row at a stride of 7 cells
// and then on into the next row; the padding is chosen, per tile shape, so
// that the cells of the lanes served together fall into distinct banks as
// often as possible (a bank-conflict model of the phases' access pattern, for
// 32 and 64 four-byte banks).
constexpr int pitch_pad(int TW, int H, int cell, bool cgs = false) {
  if (cgs)
    return cell == 16 ? (H == kHaloCgs ? (TW == 65 ? 14 : TW == 48 ? 10 : TW == 16 ? 14 : 1)
                                       : (TW == 17 ? 13 : TW == 33 ? 11 : 1))
                      : (H == kHaloCgs ? (TW == 46 ? 12 : TW == 48 ? 10 : TW == 16 ? 6 : 1)
                                       : (TW == 17 ? 13 : TW == 33 ? 11 : 1));
  // (33 x 33 pair tiles with the restriction's extra ring: 1, to fit the LDS)
  return cell == 16 ? (H == kHalo ? (TW == 65 ? 7 : TW == 56 ? 9 : TW == 48 ? 10 : TW == 16 ? 7 : 1)
                                  : (TW == 17 ? 13 : TW == 33 ? (H == 2 * kHalo ? 4 : 1) : 1))
                    : (H == kHalo ? (TW == 46 ? 3 : TW == 48 ? 12 : TW == 16 ? 8 : 1)
                                  : (TW == 17 ? 15 : TW == 33 ? 13 : 1));
}

template <int TW, int H = kHalo, int CELL = 16, bool CGS = false>
struct TileGeom {
  static constexpr int RMAX = TW + 2 * H;                           // widest / tallest region (halo H)
  static constexpr int RP = RMAX + 2 + pitch_pad(TW, H, CELL, CGS); // pitch: a guard cell each side, padding
  static constexpr int RN = RP * (RMAX + 2);                        // region cells with guard rows
};

// the two fields of one vertex side by side (one 16-byte LDS access in FP64)
template <typename T>
struct Pair;
template <>
struct Pair<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Pair<float> {
  typedef float type __attribute__((ext_vector_type(2)));
};

// Work items of a colour phase are (row, slot) pairs: slot t of a row is its
// t-th vertex of the phase's colour inside the window.  A window row of width
// w holds at most ceil(w / 7) of them.  The first window reaches H - 1 steps
// beyond the tile (LSGS) or H steps (collective smoother).
template <int TW, int H = kHalo, bool CGS = false>
struct PhaseItems {
  static constexpr int W0 = TW + 2 * (CGS ? H : H - 1);  // width and height of the widest (first) window
  static constexpr int SMAX = (W0 + 6) / 7;                // slots per row that cover every window
};

// The iterate is read from xin and written to x (the same buffer, or a
// distinct one when the sweep also moves x: xin is read only before x is
// written, per owned vertex).  NSW sweeps run in one pass over the tile
// (halo 14 NSW, or 7 NSW for the collective smoother (CGS); 7 NSW colour
// phases); bit s of reverse gives the order of sweep s.
//
// Transfers (IO): with kIoProlong the tile forms x + P x_c on its region and
// the ring around it, then r = f - A (x + P x_c) on the region, in LDS,
// instead of reading r (xin is read on the whole region: it must not alias
// x).  With kIoRestrict the halo is one vertex wider, so that the residual
// is also final on the ring around the tile, and the tile writes f_c = P^T r
// for the coarse vertices (I, J) with (2I, 2J) in the tile instead of r.
template <typename T, int TW, int NT, int NSW = 1, bool CGS = false, int IO = kIoNone>
__device__ __forceinline__ void lsgs_tile_body(const Lev& L, int ntx, int nty, int reverse, const T* xin, T* x,
                                               const T* __restrict__ rin, T* __restrict__ rout,
                                               double* __restrict__ part = nullptr, int norm_mode = 0,
                                               const SweepIO<T>* io = nullptr) {
  constexpr int H = (CGS ? kHaloCgs : kHalo) * NSW + (IO == kIoRestrict ? 1 : 0);
  using G = TileGeom<TW, H, 2 * sizeof(T), CGS>;
  using T2 = typename Pair<T>::type;
  using PI = PhaseItems<TW, H, CGS>;
  constexpr int NR = (G::RMAX * G::RMAX + NT - 1) / NT;  // region cells per thread
  constexpr int NX = (TW * TW + NT - 1) / NT;            // owned cells per thread
  constexpr int SMAX = PI::SMAX;
  // The rows of a phase window are enumerated from the tile's first row on,
  // wrapping round to the halo rows above it.  When the first pass of the
  // workgroup (NT / SMAX rows) spans the tile's height, every owned vertex of a
  // phase falls in it: each thread then has at most one owned vertex per
  // phase, known in advance, and updates its x directly (x prefetched at the
  // start, x + p stored in the phase); window rows beyond the first pass are
  // halo rows and give some threads a second vertex (kSecond).  Otherwise the
  // corrections of the owned vertices collect in LDS and x is written at the end.
  // (Several sweeps in one pass update an owned vertex once per sweep, so
  // their corrections always collect in LDS.)
  constexpr bool kOnePass = NSW == 1 && TW <= NT / SMAX;
  constexpr bool kSecond = kOnePass && PI::W0 * SMAX > NT;
  static_assert(PI::W0 * SMAX <= 2 * NT || !kOnePass, "at most two vertices per thread and phase");
  // residual (y, lambda) of the region; the guard ring and the cells of the
  // region that lie outside the square hold zeros, so the neighbours of a
  // boundary vertex can be read and written without bounds checks (their
  // coefficients in the class blocks are zero)
  __shared__ T2 s2[G::RN];
  __shared__ T2 dx2[kOnePass ? 1 : TW * TW];  // corrections of the owned x (multi-pass phases)
  __shared__ __align__(16) T tC[25 * kC5];    // per-class coefficient blocks

  const int n = L.n, ld = L.ld, V = L.V;
  const int ntiles = ntx * nty;
  const int nblk = gridDim.x, bid = blockIdx.x;
  const int tid = threadIdx.x;
  const size_t vbytes = (size_t)2 * V * sizeof(T);
  // an iterate taken as zero reads through an empty buffer: every load of it
  // returns 0 without a memory access
  const bool xzero = io != nullptr && io->xin_zero;
  const __amdgpu_buffer_rsrc_t Rin = make_rsrc(rin, vbytes), Rout = make_rsrc(rout, vbytes), Rx = make_rsrc(x, vbytes),
                              Rxi = make_rsrc(xin, xzero ? 0 : vbytes);
  const unsigned fo = (unsigned)(V * sizeof(T));  // byte offset of the lambda field

  // The workgroups of one XCD (bid % 8) take a contiguous run of tiles, which
  // share halo rows in that XCD's L2 (the grid is a multiple of 8).
  const int tile = (nblk % 8 == 0) ? (bid % 8) * (nblk / 8) + bid / 8 : bid;
  if (tile >= ntiles) return;  // padding workgroup
  const int tx = tile % ntx, ty = tile / ntx;
  const int i0 = tx * TW, i1 = min(n + 1, i0 + TW);
  const int j0 = ty * TW, j1 = min(n + 1, j0 + TW);
  const int ci0 = max(0, i0 - H), ci1 = min(n + 1, i1 + H);
  const int rj0 = max(0, j0 - H), rj1 = min(n + 1, j1 + H);
  const int RW = ci1 - ci0, RH = rj1 - rj0, OW = i1 - i0, OH = j1 - j0;

  // the vertex of work item k in phase ph (gi >= wh or k >= nitems: none)
  struct Item {
    int gi, gj;
    bool act;
  };
  auto item_of = [&](int ph, int k) {
    const int c7 = ph % 7;
    const int colour = ((reverse >> (ph / 7)) & 1) ? 6 - c7 : c7;
    const int d = CGS ? H - ph : H - 1 - 2 * ph;  // Chebyshev radius of the phase window around the tile
    const int wl = max(ci0, i0 - d), wh = min(ci1, i1 + d);
    const int wb = max(rj0, j0 - d), wt = min(rj1, j1 + d);
    // a fixed slot count (covering the widest window) keeps the decode free of
    // divisions by run-time values; slots past wh are skipped
    const int S = kOnePass ? SMAX : (wh - wl + 6) / 7;
    const int rr = k / S, t = k - rr * S;
    Item it;
    if constexpr (kOnePass) {
      it.gj = j0 + rr;  // wb <= j0 < j1 <= wt
      if (it.gj >= wt) it.gj -= wt - wb;
    } else {
      it.gj = wb + rr;
    }
    it.gi = wl + ((colour - 2 * it.gj - wl) % 7 + 7) % 7 + 7 * t;
    it.act = k < (wt - wb) * S && it.gi < wh;
    return it;
  };
  auto owned = [&](const Item& it) { return it.act && it.gi >= i0 && it.gi < i1 && it.gj >= j0 && it.gj < j1; };

  // Loads first, so that all of them are in flight before the first LDS store:
  // x of the owned vertices this thread updates (one-pass) or of the owned
  // cells it writes at the end, then the region of r.  Cells outside the
  // square load as zero (masked offset).
  constexpr int NXP = kOnePass ? 7 : NX;
  T xy[NXP], xl[NXP];
  unsigned xo[kOnePass ? 7 : 1];
  if constexpr (kOnePass) {
#pragma unroll
    for (int ph = 0; ph < 7; ph++) {
      const Item it = item_of(ph, tid);
      xo[ph] = owned(it) ? (unsigned)((it.gj * ld + it.gi) * sizeof(T)) : kOff;
      if constexpr (IO != kIoProlong) {
        xy[ph] = bload(Rxi, xo[ph], (T*)nullptr);
        xl[ph] = bload(Rxi, xo[ph] == kOff ? kOff : xo[ph] + fo, (T*)nullptr);
      }
    }
  } else if constexpr (IO != kIoProlong) {
#pragma unroll
    for (int q = 0; q < NX; q++) {
      const int e = tid + q * NT;
      const int oj = e / TW, oi = e - oj * TW;
      const bool ok = e < TW * TW && oi < OW && oj < OH;
      const unsigned o = ok ? (unsigned)(((j0 + oj) * ld + i0 + oi) * sizeof(T)) : kOff;
      xy[q] = bload(Rxi, o, (T*)nullptr);
      xl[q] = bload(Rxi, ok ? o + fo : kOff, (T*)nullptr);
    }
  }
  T ry[NR], rl[NR];
  if constexpr (IO != kIoProlong) {
#pragma unroll
    for (int q = 0; q < NR; q++) {
      const int e = tid + q * NT;
      const int lr = e / G::RMAX, li = e - lr * G::RMAX;
      const bool ok = e < G::RMAX * G::RMAX && li < RW && lr < RH;
      const unsigned o = ok ? (unsigned)(((rj0 + lr) * ld + ci0 + li) * sizeof(T)) : kOff;
      ry[q] = bload(Rin, o, (T*)nullptr);
      rl[q] = bload(Rin, ok ? o + fo : kOff, (T*)nullptr);
    }
  }
  {
    constexpr int NC = (25 * kC5 + NT - 1) / NT;
    const double* src = &L.tab->C5[0][0];
#pragma unroll
    for (int q = 0; q < NC; q++)
      if (tid + q * NT < 25 * kC5) tC[tid + q * NT] = (T)src[tid + q * NT];
  }
  if constexpr (IO == kIoProlong) {
    // (1) x + P x_c on every cell of the region and of the ring around it
    // (the guard positions), zero outside the square.  A thread takes the
    // 2 x 2 fine cells (2I + a, 2J + b), a, b in {0, 1}: P x_c there is the
    // mean of the coarse values at (I, J) and (I + a, J + b) (a coarse vertex,
    // or the two ends of the horizontal, vertical or (I,J)-(I+1,J+1) diagonal
    // coarse edge the fine vertex halves; for a coarse vertex the mean is its
    // value exactly).  The loads of a batch of blocks are all issued before
    // any of them is used; f is loaded after the batches, in flight through
    // the barrier.
    const Lev& Lc = io->Lc;
    const __amdgpu_buffer_rsrc_t Rxc = make_rsrc(io->xc, (size_t)2 * Lc.V * sizeof(T));
    const unsigned foc = (unsigned)(Lc.V * sizeof(T));
    const __amdgpu_buffer_rsrc_t Rf = make_rsrc(io->f, vbytes);
    constexpr int RA = G::RMAX + 2;               // rows and columns of region + ring in s2
    constexpr int BN = RA / 2 + 1;                // 2 x 2 blocks per row that cover them
    constexpr int NB = (BN * BN + NT - 1) / NT;  // blocks per thread
    constexpr int BB = 1;                         // blocks per batch
    const int fa = ci0 - 1, fb = rj0 - 1;         // fine cell of s2[0] (>= -1)
    const int I0 = (fa + 2) / 2 - 1, J0 = (fb + 2) / 2 - 1;  // floor(fa / 2), floor(fb / 2)
    const int nc = Lc.n;
#pragma unroll
    for (int q0 = 0; q0 < NB; q0 += BB) {
      T cv[BB][8], xv[BB][8];
#pragma unroll
      for (int u = 0; u < BB; u++) {
        const int e = tid + (q0 + u) * NT;
        const bool live = q0 + u < NB && e < BN * BN;
        const int bj = e / BN, bi = e - bj * BN;
#pragma unroll
        for (int k = 0; k < 4; k++) {  // coarse vertex (I + (k & 1), J + (k >> 1)); fine cell (2I + (k & 1), 2J + (k >> 1))
          const int I = I0 + bi + (k & 1), J = J0 + bj + (k >> 1);
          const bool okc = live && I >= 0 && I <= nc && J >= 0 && J <= nc;
          const unsigned oc = okc ? (unsigned)((J * Lc.ld + I) * sizeof(T)) : kOff;
          cv[u][2 * k] = bload(Rxc, oc, (T*)nullptr);
          cv[u][2 * k + 1] = bload(Rxc, okc ? oc + foc : kOff, (T*)nullptr);
          const int gi = 2 * (I0 + bi) + (k & 1), gj = 2 * (J0 + bj) + (k >> 1);
          const int wx = gi - fa, wy = gj - fb;
          const bool okx = live && wx < RA && wy < RA && wx <= RW + 1 && wy <= RH + 1 && gi >= 0 && gi <= n &&
                           gj >= 0 && gj <= n;
          const unsigned ox = okx ? (unsigned)((gj * ld + gi) * sizeof(T)) : kOff;
          xv[u][2 * k] = bload(Rxi, ox, (T*)nullptr);
          xv[u][2 * k + 1] = bload(Rxi, okx ? ox + fo : kOff, (T*)nullptr);
        }
      }
#pragma unroll
      for (int u = 0; u < BB; u++) {
        const int e = tid + (q0 + u) * NT;
        if (q0 + u < NB && e < BN * BN) {
          const int bj = e / BN, bi = e - bj * BN;
#pragma unroll
          for (int k = 0; k < 4; k++) {
            const int gi = 2 * (I0 + bi) + (k & 1), gj = 2 * (J0 + bj) + (k >> 1);
            const int wx = gi - fa, wy = gj - fb;
            if (wx >= 0 && wx < RA && wy >= 0 && wy < RA) {
              // loads outside the square or past region + ring returned zeros
              const bool in = wx <= RW + 1 && wy <= RH + 1 && gi >= 0 && gi <= n && gj >= 0 && gj <= n;
              const T vy = (T)0.5 * (cv[u][0] + cv[u][2 * k]), vl = (T)0.5 * (cv[u][1] + cv[u][2 * k + 1]);
              s2[wy * G::RP + wx] = in ? (T2){xv[u][2 * k] + vy, xv[u][2 * k + 1] + vl} : (T2){(T)0, (T)0};
            }
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NR; q++) {  // f of the region
      const int e = tid + q * NT;
      const int lr = e / G::RMAX, li = e - lr * G::RMAX;
      const bool ok = e < G::RMAX * G::RMAX && li < RW && lr < RH;
      const unsigned o = ok ? (unsigned)(((rj0 + lr) * ld + ci0 + li) * sizeof(T)) : kOff;
      ry[q] = bload(Rf, o, (T*)nullptr);
      rl[q] = bload(Rf, ok ? o + fo : kOff, (T*)nullptr);
    }
    lds_barrier();
    // (2) r = f - A (x + P x_c) on the region, into registers; the corrected
    // iterate of the owned vertices for the x stores
    const T ai = (T)L.ainv;
#pragma unroll
    for (int q = 0; q < NR; q++) {
      const int e = tid + q * NT;
      const int lr = e / G::RMAX, li = e - lr * G::RMAX;
      const bool ok = e < G::RMAX * G::RMAX && li < RW && lr < RH;
      const int gi = ci0 + li, gj = rj0 + lr;
      T ay = 0, al = 0;
      if (ok) {
        const int c = (lr + 1) * G::RP + li + 1;
        const T2 xc2 = s2[c];
        if (gi >= 1 && gi < n && gj >= 1 && gj < n) {
          const T2 e2 = s2[c + 1], w2 = s2[c - 1], n2 = s2[c + G::RP], s2_ = s2[c - G::RP];
          const T2 ne2 = s2[c + G::RP + 1], sw2 = s2[c - G::RP - 1];
          const T ya = e2.x + w2.x + n2.x + s2_.x;
          const T yg = ne2.x + sw2.x;
          const T la = e2.y + w2.y + n2.y + s2_.y;
          const T lg = ne2.y + sw2.y;
          const T Mc = (T)L.Mc, Mo = (T)L.Mo, Kc = (T)L.Kc, Ka = (T)L.Ka, Kd = (T)L.Kd;
          ay = Mc * xc2.x + Mo * (ya + yg) + (Kc * xc2.y + Ka * la + Kd * lg);
          al = (Kc * xc2.x + Ka * ya + Kd * yg) - ai * (Mc * xc2.y + Mo * (la + lg));
        } else {
          const T* cb = &tC[(cls5(gi, n) * 5 + cls5(gj, n)) * kC5];
#pragma unroll
          for (int d = 0; d < kNDir; d++) {
            const int ii = gi + kDI[d], jj = gj + kDJ[d];
            if (ii < 0 || ii > n || jj < 0 || jj > n) continue;
            const T2 v = s2[c + kDJ[d] * G::RP + kDI[d]];
            ay += cb[d] * v.x + cb[kNDir + d] * v.y;
            al += cb[kNDir + d] * v.x - ai * cb[d] * v.y;
          }
        }
      }
      ry[q] = ok ? ry[q] - ay : (T)0;
      rl[q] = ok ? rl[q] - al : (T)0;
    }
    if constexpr (kOnePass) {
#pragma unroll
      for (int ph = 0; ph < 7; ph++) {
        const Item it = item_of(ph, tid);
        const T2 v = s2[xo[ph] == kOff ? 0 : (it.gj - rj0 + 1) * G::RP + (it.gi - ci0) + 1];
        xy[ph] = v.x;
        xl[ph] = v.y;
      }
    } else {
#pragma unroll
      for (int q = 0; q < NX; q++) {
        const int e = tid + q * NT;
        const int oj = e / TW, oi = e - oj * TW;
        const bool ok = e < TW * TW && oi < OW && oj < OH;
        const T2 v = s2[ok ? (j0 + oj - rj0 + 1) * G::RP + (i0 + oi - ci0) + 1 : 0];
        xy[q] = v.x;
        xl[q] = v.y;
      }
    }
    lds_barrier();
  }
  // guard ring: rows 0 and RMAX + 1, columns 0 and RMAX + 1
  for (int e = tid; e < 4 * (G::RMAX + 2); e += NT) {
    const int side = e / (G::RMAX + 2), t = e - side * (G::RMAX + 2);
    const int a = side == 0 ? t : side == 1 ? (G::RMAX + 1) * G::RP + t : side == 2 ? t * G::RP
                                                                                   : t * G::RP + G::RMAX + 1;
    s2[a] = (T2){(T)0, (T)0};
  }
  if constexpr (!kOnePass)
    for (int e = tid; e < TW * TW; e += NT) dx2[e] = (T2){(T)0, (T)0};
#pragma unroll
  for (int q = 0; q < NR; q++) {
    const int e = tid + q * NT;
    const int lr = e / G::RMAX, li = e - lr * G::RMAX;
    if (e < G::RMAX * G::RMAX) s2[(lr + 1) * G::RP + li + 1] = (T2){ry[q], rl[q]};
  }
  lds_barrier();

  const T Mc = (T)L.Mc, Mo = (T)L.Mo, Kc = (T)L.Kc, Ka = (T)L.Ka, Kd = (T)L.Kd, Wi = (T)L.Winv;
  const T al = (T)L.alpha, ai = (T)L.ainv, Nyi = (T)L.Nyi, Nli = (T)L.Nli;

  // vertices at least 2 steps from the boundary share one stencil (the
  // constants above); the others take their class block.  The choice is
  // made per wave, so a wave runs one of the two paths: a wave holding any
  // near-boundary vertex runs the class-block path for all its lanes (the
  // interior class block holds the interior stencil).
  auto update_interior = [&](int b0, T& py, T& pl) {
    const int bu = b0 + G::RP, bd = b0 - G::RP;
    // the 7 residual pairs are read once; the scatter writes the gathered
    // values minus the update (no other vertex of the phase touches them)
    const T2 c = s2[b0], e = s2[b0 + 1], w = s2[b0 - 1], nn = s2[bu], ss = s2[bd], ne = s2[bu + 1], sw = s2[bd - 1];
    const T ya = e.x + w.x + nn.x + ss.x;
    const T yg = ne.x + sw.x;
    const T la = e.y + w.y + nn.y + ss.y;
    const T lg = ne.y + sw.y;
    const T qy = Wi * (Mc * c.x + Mo * (ya + yg) + al * (Kc * c.y + Ka * la + Kd * lg));
    const T ql = Wi * ((Kc * c.x + Ka * ya + Kd * yg) - (Mc * c.y + Mo * (la + lg)));
    py = qy * Nyi;
    pl = ql * Nli;
    const T dyc = Mc * py + Kc * pl, dya = Mo * py + Ka * pl, dyg = Mo * py + Kd * pl;
    const T dlc = Kc * py - ai * (Mc * pl), dla = Ka * py - ai * (Mo * pl), dlg = Kd * py - ai * (Mo * pl);
    s2[b0] = (T2){c.x - dyc, c.y - dlc};
    s2[b0 + 1] = (T2){e.x - dya, e.y - dla};
    s2[b0 - 1] = (T2){w.x - dya, w.y - dla};
    s2[bu] = (T2){nn.x - dya, nn.y - dla};
    s2[bd] = (T2){ss.x - dya, ss.y - dla};
    s2[bu + 1] = (T2){ne.x - dyg, ne.y - dlg};
    s2[bd - 1] = (T2){sw.x - dyg, sw.y - dlg};
  };
  auto update_class = [&](int b0, int gi, int gj, T& py, T& pl) {
    const T* cb = &tC[(cls5(gi, n) * 5 + cls5(gj, n)) * kC5];
    T2 v[kNDir];
#pragma unroll
    for (int d = 0; d < kNDir; d++) v[d] = s2[b0 + kDJ[d] * G::RP + kDI[d]];
    T qy = 0, ql = 0;
#pragma unroll
    for (int d = 0; d < kNDir; d++) {
      const T m = cb[d], k = cb[kNDir + d], wi = cb[2 * kNDir + d];
      qy += (m * v[d].x + al * k * v[d].y) * wi;
      ql += (k * v[d].x - m * v[d].y) * wi;
    }
    py = qy * cb[3 * kNDir];
    pl = ql * cb[3 * kNDir + 1];
#pragma unroll
    for (int d = 0; d < kNDir; d++) {
      const T m = cb[d], k = cb[kNDir + d];
      s2[b0 + kDJ[d] * G::RP + kDI[d]] = (T2){v[d].x - (m * py + k * pl), v[d].y - (k * py - ai * (m * pl))};
    }
  };
  // Collective smoother (CGS): the 2x2 system [[M_vv, K_vv], [K_vv,
  // -alpha^-1 M_vv]] d = (r^y_v, r^l_v) is solved at the vertex, x += d, and
  // r_m -= A_mv d on the closed neighbourhood (A symmetric: A_mv is the
  // vertex's own stencil entry towards m).  Its own row is the interior
  // stencil from one step inside the boundary on.
  auto cgs_interior = [&](int b0, T& py, T& pl) {
    const int bu = b0 + G::RP, bd = b0 - G::RP;
    const T2 c = s2[b0], e = s2[b0 + 1], w = s2[b0 - 1], nn = s2[bu], ss = s2[bd], ne = s2[bu + 1], sw = s2[bd - 1];
    const T b22 = -ai * Mc, det = Mc * b22 - Kc * Kc;
    py = (b22 * c.x - Kc * c.y) / det;
    pl = (Mc * c.y - Kc * c.x) / det;
    const T dyc = Mc * py + Kc * pl, dya = Mo * py + Ka * pl, dyg = Mo * py + Kd * pl;
    const T dlc = Kc * py - ai * (Mc * pl), dla = Ka * py - ai * (Mo * pl), dlg = Kd * py - ai * (Mo * pl);
    s2[b0] = (T2){c.x - dyc, c.y - dlc};
    s2[b0 + 1] = (T2){e.x - dya, e.y - dla};
    s2[b0 - 1] = (T2){w.x - dya, w.y - dla};
    s2[bu] = (T2){nn.x - dya, nn.y - dla};
    s2[bd] = (T2){ss.x - dya, ss.y - dla};
    s2[bu + 1] = (T2){ne.x - dyg, ne.y - dlg};
    s2[bd - 1] = (T2){sw.x - dyg, sw.y - dlg};
  };
  auto cgs_class = [&](int b0, int gi, int gj, T& py, T& pl) {
    const T* cb = &tC[(cls5(gi, n) * 5 + cls5(gj, n)) * kC5];
    T2 v[kNDir];
#pragma unroll
    for (int d = 0; d < kNDir; d++) v[d] = s2[b0 + kDJ[d] * G::RP + kDI[d]];
    const T m0 = cb[0], k0 = cb[kNDir];
    const T b22 = -ai * m0, det = m0 * b22 - k0 * k0;
    py = (b22 * v[0].x - k0 * v[0].y) / det;
    pl = (m0 * v[0].y - k0 * v[0].x) / det;
#pragma unroll
    for (int d = 0; d < kNDir; d++) {
      const T m = cb[d], k = cb[kNDir + d];
      s2[b0 + kDJ[d] * G::RP + kDI[d]] = (T2){v[d].x - (m * py + k * pl), v[d].y - (k * py - ai * (m * pl))};
    }
  };
  // update of item it (all lanes of the wave call this: the path choice is a ballot)
  auto update = [&](const Item& it, T& py, T& pl) {
    constexpr int e = CGS ? 1 : 2;  // first index whose update takes the interior constants
    const bool inner = it.gi >= e && it.gi <= n - e && it.gj >= e && it.gj <= n - e;
    const bool wave_inner = __builtin_amdgcn_ballot_w64(it.act && !inner) == 0;
    if (it.act) {
      const int b0 = (it.gj - rj0 + 1) * G::RP + (it.gi - ci0) + 1;
      if constexpr (CGS) {
        if (wave_inner)
          cgs_interior(b0, py, pl);
        else
          cgs_class(b0, it.gi, it.gj, py, pl);
      } else {
        if (wave_inner)
          update_interior(b0, py, pl);
        else
          update_class(b0, it.gi, it.gj, py, pl);
      }
    }
  };

  if constexpr (kOnePass) {
#pragma unroll
    for (int ph = 0; ph < 7; ph++) {
      const Item it = item_of(ph, tid);
      T py = 0, pl = 0;
      update(it, py, pl);
      // x of an owned vertex: the prefetched value plus its correction
      // (masked store for other items)
      bstore(Rx, xo[ph], xy[ph] + py);
      bstore(Rx, xo[ph] == kOff ? kOff : xo[ph] + fo, xl[ph] + pl);
      if constexpr (kSecond) {
        // a halo vertex of the rows past the first pass (no x)
        const Item it2 = item_of(ph, tid + NT);
        T qy = 0, ql = 0;
        update(it2, qy, ql);
      }
      lds_barrier();
    }
  } else {
    for (int ph = 0; ph < 7 * NSW; ph++) {
      const int d = CGS ? H - ph : H - 1 - 2 * ph;
      const int wl = max(ci0, i0 - d), wh = min(ci1, i1 + d);
      const int wb = max(rj0, j0 - d), wt = min(rj1, j1 + d);
      const int nitems = (wt - wb) * ((wh - wl + 6) / 7);
      for (int k = tid; k < nitems; k += NT) {
        const Item it = item_of(ph, k);
        T py = 0, pl = 0;
        update(it, py, pl);
        if (owned(it)) {
          T2& dv = dx2[(it.gj - j0) * TW + (it.gi - i0)];
          if constexpr (NSW == 1)
            dv = (T2){py, pl};
          else
            dv += (T2){py, pl};
        }
      }
      lds_barrier();
    }
  }

  // owned tile out: r to r_out (and x + corrections to x for multi-pass
  // phases); with norm_mode 1 / 2 also the tile's share of ||r_out||^2,
  // Euclidean or weighted by L^{-1} = blockdiag(W^{-1}, alpha W^{-1}), in
  // part[tile]
  double s2sum = 0.0;
#pragma unroll
  for (int q = 0; q < NX; q++) {
    const int e = tid + q * NT;
    const int oj = e / TW, oi = e - oj * TW;
    const bool ok = e < TW * TW && oi < OW && oj < OH;
    const int a = ok ? (oj + j0 - rj0 + 1) * G::RP + (oi + i0 - ci0) + 1 : 0;
    const unsigned o = ok ? (unsigned)(((j0 + oj) * ld + i0 + oi) * sizeof(T)) : kOff;
    const unsigned o2 = ok ? o + fo : kOff;
    const T2 rv = s2[a];
    if constexpr (IO != kIoRestrict) {
      bstore(Rout, o, rv.x);
      bstore(Rout, o2, rv.y);
    }
    if constexpr (!kOnePass) {
      const T2 dv = dx2[ok ? e : 0];
      bstore(Rx, o, xy[q] + dv.x);
      bstore(Rx, o2, xl[q] + dv.y);
    }
    if (norm_mode && ok) {
      const double ry = (double)rv.x, rl = (double)rv.y;
      if (norm_mode == 1) {
        s2sum += ry * ry + rl * rl;
      } else {
        const int gi = i0 + oi, gj = j0 + oj;
        const double wi = (gi >= 1 && gi < n && gj >= 1 && gj < n)
                              ? L.Winv
                              : (double)tC[(cls5(gi, n) * 5 + cls5(gj, n)) * kC5 + 2 * kNDir];
        s2sum += wi * (ry * ry + L.alpha * (rl * rl));
      }
    }
  }
  if constexpr (IO == kIoRestrict) {
    // f_c = P^T r: coarse vertex (I, J) collects the residual at (2I, 2J) with
    // weight 1 and at its six lattice neighbours with weight 1/2 (the ring
    // around the tile holds final values); x_c = 0 and r_c = f_c when asked
    const Lev& Lc = io->Lc;
    const int I0 = (i0 + 1) >> 1, J0 = (j0 + 1) >> 1;
    const int CW = ((i1 + 1) >> 1) - I0, CH = ((j1 + 1) >> 1) - J0;
    for (int e = tid; e < CW * CH; e += NT) {
      const int cj = e / CW, ci = e - cj * CW;
      const int I = I0 + ci, J = J0 + cj, a = 2 * I, b = 2 * J;
      const int c = (b - rj0 + 1) * G::RP + (a - ci0) + 1;
      const T2 r0 = s2[c];
      T hy = 0, hl = 0;
      if (a >= 1 && a < n && b >= 1 && b < n) {
        const T2 e2 = s2[c + 1], w2 = s2[c - 1], n2 = s2[c + G::RP], s2_ = s2[c - G::RP];
        const T2 ne2 = s2[c + G::RP + 1], sw2 = s2[c - G::RP - 1];
        hy = (e2.x + w2.x + n2.x + s2_.x) + (ne2.x + sw2.x);
        hl = (e2.y + w2.y + n2.y + s2_.y) + (ne2.y + sw2.y);
      } else {
#pragma unroll
        for (int d = 1; d < kNDir; d++) {
          const int aa = a + kDI[d], bb = b + kDJ[d];
          if (aa < 0 || aa > n || bb < 0 || bb > n) continue;
          const T2 v = s2[c + kDJ[d] * G::RP + kDI[d]];
          hy += v.x;
          hl += v.y;
        }
      }
      const int w = J * Lc.ld + I;
      const T gy = r0.x + (T)0.5 * hy, gl = r0.y + (T)0.5 * hl;
      io->fc[w] = gy;
      io->fc[Lc.V + w] = gl;
      if (io->xc0) {
        io->xc0[w] = (T)0;
        io->xc0[Lc.V + w] = (T)0;
      }
      if (io->rc) {
        io->rc[w] = gy;
        io->rc[Lc.V + w] = gl;
      }
    }
  }
  if (norm_mode) {
    // fixed-order workgroup sum: within each wave, then over the waves
    __shared__ double wsum[NT / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s2sum += __shfl_xor(s2sum, o, 64);
    if ((tid & 63) == 0) wsum[tid >> 6] = s2sum;
    lds_barrier();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < NT / 64; w++) t += wsum[w];
      part[tile] = t;
    }
  }
}

template <typename T, int TW, int NT, int NSW = 1, int IO = kIoNone>
__global__ __launch_bounds__(NT) void k_lsgs_tile(Lev L, int ntx, int nty, int reverse, const T* xin, T* x,
                                                  const T* __restrict__ rin, T* __restrict__ rout,
                                                  double* __restrict__ part, int norm_mode, SweepIO<T> io) {
  lsgs_tile_body<T, TW, NT, NSW, false, IO>(L, ntx, nty, reverse, xin, x, rin, rout, part, norm_mode, &io);
}

// NSW sweeps of the collective point smoother (the colour order of every
// sweep is 0..6; reverse is unused)
template <typename T, int TW, int NT, int NSW = 1, int IO = kIoNone>
__global__ __launch_bounds__(NT) void k_cgs_tile(Lev L, int ntx, int nty, int reverse, const T* xin, T* x,
                                                 const T* __restrict__ rin, T* __restrict__ rout,
                                                 double* __restrict__ part, int norm_mode, SweepIO<T> io) {
  lsgs_tile_body<T, TW, NT, NSW, true, IO>(L, ntx, nty, 0, xin, x, rin, rout, part, norm_mode, &io);
}

// many instances of one level: instance blockIdx.y, residual read from r
// (sel 0) or r2 (sel 1) and written to the other
template <typename T, int TW, int NT>
__global__ __launch_bounds__(NT) void kb_lsgs_tile(const BInst<T>* __restrict__ B, int ntx, int reverse, int sel) {
  const BInst<T>& a = B[blockIdx.y];
  if (!*a.active) return;
  lsgs_tile_body<T, TW, NT>(a.L, ntx, ntx, reverse, a.x, a.x, sel ? a.r2 : a.r, sel ? a.r : a.r2);
}

inline int tiles_along(int npts, int TW) { return (npts + TW - 1) / TW; }

// One workgroup per tile; the grid is padded to a multiple of 8 so that the
// XCD-aware tile order applies (spare workgroups exit at once).
//
// Tile shapes per level (measured on gfx950, us per sweep).  A tile of
// 1024 threads holds one CU (FP64 regions need 100-150 KB of LDS), so a sweep
// runs in rounds of 256 tiles and the tile edge is picked for whole rounds:
//   FP64  1025^2: 48 x 48 (484 tiles, 2 rounds) 33.1, 65 x 65 (256, 1) 28.7
//         2049^2: 48 x 48 (1849, 8 rounds) 108.9, 65 x 65 (1024, 4) 102.7
//         4097^2: 48 x 48 467.5, 56 x 56 439.1, 65 x 65 484.0
//          513^2: 48 x 48 18.1 (65 x 65: 24.8)
//   FP32 (512-thread tiles, 70 KB, two per CU): 48 x 48 except at 2049^2,
//         where 46 x 46 tiles (2025 tiles, 4 rounds of 512) take 55.9 against 58.8.
// Levels up to 257^2 vertices (FP64) or 513^2 (FP32) run one round of small
// tiles and are latency-bound: 16 x 16 tiles with 256 threads take about
// 10-15 us per sweep there instead of about 25 us (inside a cycle, the coarse
// levels up to 513^2 run two sweeps per launch instead, launch_lsgs_sweep2).
// (A persistent grid that
// keeps a workgroup per CU and prefetches the next tile's region measured
// slower at every size: 123 against 110 us at 2049^2 with 44 x 44 tiles and
// 768 threads, since its extra registers cap the threads per CU.)
inline int round8(int v) { return (v + 7) / 8 * 8; }

template <typename T>
struct SweepShape;
template <>
struct SweepShape<double> {
  static constexpr int TW = 48, NT = 1024;  // batched launches, 513^2
  static constexpr int kSmallMaxN = 256;    // n of the largest level swept with small tiles
};
template <>
struct SweepShape<float> {
  static constexpr int TW = 48, NT = 512;
  static constexpr int kSmallMaxN = 512;
};
constexpr int kSmallTW = 16, kSmallNT = 256;

// transfers of a launch: kIoProlong, kIoRestrict or kIoNone
template <typename T>
int io_kind(const SweepIO<T>* io) {
  return !io ? kIoNone : io->xc ? kIoProlong : io->fc ? kIoRestrict : kIoNone;
}

// the kernel of a tile shape with the launch's transfers (IO picked at run time)
template <typename T, int TW, int NT, int NSW, bool CGS>
hipError_t launch_tile_io(int nblocks, const Lev& L, int ntx, int reverse, const T* xin, T* x, const T* rin, T* rout,
                          hipStream_t s, double* part, int norm_mode, const SweepIO<T>* io) {
  const SweepIO<T> a = io ? *io : SweepIO<T>{};
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(NT), 0, s, L, ntx, ntx, reverse, xin, x, rin, rout, part, norm_mode,
                       a);
    return hipGetLastError();
  };
  switch (io_kind(io)) {
    case kIoProlong:
      if constexpr (CGS) return go(k_cgs_tile<T, TW, NT, NSW, kIoProlong>);
      else return go(k_lsgs_tile<T, TW, NT, NSW, kIoProlong>);
    case kIoRestrict:
      if constexpr (CGS) return go(k_cgs_tile<T, TW, NT, NSW, kIoRestrict>);
      else return go(k_lsgs_tile<T, TW, NT, NSW, kIoRestrict>);
    default:
      if constexpr (CGS) return go(k_cgs_tile<T, TW, NT, NSW>);
      else return go(k_lsgs_tile<T, TW, NT, NSW>);
  }
}

template <typename T, int TW, int NT, bool CGS>
hipError_t launch_tile(const Lev& L, int reverse, const T* xin, T* x, const T* rin, T* rout, hipStream_t s,
                       double* part, int norm_mode, int* nparts, const SweepIO<T>* io) {
  const int nt = tiles_along(L.n + 1, TW);
  if (nparts) *nparts = nt * nt;
  return launch_tile_io<T, TW, NT, 1, CGS>(round8(nt * nt), L, nt, CGS ? 0 : reverse, xin, x, rin, rout, s, part,
                                           norm_mode, io);
}

// the collective smoother (CGS = true) takes the LSGS tile shapes
template <typename T, bool CGS = false>
hipError_t launch_tile_cfg(const Lev& L, int reverse, const T* xin, T* x, const T* rin, T* rout, hipStream_t s,
                           double* part = nullptr, int norm_mode = 0, int* nparts = nullptr,
                           const SweepIO<T>* io = nullptr) {
  if (L.n <= SweepShape<T>::kSmallMaxN)
    return launch_tile<T, kSmallTW, kSmallNT, CGS>(L, reverse, xin, x, rin, rout, s, part, norm_mode, nparts, io);
  if constexpr (std::is_same<T, double>::value) {
    if (L.n == 1024 || L.n == 2048)
      return launch_tile<T, 65, 1024, CGS>(L, reverse, xin, x, rin, rout, s, part, norm_mode, nparts, io);
    if (L.n >= 4096)
      return launch_tile<T, 56, 1024, CGS>(L, reverse, xin, x, rin, rout, s, part, norm_mode, nparts, io);
  } else {
    if (L.n == 2048)
      return launch_tile<T, 46, 512, CGS>(L, reverse, xin, x, rin, rout, s, part, norm_mode, nparts, io);
  }
  return launch_tile<T, SweepShape<T>::TW, SweepShape<T>::NT, CGS>(L, reverse, xin, x, rin, rout, s, part, norm_mode,
                                                                   nparts, io);
}

}  // namespace

// Batched sweeps (launch_b_lsgs_sweep): one launch over every instance of a
// level, instance blockIdx.y.  The tile shape of each level is picked at batch
// setup by timing the candidates below on the batch's own buffers
// (b_sweep_shapes: their count; shape 0 is the default).
//   FP64: 48 x 48, 65 x 65, 56 x 56 (1024 threads, one tile per CU)
//   FP32: 48 x 48 (512 threads, corrections in LDS), 46 x 46 (512 threads,
//         one vertex per thread and phase), 65 x 65 (1024 threads)
template <typename T>
hipError_t launch_b_lsgs_sweep(const BInst<T>* d, int count, int n, int reverse, int sel, hipStream_t s, int shape) {
  auto go = [&](auto kern, int TW, int NT) {
    const int nt = tiles_along(n + 1, TW);
    hipLaunchKernelGGL(kern, dim3(round8(nt * nt), count), dim3(NT), 0, s, d, nt, reverse, sel);
    return hipGetLastError();
  };
  if constexpr (std::is_same<T, double>::value) {
    if (shape == 1) return go(kb_lsgs_tile<T, 65, 1024>, 65, 1024);
    if (shape == 2) return go(kb_lsgs_tile<T, 56, 1024>, 56, 1024);
    return go(kb_lsgs_tile<T, 48, 1024>, 48, 1024);
  } else {
    if (shape == 1) return go(kb_lsgs_tile<T, 46, 512>, 46, 512);
    if (shape == 2) return go(kb_lsgs_tile<T, 65, 1024>, 65, 1024);
    return go(kb_lsgs_tile<T, 48, 512>, 48, 512);
  }
}
template hipError_t launch_b_lsgs_sweep<double>(const BInst<double>*, int, int, int, int, hipStream_t, int);
template hipError_t launch_b_lsgs_sweep<float>(const BInst<float>*, int, int, int, int, hipStream_t, int);
int b_sweep_shapes() { return 3; }  // candidates of launch_b_lsgs_sweep per precision
int b_sweep_tile(int precision_fp32, int shape) {  // tile edge of a launch_b_lsgs_sweep shape
  static const int t64[3] = {48, 65, 56}, t32[3] = {48, 46, 65};
  return (shape < 0 || shape > 2) ? 0 : precision_fp32 ? t32[shape] : t64[shape];
}

template <>
hipError_t launch_lsgs_sweep<double>(const Lev& L, int reverse, double* x, const double* rin, double* rout,
                                     hipStream_t s) {
  return launch_tile_cfg<double>(L, reverse, x, x, rin, rout, s);
}

template <>
hipError_t launch_lsgs_sweep<float>(const Lev& L, int reverse, float* x, const float* rin, float* rout,
                                    hipStream_t s) {
  return launch_tile_cfg<float>(L, reverse, x, x, rin, rout, s);
}

template <>
hipError_t launch_lsgs_sweep_from<double>(const Lev& L, int reverse, const double* xin, double* x, const double* rin,
                                          double* rout, hipStream_t s, const SweepIO<double>* io) {
  return launch_tile_cfg<double>(L, reverse, xin, x, rin, rout, s, nullptr, 0, nullptr, io);
}

template <>
hipError_t launch_lsgs_sweep_from<float>(const Lev& L, int reverse, const float* xin, float* x, const float* rin,
                                         float* rout, hipStream_t s, const SweepIO<float>* io) {
  return launch_tile_cfg<float>(L, reverse, xin, x, rin, rout, s, nullptr, 0, nullptr, io);
}

// Two sweeps in one launch (bit s of revmask: sweep s in reverse colour
// order) on the coarse levels up to 513^2, where a sweep is about one
// latency-bound round of tiles: a 28-vertex halo, 14 colour phases, the
// corrections of both sweeps collected in LDS; 17 x 17 tiles up to 257^2,
// 33 x 33 tiles (256 of them) on 513^2.  r is read from rin and the residual
// after both sweeps written to rout.
constexpr int kSweep2MaxN = 512;
template <typename T, bool CGS>
hipError_t sweep2(const Lev& L, int revmask, const T* xin, T* x, const T* rin, T* rout, hipStream_t s,
                  const SweepIO<T>* io) {
  if (L.n > kSweep2MaxN) return hipErrorInvalidValue;
  if (L.n <= 256) {
    const int nt = tiles_along(L.n + 1, 17);
    return launch_tile_io<T, 17, 1024, 2, CGS>(round8(nt * nt), L, nt, CGS ? 0 : revmask, xin, x, rin, rout, s,
                                               nullptr, 0, io);
  }
  const int nt = tiles_along(L.n + 1, 33);
  return launch_tile_io<T, 33, 1024, 2, CGS>(round8(nt * nt), L, nt, CGS ? 0 : revmask, xin, x, rin, rout, s, nullptr,
                                             0, io);
}

template <typename T>
hipError_t launch_lsgs_sweep2(const Lev& L, int revmask, const T* xin, T* x, const T* rin, T* rout, hipStream_t s,
                              const SweepIO<T>* io) {
  return sweep2<T, false>(L, revmask, xin, x, rin, rout, s, io);
}
template hipError_t launch_lsgs_sweep2<double>(const Lev&, int, const double*, double*, const double*, double*,
                                               hipStream_t, const SweepIO<double>*);
template hipError_t launch_lsgs_sweep2<float>(const Lev&, int, const float*, float*, const float*, float*,
                                              hipStream_t, const SweepIO<float>*);
int lsgs_sweep2_max_n() { return kSweep2MaxN; }

hipError_t launch_lsgs_sweep_norm(const Lev& L, int reverse, const double* xin, double* x, const double* rin,
                                  double* rout, double* part, int norm_mode, int* nparts, hipStream_t s,
                                  const SweepIO<double>* io) {
  if (!part || (norm_mode != 1 && norm_mode != 2) || io_kind(io) == kIoRestrict) return hipErrorInvalidValue;
  return launch_tile_cfg<double>(L, reverse, xin, x, rin, rout, s, part, norm_mode, nparts, io);
}

// ---- collective point smoother: one or two fused sweeps per launch
template <typename T>
hipError_t launch_cgs_sweep_from(const Lev& L, const T* xin, T* x, const T* rin, T* rout, hipStream_t s,
                                 const SweepIO<T>* io) {
  return launch_tile_cfg<T, true>(L, 0, xin, x, rin, rout, s, nullptr, 0, nullptr, io);
}
template hipError_t launch_cgs_sweep_from<double>(const Lev&, const double*, double*, const double*, double*,
                                                  hipStream_t, const SweepIO<double>*);
template hipError_t launch_cgs_sweep_from<float>(const Lev&, const float*, float*, const float*, float*, hipStream_t,
                                                 const SweepIO<float>*);

template <typename T>
hipError_t launch_cgs_sweep2(const Lev& L, const T* xin, T* x, const T* rin, T* rout, hipStream_t s,
                             const SweepIO<T>* io) {
  return sweep2<T, true>(L, 0, xin, x, rin, rout, s, io);
}
template hipError_t launch_cgs_sweep2<double>(const Lev&, const double*, double*, const double*, double*,
                                              hipStream_t, const SweepIO<double>*);
template hipError_t launch_cgs_sweep2<float>(const Lev&, const float*, float*, const float*, float*, hipStream_t,
                                             const SweepIO<float>*);

hipError_t launch_cgs_sweep_norm(const Lev& L, const double* xin, double* x, const double* rin, double* rout,
                                 double* part, int norm_mode, int* nparts, hipStream_t s, const SweepIO<double>* io) {
  if (!part || (norm_mode != 1 && norm_mode != 2) || io_kind(io) == kIoRestrict) return hipErrorInvalidValue;
  return launch_tile_cfg<double, true>(L, 0, xin, x, rin, rout, s, part, norm_mode, nparts, io);
}

}  // namespace mgk
