// lbm_ehd_kernels.hpp -- kernels of the five-equation sweep and its helpers.
//
// k_sweep_batch is the hot path: one pass over the grid (or over the grids
// of a batch) advances f, h, p, n and g by one time step (pull streaming
// fused with the collisions).  Each
// workgroup of NW wavefronts owns a strip of 64 NW columns of a band of rows
// and walks down the band, one row per barrier, so that its waves read each
// row's lines together (the pull shifts and strip edges then fall in lines
// the workgroup is already fetching; measured on MI355X, four waves in step
// draw ~15 % more bandwidth than independent single-wave strips).  phi and
// psi, needed at the eight neighbours for the isotropic stencils (Eq. 59),
// are the moments of the *pulled* h and g of those neighbours, so the
// workgroup computes them one row ahead into a small LDS ring (4 rows x
// 64 NW + 2 columns, the two halo columns by threads 0 and 1) and each thread
// parks the pulled h and g of its node in LDS for the row's own update (with
// bfloat16 storage a third ring holds each node's momentum reference J~).
// Every population is read once and written once per step; only h and g of
// the two halo columns and of the rows just outside a band are read twice.
#pragma once

#include <type_traits>

#include "lbm_ehd_device.hpp"

namespace lbm {

template <class T>
__device__ inline const T* elem(const T* base, uint32_t e) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + e * (uint32_t)sizeof(T));
}

// Offsets of the pull sources of node (xc, yy): the population arriving along
// c_i comes from (xc - c_ix, yy - c_iy).  With side walls (halfway at
// x = -1/2 and nx - 1/2) the populations whose source lies beyond a wall are
// read elsewhere (see the pulls): lw / rw mark the wall columns.  ColsP is
// the form of the plain sweep (no side walls, no local field), whose flags
// are compile-time false: the flags alone, even when constant, change how
// the 16-bit sweeps are scheduled, and cost 1.6 % on MI355X at 2048^2.
struct Cols {
  int c, m, p;  // xc, xc - 1, xc + 1 (periodic in x)
  bool lw, rw;  // xc is next to the left / right side wall
};
struct ColsP {
  int c, m, p;
  static constexpr bool lw = false, rw = false;
};
// the form of the sweep that also has the local field of Eq. (50)
struct ColsL : Cols {};
// the plain form with the ions on D2Q9 (Eq. 34-38 as printed), and the form
// with side walls and the ions on D2Q9
struct ColsP9 : ColsP {};
struct ColsS9 : Cols {};

// Column type of sweep form EXT: 0 plain, 1 side walls, 2 side walls and the
// local field, 3 plain with the ions on D2Q9, 4 side walls with the ions on
// D2Q9.
template <int EXT>
using ColsOf = typename std::conditional<
    EXT == 0, ColsP,
    typename std::conditional<
        EXT == 1, Cols,
        typename std::conditional<
            EXT == 2, ColsL,
            typename std::conditional<EXT == 3, ColsP9, ColsS9>::type>::type>::type>::type;
template <class K>
constexpr bool ion9_of() {
  return std::is_same<K, ColsP9>::value || std::is_same<K, ColsS9>::value;
}

template <int EXT>
__device__ inline ColsOf<EXT> cols_for(int xc, int nx, int side) {
  ColsOf<EXT> k;
  k.c = xc;
  k.m = xc == 0 ? nx - 1 : xc - 1;
  k.p = xc == nx - 1 ? 0 : xc + 1;
  if constexpr (EXT == 1 || EXT == 2 || EXT == 4) {
    k.lw = side && xc == 0;
    k.rw = side && xc == nx - 1;
  }
  return k;
}

__device__ inline Cols cols_of(int xc, int nx, int side) { return cols_for<1>(xc, nx, side); }

// The diagonal directions 5-8 of a D2Q9 ion set whose diagonals sit in lines
// q9..q9+3: x[0..3] = directions 5..8.  At a side wall the ions bounce back:
// a diagonal coming through the wall is the node's own opposite one, read
// through the same load two lines up or down (lines are pitch apart).
template <class S, class R, class K>
__device__ inline void pull_diag(const PopView<S, R>& P, int q9, K k, int yy, R x[4]) {
  const uint32_t rm = P.row(yy), r0 = P.row(yy + 1), rp = P.row(yy + 2);
  const uint32_t pc = P.kp->pitch, own = r0 + k.c;
  x[0] = P.at(q9 + 0, k.lw ? own + 2 * pc : rm + k.m);  // <- 7
  x[1] = P.at(q9 + 1, k.rw ? own + 2 * pc : rm + k.p);  // <- 8
  x[2] = P.at(q9 + 2, k.rw ? own - 2 * pc : rp + k.p);  // <- 5
  x[3] = P.at(q9 + 3, k.lw ? own - 2 * pc : rp + k.m);  // <- 6
}
// Deviation content of the diagonals of the ion set at line q9 (0 unless
// the ions are on D2Q9), for the helpers outside the hot loop.
template <class S, class R, class K>
__device__ inline R ion_diag_sum(const PopView<S, R>& P, int q9, K k, int yy) {
  if (!P.kp->ion_q9) return R(0);
  R x[4];
  pull_diag(P, q9, k, yy, x);
  return x[0] + x[1] + x[2] + x[3];
}

// The f set of node (xc, yy).  At a side wall f bounces back (u = 0): the
// populations coming through the wall are the node's own opposite ones,
// read through the same line's load by shifting the offset to the other
// line (lines are pitch apart within a row).
template <class S, class R, class K>
__device__ inline void pull9(const PopView<S, R>& P, int q0, K k, int yy, R x[9]) {
  const uint32_t rm = P.row(yy), r0 = P.row(yy + 1), rp = P.row(yy + 2);
  const uint32_t pc = P.kp->pitch, own = r0 + k.c;
  x[0] = P.at(q0 + 0, own);
  x[1] = P.at(q0 + 1, k.lw ? own + 2 * pc : r0 + k.m);  // <- 3
  x[2] = P.at(q0 + 2, rm + k.c);
  x[3] = P.at(q0 + 3, k.rw ? own - 2 * pc : r0 + k.p);  // <- 1
  x[4] = P.at(q0 + 4, rp + k.c);
  x[5] = P.at(q0 + 5, k.lw ? own + 2 * pc : rm + k.m);  // <- 7
  x[6] = P.at(q0 + 6, k.rw ? own + 2 * pc : rm + k.p);  // <- 8
  x[7] = P.at(q0 + 7, k.rw ? own - 2 * pc : rp + k.p);  // <- 5
  x[8] = P.at(q0 + 8, k.lw ? own - 2 * pc : rp + k.m);  // <- 6
}

// The f set of node (xc, yy) as pulled by pull9, with the references of
// bfloat16 storage added back (LocalF): 3 w_i c_i . J~ of the node that sent
// population i, read at the same buffer position as the population (lines
// QJX, QJY); 0 for populations that come through a ghost row; for one
// reflected at a side wall (the node's own population of the opposite
// direction) the node's own reference of that direction.
template <class S, class R, class K, bool REFS = true>
__device__ inline void pull_f(const PopView<S, R>& P, K k, int yy, R x[9]) {
  pull9(P, QF, k, yy, x);
  if constexpr (LocalF<S>::value && REFS) {
    const uint32_t rm = P.row(yy), r0 = P.row(yy + 1), rp = P.row(yy + 2);
    const bool gd = yy == 0, gu = yy == P.kp->ny - 1;  // sources in a ghost row
    const uint32_t own = r0 + k.c;
    R ox = R(0), oy = R(0);
    if (k.lw || k.rw) {
      ox = P.at(QJX, own);
      oy = P.at(QJY, own);
    }
    // direction i pulled from element offset `off` (ghost: reference 0), or
    // at a side wall (`bb`) the node's own population of direction `opp`
    auto add = [&](int i, uint32_t off, bool ghost, bool bb, int opp) {
      if (bb) {
        x[i] += f_ref(opp, ox, oy);
      } else if (!ghost) {
        x[i] += f_ref(i, P.at(QJX, off), P.at(QJY, off));
      }
    };
    add(1, r0 + k.m, false, k.lw, 3);
    add(2, rm + k.c, gd, false, 4);
    add(3, r0 + k.p, false, k.rw, 1);
    add(4, rp + k.c, gu, false, 2);
    add(5, rm + k.m, gd, k.lw, 7);
    add(6, rm + k.p, gd, k.rw, 8);
    add(7, rp + k.p, gu, k.rw, 5);
    add(8, rp + k.m, gu, k.lw, 6);
  }
}

// J~ of the nodes of the sweep's ring rows with bfloat16 storage: the 16-bit
// patterns of lines QJX (low half) and QJY (high half) of each node, loaded
// once per row of a band instead of once per receiving neighbour (16 loads
// per node otherwise).  Other storage types keep no J~.
template <bool ON, int TW>
struct JRing {};
template <int TW>
struct JRing<true, TW> {
  uint32_t v[RING][TW + 2];
};
template <class S, class R>
__device__ inline uint32_t j_bits(const PopView<S, R>& P, int yy, int xc) {
  const uint32_t o = P.row(yy + 1) + xc;
  return (uint32_t)P.bits(QJX, o) | ((uint32_t)P.bits(QJY, o) << 16);
}
// The references of pull_f added to an f set pulled without them, with each
// sender's J~ taken from the ring: column c of slots sd, sc, su (rows yy - 1,
// yy, yy + 1).  The same sums, in the same order, as pull_f.
template <int TW, class K>
__device__ inline void add_f_refs(const JRing<true, TW>& J, int sd, int sc, int su, int c,
                                  int yy, int ny, K k, float x[9]) {
  const bool gd = yy == 0, gu = yy == ny - 1;  // sources in a ghost row
  const uint32_t own = J.v[sc][c];
  auto jx = [](uint32_t b) { return __uint_as_float(b << 16); };
  auto jy = [](uint32_t b) { return __uint_as_float(b & 0xFFFF0000u); };
  auto one = [&](int i, uint32_t b, bool ghost, bool bb, int opp) {
    if (bb) {
      x[i] += f_ref(opp, jx(own), jy(own));
    } else if (!ghost) {
      x[i] += f_ref(i, jx(b), jy(b));
    }
  };
  one(1, J.v[sc][c - 1], false, k.lw, 3);
  one(2, J.v[sd][c], gd, false, 4);
  one(3, J.v[sc][c + 1], false, k.rw, 1);
  one(4, J.v[su][c], gu, false, 2);
  one(5, J.v[sd][c - 1], gd, k.lw, 7);
  one(6, J.v[sd][c + 1], gd, k.rw, 8);
  one(7, J.v[su][c + 1], gu, k.rw, 5);
  one(8, J.v[su][c - 1], gu, k.lw, 6);
}

// Directions 1..4 of a D2Q5 set (the rest population is pulled separately).
// At a side wall the ion and potential populations bounce back (zero flux;
// on D2Q5 the same as specular reflection).
template <class S, class R, class K>
__device__ inline void pull4(const PopView<S, R>& P, int q0, K k, int yy, R x[4]) {
  const uint32_t rm = P.row(yy), r0 = P.row(yy + 1), rp = P.row(yy + 2);
  const uint32_t pc = P.kp->pitch, own = r0 + k.c;
  x[0] = P.at(q0 + 1, k.lw ? own + 2 * pc : r0 + k.m);  // <- 3
  x[1] = P.at(q0 + 2, rm + k.c);
  x[2] = P.at(q0 + 3, k.rw ? own - 2 * pc : r0 + k.p);  // <- 1
  x[3] = P.at(q0 + 4, rp + k.c);
}

// The h set of node (xc, yy): h0 from the rest plane (in place; also
// returned in its own wider type), h1..h8 pulled.  At a side wall h reflects
// specularly: the population coming through the wall is that of the mirror
// image of its source, i.e. the wall column's population in the x-mirrored
// direction one row up or down; where that row lies beyond an electrode (a
// corner), h bounces back.
template <class S, class R, class T0, class K>
__device__ inline void pull_h(const PopView<S, R>& P, const T0* __restrict__ h0x, K k,
                              int yy, R x[9], T0* h0 = nullptr) {
  const uint32_t rm = P.row(yy), r0 = P.row(yy + 1), rp = P.row(yy + 2);
  const uint32_t pc = P.kp->pitch, own = r0 + k.c;
  const bool ywalls = P.kp->walls != WALL_PERIODIC;
  const bool bot = ywalls && yy == 0, top = ywalls && yy == P.kp->ny - 1;
  const T0 r = *elem(h0x, (uint32_t)yy * pc + k.c);
  if (h0) *h0 = r;
  x[0] = (R)rest_val(r);
  x[1] = P.at(QH + 1, k.lw ? own + 2 * pc : r0 + k.m);                    // <- 3
  x[2] = P.at(QH + 2, rm + k.c);
  x[3] = P.at(QH + 3, k.rw ? own - 2 * pc : r0 + k.p);                    // <- 1
  x[4] = P.at(QH + 4, rp + k.c);
  x[5] = P.at(QH + 5, !k.lw ? rm + k.m : (bot ? own + 2 * pc : rm + k.c + pc));  // <- 6 / 7
  // at the right wall the load is based at line 5: in the bottom ghost row
  // (row 0) of a y-periodic box the specular source rm + c - pc of line 6
  // would be a negative offset, which the buffer's range check reads as zero
  x[6] = !k.rw ? P.at(QH + 6, rm + k.p)
               : P.at(QH + 5, bot ? own + 3 * pc : rm + k.c);  // <- 5 / 8
  x[7] = P.at(QH + 7, !k.rw ? rp + k.p : (top ? own - 2 * pc : rp + k.c + pc));  // <- 8 / 5
  x[8] = P.at(QH + 8, !k.lw ? rp + k.m : (top ? own - 2 * pc : rp + k.c - pc));  // <- 7 / 6
  if (LocalH<S>::value) {
    const R t = P.at(QH, r0 + k.c);  // the node's own reference phase
#pragma unroll
    for (int i = 1; i < 9; ++i) x[i] = h_from(x[i], i, t);
  }
}

// Rest population (deviation) of the ion set starting at line q0 (QP or QN)
// of node (x, y): from its FP64 plane (16-bit storage) or from line q0.
template <class S, class R, class T0>
__device__ inline double ion_rest(const PopView<S, R>& P, const T0* __restrict__ h0x, int q0,
                                  int x, int y) {
  if constexpr (IonRest<S>::value)
    return rest_val(*elem(h0x, (uint32_t)(q0 == QP ? 1 : 2) * P.kp->cells +
                                   (uint32_t)y * P.kp->pitch + x));
  return (double)P.at(q0, P.row(y + 1) + x);
}

// Directions 1..4 of the g set of node (xc, yy), as deviations from the
// uncharged steady state (with 16-bit storage: stored relative to psi'~ / 6
// of the node itself, see LocalG).
template <class S, class R, class K>
__device__ inline void pull_g(const PopView<S, R>& P, K k, int yy, R x[4]) {
  pull4(P, QG, k, yy, x);
  if (LocalG<S>::value) {
    const R t = P.at(QRG, P.row(yy + 1) + k.c) * R(1.0 / 6.0);
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] += t;
  }
}
// g0 of node (x, yy), as a deviation.
template <class S, class R>
__device__ inline R g_rest(const PopView<S, R>& P, int x, int yy) {
  const uint32_t o = P.row(yy + 1) + x;
  R g0 = P.at(QG, o);
  if (LocalG<S>::value) g0 -= R(2.0 / 3.0) * P.at(QRG, o);
  return g0;
}

template <class R>
__device__ inline R sum9(const R h[9]) {
  return h[0] + h[1] + h[2] + h[3] + h[4] + h[5] + h[6] + h[7] + h[8];
}
// phi' of Eq. (33) in the ring type RP, from the wide rest population and the
// eight pulled ones
template <class RP, class R>
__device__ inline RP phi_of(RP h0, const R h[9]) {
  RP s = h0;
#pragma unroll
  for (int i = 1; i < 9; ++i) s += (RP)h[i];
  return s;
}
// psi' of Eq. (49): 1/(1 - 1/3) = 3/2 times the deviations of g1..g4 (their
// references add up to psi_lin of the node's row)
template <class R>
__device__ inline R psi_of(const R g4[4]) {
  return R(1.5) * (g4[0] + g4[1] + g4[2] + g4[3]);
}
// the same sum in the wider type T
template <class T, class R>
__device__ inline T psi_as(const R g4[4]) {
  return T(1.5) * ((T)g4[0] + (T)g4[1] + (T)g4[2] + (T)g4[3]);
}

// Neighbourhood of a node from three rows (down, centre, up), each given as
// columns (x-1, x, x+1), in velocity order.
template <class R>
__device__ inline void nine(const R d[3], const R c[3], const R u[3], R o[9]) {
  o[0] = c[1];
  o[1] = c[2];
  o[2] = u[1];
  o[3] = c[0];
  o[4] = d[1];
  o[5] = u[2];
  o[6] = u[0];
  o[7] = d[0];
  o[8] = d[2];
}

// Wall ghosts of the stencils: phi mirrored, psi odd about the wall value.
// In deviation form the wall value of psi' is 0 at both electrodes.
template <class RP, class R>
__device__ inline void ghost_row(const RP phc[3], const R psc[3], RP phg[3], R psg[3]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    phg[j] = phc[j];
    psg[j] = -psc[j];
  }
}

// Ghost-row writes of a node on a wall row (or on an edge row of a
// y-periodic box).  At a wall, the population that comes back along c_i to
// node x is pulled at step t+1 from ghost column x - c_ix; in a periodic box
// the ghost row receives the populations leaving the opposite edge.  Values
// are deviations (the wall rules below are written for them).
template <class S, class R, class K>
struct Ghosts {
  const PopView<S, R>& D;
  const KP<R>& kp;
  int y;
  K k;
  __device__ inline uint32_t top() const { return D.row(kp.ny + 1); }
  // D2Q9 set starting at plane q0 (f or h): bounce-back at walls
  __device__ inline void set9(int q0, const R x[9]) const {
    if (kp.walls == WALL_PERIODIC) {
      if (y == kp.ny - 1) { D.put(q0 + 2, k.c, x[2]); D.put(q0 + 5, k.c, x[5]); D.put(q0 + 6, k.c, x[6]); }
      if (y == 0) {
        D.put(q0 + 4, top() + k.c, x[4]); D.put(q0 + 7, top() + k.c, x[7]);
        D.put(q0 + 8, top() + k.c, x[8]);
      }
      return;
    }
    if (y == 0) { D.put(q0 + 2, k.c, x[4]); D.put(q0 + 5, k.m, x[7]); D.put(q0 + 6, k.p, x[8]); }
    if (y == kp.ny - 1) {
      D.put(q0 + 4, top() + k.c, x[2]); D.put(q0 + 7, top() + k.p, x[5]);
      D.put(q0 + 8, top() + k.m, x[6]);
    }
  }
  // D2Q5 set: reflected value at the bottom and top walls given by the caller
  __device__ inline void set5(int q0, const R x[5], R bottom, R topv) const {
    if (kp.walls == WALL_PERIODIC) {
      if (y == kp.ny - 1) D.put(q0 + 2, k.c, x[2]);
      if (y == 0) D.put(q0 + 4, top() + k.c, x[4]);
      return;
    }
    if (y == 0) D.put(q0 + 2, k.c, bottom);
    if (y == kp.ny - 1) D.put(q0 + 4, top() + k.c, topv);
  }
};

// Ghost-row writes of a D2Q9 ion set (lines q0.. for directions 0-4, q9..
// for 5-8) of a node on an electrode row (or an edge row of a y-periodic
// box): the populations that come back through the wall, by the rule of the
// electrode in deviation form (reference w_i c0): kind 0 ion-tight,
// bounce-back x*_opp; kind 1, c = 0 at the wall, -x*_opp - 2 w_i c0; kind 2,
// dc/dn = 0, -x*_opp + 2 w_i c' with c' the node's own c - c0.
template <class S, class R, class K>
__device__ inline void ion9_ghosts(const PopView<S, R>& D, const KP<R>& kp, int y, K k, int q0,
                                   int q9, const R x[9], int bottom, int topk, R cd) {
  const uint32_t top = D.row(kp.ny + 1);
  if (kp.walls == WALL_PERIODIC) {
    if (y == kp.ny - 1) {
      D.put(q0 + 2, k.c, x[2]);
      D.put(q9 + 0, k.c, x[5]);
      D.put(q9 + 1, k.c, x[6]);
    }
    if (y == 0) {
      D.put(q0 + 4, top + k.c, x[4]);
      D.put(q9 + 2, top + k.c, x[7]);
      D.put(q9 + 3, top + k.c, x[8]);
    }
    return;
  }
  const R a2 = R(2.0 / 9.0), d2 = R(1.0 / 18.0);  // 2 w_i, axis and diagonal
  auto rule = [&](R v, R w2, int kind) {
    return kind == 0 ? v : (kind == 1 ? -v - w2 * kp.c0 : -v + w2 * cd);
  };
  if (y == 0) {
    D.put(q0 + 2, k.c, rule(x[4], a2, bottom));
    D.put(q9 + 0, k.m, rule(x[7], d2, bottom));
    D.put(q9 + 1, k.p, rule(x[8], d2, bottom));
  }
  if (y == kp.ny - 1) {
    D.put(q0 + 4, top + k.c, rule(x[2], a2, topk));
    D.put(q9 + 2, top + k.p, rule(x[5], d2, topk));
    D.put(q9 + 3, top + k.m, rule(x[6], d2, topk));
  }
}

// Store the post-collision g of node (x, y) (deviations, g[0..4]) with the
// electrode rules.  psi9 is the psi' neighbourhood: with 16-bit storage each
// moving population is stored relative to psi'~ / 6 of the node it arrives
// at (the node itself for the populations an electrode sends back), g0
// relative to -2/3 psi'~ of the node, and the node stores its own psi'~.
template <class S, class R, class K, class P9>
__device__ inline void store_g(const PopView<S, R>& D, const KP<R>& kp, int x, int y, K k,
                               const R g[5], const P9 psi9[9]) {
  const uint32_t o = D.row(y + 1) + x;
  const Ghosts<S, R, K> G{D, kp, y, k};
  const bool edge = y == 0 || y == kp.ny - 1;
  if (!LocalG<S>::value) {
#pragma unroll
    for (int i = 0; i < 5; ++i) D.put(QG + i, o, g[i]);
    // psi = dpsi at the anode, 0 at the cathode: -x*_opp in deviation form
    if (edge) G.set5(QG, g, -g[4], -g[2]);
    return;
  }
  R t[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) t[i] = D.stored(QRG, (R)psi9[i]);
  if (k.lw) t[3] = t[0];
  if (k.rw) t[1] = t[0];
  if (kp.walls != WALL_PERIODIC) {
    if (y == 0) t[4] = t[0];
    if (y == kp.ny - 1) t[2] = t[0];
  }
  D.put(QRG, o, t[0]);
  const R sixth = R(1.0 / 6.0);
  R e[5];
  e[0] = g[0] + R(2.0 / 3.0) * t[0];
#pragma unroll
  for (int i = 1; i < 5; ++i) e[i] = g[i] - t[i] * sixth;
#pragma unroll
  for (int i = 0; i < 5; ++i) D.put(QG + i, o, e[i]);
  if (edge) G.set5(QG, e, -g[4] - t[0] * sixth, -g[2] - t[0] * sixth);
}

// Per-node update once the pulled populations and the phi'/psi'
// neighbourhood are known: macroscopic quantities, then the five collisions,
// each stored as soon as it is done.  h and g (directions 1-4) of the node
// are fetched through `hg` right before their collisions; they were pulled one
// row earlier and parked in LDS.
//
// Wall rules in deviation form: bounce-back keeps the deviation; the
// anti-bounce-back of an ion with wall concentration c_w stores
// -x*_opp + 2 wbar (c_w - c0), i.e. -x*_opp - c0/3 for c_w = 0 and
// -x*_opp + c'/3 for c_w = c(node); for g the linear potential meets the
// electrode potentials exactly, so the rule is -x*_opp.
template <class S, class R, class T0, bool STD, class HG, class K>
__device__ inline void update_node(const PopView<S, R>& D, R* __restrict__ jprev,
                                   const T0* __restrict__ h0src, T0* __restrict__ h0dst,
                                   const KP<R>& kp, const KP<typename WorkOf<S>::type>& kpw, int x,
                                   int y, K k, const typename WorkOf<S>::type phi9[9],
                                   const typename WorkOf<S>::type psi9[9], R f[9], R p[9],
                                   R n[9], R g0,
                                   const HG& hg) {
  // Working type W: the wide type (FP64 with FP32 storage) for the
  // macroscopic quantities and all five collisions.  In FP32 the pressure
  // and the potential, which the method integrates over many steps with
  // little damping, random-walk away at the 1e-5 level over 20k steps, and
  // the rounding of an FP32 h collision reaches the velocity of a slow,
  // nearly steady flow (3e-5 after 160 000 steps of a droplet in a closed
  // box); in FP64 they stay at the storage's rounding.
  typedef typename WorkOf<S>::type W;
  // the ions on D2Q9 (Eq. 34-38 as printed): nine populations per species
  constexpr bool I9 = ion9_of<K>();
  constexpr int QI = I9 ? 9 : 5;
  W fw[9], pw[QI], nw[QI], ps9[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    fw[i] = (W)f[i];
    ps9[i] = (W)psi9[i];
  }
#pragma unroll
  for (int i = 0; i < QI; ++i) {
    pw[i] = (W)p[i];
    nw[i] = (W)n[i];
  }
  const uint32_t jo = (uint32_t)y * kp.pitch + x;
  // exact incoming ion content of the node (FP64 ion rest populations)
  double Pin = 0.0, Qin = 0.0;
  if constexpr (IonRest<S>::value) {
    Pin = rest_val(*elem(h0src, kp.cells + jo));
    Qin = rest_val(*elem(h0src, 2 * kp.cells + jo));
    pw[0] = (W)Pin;
    nw[0] = (W)Qin;
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      Pin += (double)p[i];
      Qin += (double)n[i];
    }
  }
  W Pd = pw[0] + pw[1] + pw[2] + pw[3] + pw[4];
  W Qd = nw[0] + nw[1] + nw[2] + nw[3] + nw[4];
  if constexpr (I9) {
    Pd = Pd + pw[5] + pw[6] + pw[7] + pw[8];
    Qd = Qd + nw[5] + nw[6] + nw[7] + nw[8];
  }
  // the local field of Eq. (50), from the node's incoming g (its own form
  // of the sweep)
  W Eg[2];
  const W* Eloc = nullptr;
  if constexpr (std::is_same<K, ColsL>::value) {
    if (kp.local_field) {
      R gl[4];
      hg.g4(gl);
      field_from_g(gl, kpw, Eg);
      Eloc = Eg;
    }
  }
  Macro<W> m;
  macro(phi9, ps9, Pd, Qd, fw, kpw, m, Eloc);

  const uint32_t o = D.row(y + 1) + x;
  const bool edge = y == 0 || y == kp.ny - 1;
  const Ghosts<S, R, K> G{D, kp, y, k};
  const bool ins = kp.walls == WALL_INSULATING;
  const R third = R(1) / R(3);

  // f first: its nine wide populations are then free for the rest
  collide_f<STD>(fw, m, kpw);
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = (R)fw[i];
  if constexpr (LocalF<S>::value) {
    // this node's momentum, the reference of the moving f it sends
    const R jx = D.stored(QJX, (R)(m.rho * m.u[0])), jy = D.stored(QJY, (R)(m.rho * m.u[1]));
    D.put(QJX, o, jx);
    D.put(QJY, o, jy);
    D.put(QF, o, f[0]);
#pragma unroll
    for (int i = 1; i < 9; ++i) D.put(QF + i, o, f[i] - f_ref(i, jx, jy));
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) D.put(QF + i, o, f[i]);
  }
  // the ghost rows hold f relative to 0
  if (edge) G.set9(QF, f);

  {  // g: Eq. (44)-(47)
    R g4[4];
    hg.g4(g4);
    W gw[5] = {(W)g0, (W)g4[0], (W)g4[1], (W)g4[2], (W)g4[3]};
    collide_g<STD>(gw, m.psid, poisson_source<W>(m.rhoe, m.ieps, m.geps, m.gpsi, kpw), kpw);
    R g[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = (R)gw[i];
    store_g(D, kp, x, y, k, g, psi9);
  }

  if constexpr (I9) {
    collide_ion9<STD>(pw, m.cpd, m.mup, m.itau_p, kpw.mask_p, W(-1), m, kpw);
    collide_ion9<STD>(nw, m.cmd, m.mum, m.itau_n, kpw.mask_n, W(1), m, kpw);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      p[i] = (R)pw[i];
      n[i] = (R)nw[i];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) D.put(i < 5 ? QP + i : QP9 + i - 5, o, p[i]);
#pragma unroll
    for (int i = 0; i < 9; ++i) D.put(i < 5 ? QN + i : QN9 + i - 5, o, n[i]);
    if (edge) {
      const R cpd = (R)m.cpd, cmd = (R)m.cmd;
      // anode: c+ = 0, d c-/dn = 0; cathode: d c+/dn = 0, c- = 0
      ion9_ghosts(D, kp, y, k, QP, QP9, p, ins ? 0 : 1, ins ? 0 : 2, cpd);
      ion9_ghosts(D, kp, y, k, QN, QN9, n, ins ? 0 : 2, ins ? 0 : 1, cmd);
    }
  } else {
  collide_ion<STD>(pw, m.cpd, m.mup, m.itau_p, kpw.mask_p, W(-1), m, kpw);
  collide_ion<STD>(nw, m.cmd, m.mum, m.itau_n, kpw.mask_n, W(1), m, kpw);
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    p[i] = (R)pw[i];
    n[i] = (R)nw[i];
  }
  if constexpr (IonRest<S>::value) {
    // the collision adds the reaction term to each ion's content (Eq. 41);
    // the rest populations take what the stored moving ones leave of it
    double Pout = Pin + (double)m.Rr, Qout = Qin + (double)m.Rr;
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      D.put(QP + i, o, p[i]);
      Pout -= (double)D.stored(QP + i, p[i]);
    }
    *elem(h0dst, kp.cells + jo) = (T0)Pout;
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      D.put(QN + i, o, n[i]);
      Qout -= (double)D.stored(QN + i, n[i]);
    }
    *elem(h0dst, 2 * kp.cells + jo) = (T0)Qout;
  } else {
#pragma unroll
    for (int i = 0; i < 5; ++i) D.put(QP + i, o, p[i]);
#pragma unroll
    for (int i = 0; i < 5; ++i) D.put(QN + i, o, n[i]);
  }
  const R cpd = (R)m.cpd, cmd = (R)m.cmd;
  // anode: c+ = 0; cathode: d c+/dn = 0 (wall value = node value)
  if (edge) G.set5(QP, p, ins ? p[4] : -p[4] - third * kp.c0, ins ? p[2] : -p[2] + third * cpd);
  // anode: d c-/dn = 0; cathode: c- = 0
  if (edge) G.set5(QN, n, ins ? n[4] : -n[4] + third * cmd, ins ? n[2] : -n[2] - third * kp.c0);
  }

  {  // h: Eq. (27)-(32), with d(phi u)/dt of Eq. (58), in W.  (phi u)(t) is
    // rounded to the type it is kept in before the difference is taken, so
    // that the differences of successive steps telescope: the rounding of
    // (phi u)(t-1) alone would enter every step with the same sign wherever
    // the flow is steady.
    const uint32_t jpl = kp.cells;
    const R Jx = (R)(m.phi * m.u[0]), Jy = (R)(m.phi * m.u[1]);
    const W dJ[2] = {(W)Jx - (W)*elem(jprev, jo), (W)Jy - (W)*elem(jprev, jpl + jo)};
    *elem(jprev, jo) = Jx;
    *elem(jprev, jpl + jo) = Jy;
    const T0 h0in = *elem(h0src, jo);
    R h[9];
    hg.h9(h);
    // the node's phi content: its rest plus its incoming h (see RestOf)
    RestAcc<T0> mass = RestAcc<T0>::from_rest(h0in);
#pragma unroll
    for (int i = 1; i < 9; ++i) mass.add(h[i]);
    W hw[9];
    hw[0] = (W)rest_val(h0in);
#pragma unroll
    for (int i = 1; i < 9; ++i) hw[i] = (W)h[i];
    collide_h<STD>(hw, m, dJ, kpw);
#pragma unroll
    for (int i = 0; i < 9; ++i) h[i] = (R)hw[i];
    // reference phase of each destination (16-bit storage; 0 otherwise):
    // phi'~ of node x + c_i, or of the node itself for populations that a
    // wall sends back to it
    R t[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) t[i] = R(0);
    if (LocalH<S>::value) {
#pragma unroll
      for (int i = 0; i < 9; ++i) t[i] = D.stored(QH, (R)phi9[i]);
      // a population sent through a side wall arrives, reflected, at the
      // mirror image of its destination: the node itself, or its neighbour
      // up or down
      if (k.lw) { t[3] = t[0]; t[6] = t[2]; t[7] = t[4]; }
      if (k.rw) { t[1] = t[0]; t[5] = t[2]; t[8] = t[4]; }
      if (kp.walls != WALL_PERIODIC) {  // (after the side walls: corners)
        if (y == 0) t[4] = t[7] = t[8] = t[0];
        if (y == kp.ny - 1) t[2] = t[5] = t[6] = t[0];
      }
      D.put(QH, o, t[0]);  // this node's reference for the next step
    }
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      h[i] = D.stored(QH + i, h[i] - (R)W9F[i] * t[i]);
      D.put(QH + i, o, h[i]);
      mass.sub(h_from(h[i], i, t[i]));
    }
    // the rest population takes what the eight stored ones leave of the content
    *elem(h0dst, jo) = mass.rest();
    if (edge) G.set9(QH, h);
  }

}

// Type the pulled h1-h8 and g1-g4 are parked in: the storage type where the
// pulls are its values widened (FP32 storage with FP64 arithmetic: exact, and
// half the LDS, so that four workgroups of four waves fit on a CU instead of
// two), else the pull type.
template <class S, class R>
struct ParkOf {
  typedef R type;
};
template <>
struct ParkOf<float, double> {
  typedef float type;
};
// h1-h8 and g1-g4 of one node parked in LDS, one column per thread (h0 is
// read again from the rest plane in its wider type).
template <class R, class P, int TW>
struct HGLds {
  const P (*s)[TW];
  int lane;
  __device__ inline void h9(R o[9]) const {
    o[0] = R(0);
#pragma unroll
    for (int i = 1; i < 9; ++i) o[i] = (R)s[i - 1][lane];
  }
  __device__ inline void g4(R o[4]) const {
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = (R)s[8 + i][lane];
  }
};

// The psi' ring of a sweep workgroup, in the working type W.  With FP32
// storage (W = FP64) it holds each value as its FP32 rounding plus the
// bfloat16 rounding of the remainder: about 32 significant bits in 6 bytes.
// A plain FP32 ring (24 bits), whose rounding is the same at every step where
// the potential is steady, drove the velocity of a slow nearly steady flow
// 2e-5 away from the oracle over 160 000 steps (1e-5, the floor of FP32
// storage, with an FP64 ring); a full FP64 ring leaves too little LDS for
// two 8-wave or four 4-wave workgroups per CU (-18 % / -3 % at 2048^2 on
// MI355X).
template <class S, class W, int TW>
struct PsiRing {
  W v[RING][TW + 2];
  __device__ inline void set(int s, int c, W x) { v[s][c] = x; }
  __device__ inline W get(int s, int c) const { return v[s][c]; }
};
template <int TW>
struct PsiRing<float, double, TW> {
  float hi[RING][TW + 2];
  uint16_t lo[RING][TW + 2];
  __device__ inline void set(int s, int c, double x) {
    const float h = (float)x;
    uint32_t b = __float_as_uint((float)(x - (double)h));
    b += 0x7FFFu + ((b >> 16) & 1u);  // to nearest, ties to even
    hi[s][c] = h;
    lo[s][c] = (uint16_t)(b >> 16);
  }
  __device__ inline double get(int s, int c) const {
    return (double)hi[s][c] + (double)__uint_as_float((uint32_t)lo[s][c] << 16);
  }
};

// LDS of one sweep workgroup: the phi' ring (in the working type W), the
// psi' ring, the parked h1-h8, g1-g4 and, with bfloat16 storage, the J~ ring.
template <class S, class R, int TW>
struct SweepLds {
  typename WorkOf<S>::type phi[RING][TW + 2];
  PsiRing<S, typename WorkOf<S>::type, TW> psi;
  typename ParkOf<S, R>::type pull[2][12][TW];  // pulled h1-8 and g1-4 of a row, by row parity
  JRing<LocalF<S>::value, TW> jref;
};

// One tile of the fused sweep: columns [x0, x0 + 64 NW) of rows [y0, yend)
// of one simulation, walked down row by row by the whole workgroup.
template <class S, class R, class T0, int NW, int EXT, bool STD>
__device__ inline void sweep_tile(SweepLds<S, R, 64 * NW>& L,
                                  const S* __restrict__ src, S* __restrict__ dst,
                                  R* __restrict__ jprev, const T0* __restrict__ h0x,
                                  T0* __restrict__ h0dst, const KP<R>& kp,
                                  const KP<typename WorkOf<S>::type>& kpw, int x0, int y0,
                                  int yend) {
  typedef typename WorkOf<S>::type W;
  constexpr int TW = 64 * NW;
  const int nx = kp.nx, ny = kp.ny;
  const int w = min(TW, nx - x0);
  const int lane = threadIdx.x;
  const bool valid = lane < w;
  const int x = x0 + (valid ? lane : 0);
  // side walls and the local field are compiled in only where a member of
  // the launch has them
  const bool side = EXT != 0 && kp.side_walls;
  const ColsOf<EXT> k = cols_for<EXT>(x, nx, kp.side_walls);
  const bool periodic = kp.walls == WALL_PERIODIC;
  // Non-temporal population loads pay off where a strip's row of one line
  // spans at least 1 KB.  In narrower strips the column-shifted pulls at the
  // strip edges reach into cache lines that the neighbouring strip also
  // reads, and evict-first makes HBM serve them twice.  Measured on MI355X:
  // single grids with 1-2 KB strips gain 4-14 % (FP32 512^2 to 2048^2, FP16
  // 2048^2); the batched FP16 droplets of 128^2 to 1024^2 lose 23 % in
  // 128-byte strips and 9 % in 512-byte ones.
  constexpr bool kNT = 64 * NW * sizeof(S) >= 1024;
  const PopView<S, R> Ph{make_rsrc(src, kp.pop_bytes), &kp, kNT};
  // the ring rows that the neighbouring bands pull too are loaded cached
  const PopView<S, R> Pc{make_rsrc(src, kp.pop_bytes), &kp, false};
  const PopView<S, R> D{make_rsrc(dst, kp.pop_bytes), &kp};

  // halo column handled by lanes 0 (left) and 1 (right); beyond a side wall
  // the stencils see the mirror image, i.e. the wall column itself
  const int xh = lane == 0 ? (x0 == 0 ? (side ? 0 : nx - 1) : x0 - 1)
                           : (x0 + w == nx ? (side ? nx - 1 : 0) : x0 + w);
  const ColsOf<EXT> kh = cols_for<EXT>(xh, nx, kp.side_walls);
  const int kcol = lane == 0 ? 0 : w + 1;

  auto slot = [&](int yy) { return (yy - y0 + 1) % RING; };
  // phi', psi' of row yy into the ring; each thread's own pulls are parked
  // in LDS.  The h and g lines of the ring rows are loaded cached with FP32
  // storage and arithmetic; with FP64 storage, or FP32 storage and FP64
  // arithmetic, those of the two ring rows at each end of the band, which the
  // neighbouring band (put on the same XCD soon after by the tile order) pulls
  // too; the others non-temporal.  Measured on
  // MI355X at 2048^2 against all non-temporal: the end rows cached, FP32
  // +1.7 % (bands of 16) / +3.1 % (bands of 8), FP64 +1.1 %, FP16 -0.4 % (and
  // -7 % for the batched FP16 droplets of 128^2 to 1024^2, whose short bands
  // make most ring rows edge rows); every ring row cached, FP32 +2.7 %, FP16
  // -2.6 %, FP64 -4 % (and, with the specialised sweep and 280 B/LUP, FP32
  // +0.8 % but FP32 storage with FP64 arithmetic -2.6 % over the end rows
  // only).
  auto ring_row = [&](int yy) {
    const int ys = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
    const int sl = slot(yy);
    auto pulls = [&](const PopView<S, R>& V) {
      // With FP64 storage each thread's own loads are issued before the halo
      // lanes' block, so that the wave holding those lanes waits once for
      // both sets (+1.4 % at 2048^2 on MI355X); the 16-bit forms lose 1-3 %
      // that way (longer live ranges), FP32 is even.
      constexpr bool kOwnFirst = sizeof(S) == 8;
      R h[9], g4[4];
      T0 h0;
      if (kOwnFirst && valid) {
        pull_h(V, h0x, k, ys, h, &h0);
        pull_g(V, k, ys, g4);
      }
      if (lane < 2) {
        R hh[9], gg[4];
        T0 hh0;
        pull_h(V, h0x, kh, ys, hh, &hh0);
        pull_g(V, kh, ys, gg);
        L.phi[sl][kcol] = phi_of<W>((W)rest_val(hh0), hh);
        L.psi.set(sl, kcol, psi_as<W>(gg));
        if constexpr (LocalF<S>::value) L.jref.v[sl][kcol] = j_bits(V, ys, kh.c);
      }
      if (valid) {
        if (!kOwnFirst) {
          pull_h(V, h0x, k, ys, h, &h0);
          pull_g(V, k, ys, g4);
        }
        L.phi[sl][lane + 1] = phi_of<W>((W)rest_val(h0), h);
        L.psi.set(sl, lane + 1, psi_as<W>(g4));
        if constexpr (LocalF<S>::value) L.jref.v[sl][lane + 1] = j_bits(V, ys, k.c);
        const int b = (yy - y0 + 2) & 1;
#pragma unroll
        for (int i = 1; i < 9; ++i) L.pull[b][i - 1][lane] = (typename ParkOf<S, R>::type)h[i];
#pragma unroll
        for (int i = 0; i < 4; ++i) L.pull[b][8 + i][lane] = (typename ParkOf<S, R>::type)g4[i];
      }
    };
    if (kNT && ((sizeof(S) == 4 && sizeof(R) == 4) || (sizeof(S) >= 4 && (yy <= y0 || yy >= yend - 1))))
      pulls(Pc);
    else
      pulls(Ph);
  };

  if (y0 > 0 || periodic) ring_row(y0 - 1);
  ring_row(y0);

  for (int y = y0; y < yend; ++y) {
    const bool up = y + 1 < ny || periodic;
    const bool down = y > 0 || periodic;
    // The row's own f, p, n and g0 are requested before the ring row, so that
    // both sets of loads are in flight together (one memory round trip per
    // row instead of two).  Lanes past the grid edge read column x0.  The
    // loads are issued at raised wave priority: a wave starting its row gets
    // its ~46 loads out ahead of the arithmetic of the other waves on its
    // SIMD (measured on MI355X at 2048^2: +1.2 % FP32, +1.6 % FP16; the
    // level, 1 to 3, makes no difference).
    R f[9], p[9], n[9], t4[4];
    __builtin_amdgcn_s_setprio(2);
    pull_f<S, R, ColsOf<EXT>, false>(Ph, k, y, f);  // (references: after the barrier)
    const uint32_t r0 = Ph.row(y + 1);
    // (the ion rest populations of 16-bit storage are read by the update)
    p[0] = IonRest<S>::value ? R(0) : Ph.at(QP, r0 + x);
    n[0] = IonRest<S>::value ? R(0) : Ph.at(QN, r0 + x);
    const R g0 = g_rest(Ph, x, y);
    pull4(Ph, QP, k, y, t4);
    p[1] = t4[0]; p[2] = t4[1]; p[3] = t4[2]; p[4] = t4[3];
    pull4(Ph, QN, k, y, t4);
    n[1] = t4[0]; n[2] = t4[1]; n[3] = t4[2]; n[4] = t4[3];
    if constexpr (EXT == 3 || EXT == 4) {  // the D2Q9 ions' diagonals
      pull_diag(Ph, QP9, k, y, t4);
      p[5] = t4[0]; p[6] = t4[1]; p[7] = t4[2]; p[8] = t4[3];
      pull_diag(Ph, QN9, k, y, t4);
      n[5] = t4[0]; n[6] = t4[1]; n[7] = t4[2]; n[8] = t4[3];
    }
    if (up) ring_row(y + 1);
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    if (valid) {
      const int c = lane + 1, sc = slot(y);
      W phC[3] = {L.phi[sc][c - 1], L.phi[sc][c], L.phi[sc][c + 1]};
      W psC[3] = {L.psi.get(sc, c - 1), L.psi.get(sc, c), L.psi.get(sc, c + 1)};
      W phU[3], phD[3];
      W psU[3], psD[3];
      if (up) {
        const int su = slot(y + 1);
        phU[0] = L.phi[su][c - 1]; phU[1] = L.phi[su][c]; phU[2] = L.phi[su][c + 1];
        psU[0] = L.psi.get(su, c - 1); psU[1] = L.psi.get(su, c); psU[2] = L.psi.get(su, c + 1);
      } else {
        ghost_row(phC, psC, phU, psU);
      }
      if (down) {
        const int sd = slot(y - 1);
        phD[0] = L.phi[sd][c - 1]; phD[1] = L.phi[sd][c]; phD[2] = L.phi[sd][c + 1];
        psD[0] = L.psi.get(sd, c - 1); psD[1] = L.psi.get(sd, c); psD[2] = L.psi.get(sd, c + 1);
      } else {
        ghost_row(phC, psC, phD, psD);
      }
      W phi9[9], psi9[9];
      nine(phD, phC, phU, phi9);
      nine(psD, psC, psU, psi9);
      if constexpr (LocalF<S>::value)
        add_f_refs(L.jref, slot(y - 1), sc, slot(y + 1), c, y, ny, k, f);

      const HGLds<R, typename ParkOf<S, R>::type, TW> hg{L.pull[(y - y0 + 2) & 1], lane};
      update_node<S, R, T0, STD>(D, jprev, h0x, h0dst, kp, kpw, x, y, k, phi9, psi9, f, p, n, g0,
                                 hg);
    }
  }
}

// Workgroups are dispatched round-robin over the 8 XCDs; the remap gives each
// XCD a contiguous run of tiles (`xcd_chunk` = tiles / 8, 0: no remap).
__device__ inline int xcd_tile(int xcd_chunk) {
  const int t = blockIdx.x;
  return xcd_chunk > 0 ? (t & 7) * xcd_chunk + (t >> 3) : t;
}

// One member of a batch of simulations swept by a single launch: its
// parameters, its two population buffers, (phi u)(t-1) and the two time
// levels of the rest population of h.  `cur` is the buffer holding its
// current state.
template <class S, class R, class T0>
struct SimDesc {
  KP<R> kp;
  KP<typename WorkOf<S>::type> kpw;  // the same constants in the working type
  S* pop[2];
  R* jprev;
  T0* h0[2];
  int cur;
};

// A tile of a batched sweep: simulation index (-1: padding), first column,
// first row and end row.
struct BatchTile {
  int sim, x0, y0, yend;
};

// The fused sweep: one workgroup per tile of the list, each running the tile
// code on its own simulation.  A single simulation is a list of one member;
// a batch of simulations of any sizes is swept by one launch.  Tiles of a
// member go band by band across all its strips, and the remap gives each XCD
// a contiguous run of them, so that the workgroups running together on an
// XCD hold neighbouring strips of the same rows and the cache lines they
// share are fetched from HBM once.  `flip` = 1 swaps every member's buffers
// (odd steps of a captured block).  EXT selects the form: 0 plain, 1 with
// the side walls, 2 with the side walls and the local field of Eq. (50), 3
// plain with the ions on D2Q9; STD compiles in the default MRT rates (see
// STD_MASK_F), which saves ~8 % of the vector instructions.  A launch covers
// members of one form.  The per-lane address and reference
// selects of the side walls cost 2-6 % on MI355X at 2048^2, and the local
// field's code another ~13 % (more spills) where it is compiled in.
//
// At least four waves per SIMD are asked of the register allocator (two with
// FP64 arithmetic): with the FP64 working type of FP32 storage it otherwise
// settles on 144 VGPRs (three waves); four waves with a few spilled
// registers are up to 18 % faster on MI355X at 2048^2.
template <class S, class R, class T0, int NW, int EXT, bool STD>
__global__ __launch_bounds__(64 * NW)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2))) void k_sweep_batch(
    const SimDesc<S, R, T0>* __restrict__ sims,
    const BatchTile* __restrict__ tiles, int xcd_chunk, int flip) {
  __shared__ SweepLds<S, R, 64 * NW> L;
  const BatchTile tl = tiles[xcd_tile(xcd_chunk)];
  if (tl.sim < 0) return;
  const SimDesc<S, R, T0>& sd = sims[tl.sim];
  const int a = (sd.cur + flip) & 1;
  const S* src = sd.pop[a];
  sweep_tile<S, R, T0, NW, EXT, STD>(L, src, sd.pop[1 - a], sd.jprev, sd.h0[a], sd.h0[1 - a],
                                     sd.kp, sd.kpw, tl.x0, tl.y0, tl.yend);
}

// ---------------------------------------------------------------------------
// Helpers outside the hot loop.
// ---------------------------------------------------------------------------

// phi', psi' and rho_e = e0 (P' - Q') of every node into compact planes.
template <class S, class R, class T0>
__global__ void k_moments(const S* __restrict__ src, const S* __restrict__ gsrc,
                          const T0* __restrict__ h0x, R* __restrict__ mom, const KP<R> kp) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= kp.nx) return;
  const PopView<S, R> Ph{make_rsrc(src, kp.pop_bytes), &kp};
  const PopView<S, R> Pg{make_rsrc(gsrc, kp.pop_bytes), &kp};
  const Cols k = cols_of(x, kp.nx, kp.side_walls);
  R h[9], g4[4], t4[4];
  pull_h(Ph, h0x, k, y, h);
  pull_g(Pg, k, y, g4);
  pull4(Ph, QP, k, y, t4);
  const R Pd = (R)ion_rest(Ph, h0x, QP, x, y) + t4[0] + t4[1] + t4[2] + t4[3] +
               ion_diag_sum(Ph, QP9, k, y);
  pull4(Ph, QN, k, y, t4);
  const R Qd = (R)ion_rest(Ph, h0x, QN, x, y) + t4[0] + t4[1] + t4[2] + t4[3] +
               ion_diag_sum(Ph, QN9, k, y);
  const long long c = (long long)y * kp.nx + x, np = (long long)kp.nx * kp.ny;
  mom[c] = sum9(h);
  mom[np + c] = psi_of(g4);
  mom[2 * np + c] = kp.q * (Pd - Qd);
}

// psi' of every node into its moment plane (the g-only sweeps of a
// pre-solve, where phi' and rho_e stay as k_moments left them): the same
// value k_moments writes there, from the g lines alone.
template <class S, class R>
__global__ void k_psi_plane(const S* __restrict__ gsrc, R* __restrict__ mom, const KP<R> kp) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= kp.nx) return;
  const PopView<S, R> Pg{make_rsrc(gsrc, kp.pop_bytes), &kp};
  const Cols k = cols_of(x, kp.nx, kp.side_walls);
  R g4[4];
  pull_g(Pg, k, y, g4);
  mom[(long long)kp.nx * kp.ny + (long long)y * kp.nx + x] = psi_of(g4);
}

// phi' / psi' neighbourhood of (x, y) from the compact moment planes.
template <class R>
__device__ inline void hood(const R* __restrict__ mom, const KP<R>& kp, int x, int y,
                            R phi9[9], R psi9[9]) {
  const long long np = (long long)kp.nx * kp.ny;
  const Cols k = cols_of(x, kp.nx, kp.side_walls);
  // beyond a side wall: the mirror image, the wall column itself
  const int cols[3] = {k.lw ? k.c : k.m, k.c, k.rw ? k.c : k.p};
  R ph[3][3], ps[3][3];  // [row: down, centre, up][col]
  const bool periodic = kp.walls == WALL_PERIODIC;
  for (int r = 0; r < 3; ++r) {
    int yy = y + r - 1;
    if (yy < 0 || yy >= kp.ny) {
      if (!periodic) continue;
      yy = (yy + kp.ny) % kp.ny;
    }
    for (int j = 0; j < 3; ++j) {
      ph[r][j] = mom[(long long)yy * kp.nx + cols[j]];
      ps[r][j] = mom[np + (long long)yy * kp.nx + cols[j]];
    }
  }
  if (!periodic) {
    if (y == 0) ghost_row(ph[1], ps[1], ph[0], ps[0]);
    if (y == kp.ny - 1) ghost_row(ph[1], ps[1], ph[2], ps[2]);
  }
  nine(ph[0], ph[1], ph[2], phi9);
  nine(ps[0], ps[1], ps[2], psi9);
}

// Macroscopic fields (FP64 output, [10][ny][nx]), absolute values.
template <class S, class R, class T0>
__global__ void k_fields(const S* __restrict__ src, const T0* __restrict__ h0x,
                         const R* __restrict__ mom, double* __restrict__ out, const KP<R> kp) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= kp.nx) return;
  const PopView<S, R> Ph{make_rsrc(src, kp.pop_bytes), &kp};
  const Cols k = cols_of(x, kp.nx, kp.side_walls);
  R phi9[9], psi9[9], f[9], t4[4];
  hood(mom, kp, x, y, phi9, psi9);
  pull_f(Ph, k, y, f);
  pull4(Ph, QP, k, y, t4);
  const R Pd = (R)ion_rest(Ph, h0x, QP, x, y) + t4[0] + t4[1] + t4[2] + t4[3] +
               ion_diag_sum(Ph, QP9, k, y);
  pull4(Ph, QN, k, y, t4);
  const R Qd = (R)ion_rest(Ph, h0x, QN, x, y) + t4[0] + t4[1] + t4[2] + t4[3] +
               ion_diag_sum(Ph, QN9, k, y);
  R Eg[2];
  const R* Eloc = nullptr;
  if (kp.local_field) {
    R g4[4];
    pull_g(Ph, k, y, g4);
    field_from_g(g4, kp, Eg);
    Eloc = Eg;
  }
  Macro<R> m;
  macro(phi9, psi9, Pd, Qd, f, kp, m, Eloc);
  const long long c = (long long)y * kp.nx + x, np = (long long)kp.nx * kp.ny;
  const double psi_lin =
      kp.walls == WALL_PERIODIC ? 0.0 : (double)kp.dpsi * (kp.ny - 0.5 - y) / kp.ny;
  out[0 * np + c] = 0.5 + (double)m.phid;
  out[1 * np + c] = psi_lin + (double)m.psid;
  out[2 * np + c] = (double)kp.c0 + (double)m.cpd;
  out[3 * np + c] = (double)kp.c0 + (double)m.cmd;
  out[4 * np + c] = m.rhoe;
  out[5 * np + c] = m.u[0];
  out[6 * np + c] = m.u[1];
  out[7 * np + c] = m.p;
  out[8 * np + c] = m.E[0];
  out[9 * np + c] = m.E[1];
}

// One g-only sweep (phi and rho_e held fixed): reads the g set of buffer
// gsrc, writes that of buffer gdst (the other lines of gdst are untouched).
template <class S, class R>
__global__ void k_poisson(const S* __restrict__ gsrc, S* __restrict__ gdst,
                          const R* __restrict__ mom, const KP<R> kp) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= kp.nx) return;
  const PopView<S, R> Pg{make_rsrc(gsrc, kp.pop_bytes), &kp};
  const PopView<S, R> DG{make_rsrc(gdst, kp.pop_bytes), &kp};
  const Cols k = cols_of(x, kp.nx, kp.side_walls);
  R phi9[9], psi9[9], g4[4];
  hood(mom, kp, x, y, phi9, psi9);
  const long long np = (long long)kp.nx * kp.ny;
  const long long c = (long long)y * kp.nx + x;
  pull_g(Pg, k, y, g4);
  R g[5] = {g_rest(Pg, x, y), g4[0], g4[1], g4[2], g4[3]};
  const R eps = (R(0.5) + phi9[0]) * kp.deps + kp.eps_v;
  R gphi[2], gpsi[2];
  grad_lap<R>(phi9, gphi, nullptr);
  if (kp.local_field) {
    R E[2];
    field_from_g(g4, kp, E);
    gpsi[0] = -E[0];
    gpsi[1] = -E[1];
  } else {
    grad_lap<R>(psi9, gpsi, nullptr);
    gpsi[1] += kp.psi_slope;
  }
  const R geps[2] = {kp.deps * gphi[0], kp.deps * gphi[1]};
  collide_g(g, psi9[0], poisson_source<R>(mom[2 * np + c], recip(eps), geps, gpsi, kp), kp);
  store_g(DG, kp, x, y, k, g, psi9);
}

// SplitMix64 (Steele, Lea, Flood 2014): output number n (n >= 1) of the
// generator started at `seed`.
__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t n) {
  uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ inline double unit_noise(uint64_t seed, uint64_t n) {
  return 2.0 * ((double)(splitmix64(seed, n) >> 11) * 0x1.0p-53) - 1.0;
}

struct InitSpec {
  // droplet
  double xc, yc, radius, noise;
  uint64_t seed;
  // or host-provided fields (device copies, [ny][nx]); ux/uy may be null
  const double *phi, *cp, *cm, *psi, *ux, *uy;
  // absolute parameters (FP64)
  double W, c0, dpsi, rho_v, drho, a_g;
};

// Equilibrium initial state.  The population arriving at node (x, y) along
// c_i at the first step is the equilibrium there, so it is written where
// that node pulls it from: row y - c_iy, column x - c_ix, as a deviation from
// the reference of that row.  AA: in-place streaming, whose first step reads
// the arrivals from the node's own slots; they are written there (still as
// deviations from the reference of the row they come from).
template <class S, class R, class T0, bool AA = false>
__global__ void k_init(S* __restrict__ dst, R* __restrict__ jprev, T0* __restrict__ h0x,
                       const KP<R> kp, const InitSpec sp) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= kp.nx) return;
  const long long c = (long long)y * kp.nx + x;
  double phi, cp, cm, psi, ux = 0.0, uy = 0.0;
  if (sp.phi) {
    phi = sp.phi[c];
    cp = sp.cp[c];
    cm = sp.cm[c];
    psi = sp.psi[c];
    if (sp.ux) ux = sp.ux[c];
    if (sp.uy) uy = sp.uy[c];
  } else {
    const double dx = x - sp.xc, dy = y - sp.yc;
    const double r = sqrt(dx * dx + dy * dy);
    phi = 0.5 * (1.0 + tanh(2.0 * (sp.radius - r) / sp.W));
    cp = sp.c0 * (1.0 + sp.noise * unit_noise(sp.seed, 2 * (uint64_t)c + 1));
    cm = sp.c0 * (1.0 + sp.noise * unit_noise(sp.seed, 2 * (uint64_t)c + 2));
    psi = kp.walls == WALL_PERIODIC ? 0.0 : sp.dpsi * (kp.ny - 0.5 - y) / kp.ny;
  }
  const double rho = phi * sp.drho + sp.rho_v;
  const double uu = ux * ux + uy * uy;
  const int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const double w9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                        1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  const double w5[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
  const PopView<S, R> D{make_rsrc(dst, kp.pop_bytes), &kp};
  // Behind a side wall the pull reads the wall column instead (see the
  // pulls): f, the ions and g in the opposite direction at the node itself;
  // h in the x-mirrored direction one row up or down (at a corner, the
  // opposite direction at the node itself).
  const int opp9[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  const int mir9[9] = {0, 3, 2, 1, 4, 6, 5, 8, 7};
  const int opp5[5] = {0, 3, 4, 1, 2};
  auto put = [&](int q, int i, double v) {
    const int xs = x - cx[i], ys = y - cy[i];
    if constexpr (AA) {
      const double ref = plane_ref(q, ys, kp.ny, kp.walls, sp.c0, sp.dpsi, sp.a_g);
      D.put(q, D.row(y + 1) + x, (R)(v - ref));
      return;
    }
    int qt = q, xt = xs, yt = ys;
    if (kp.side_walls && (xs < 0 || xs >= kp.nx)) {
      const bool corner = kp.walls != WALL_PERIODIC && (ys < 0 || ys >= kp.ny);
      xt = x;
      if (q >= QH && q < QP && !corner) {
        qt = q - i + mir9[i];
      } else {  // (lines from QP9 on: the diagonals of D2Q9 ions, direction i - 5)
        qt = q - i + ((q < QP || q >= QP9) ? opp9[i] : opp5[i]);
        yt = y;
      }
    } else {
      xt = xs < 0 ? xs + kp.nx : (xs >= kp.nx ? xs - kp.nx : xs);
    }
    const double ref = plane_ref(qt, yt, kp.ny, kp.walls, sp.c0, sp.dpsi, sp.a_g, kp.ion_q9);
    D.put(qt, D.row(yt + 1) + xt, (R)(v - ref));
  };
  // h: the rest population (which does not move) takes phi minus what the
  // eight stored moving populations hold, so that phi is exact from the start
  RestAcc<T0> hrest = RestAcc<T0>::from_content(phi - 0.5);
  R tref = R(0);  // this node's reference phase (16-bit storage)
  if (LocalH<S>::value) {
    tref = D.stored(QH, (R)(phi - 0.5));
    D.put(QH, D.row(y + 1) + x, tref);
  }
  for (int i = 0; i < 9; ++i) {
    const double cu = cx[i] * ux + cy[i] * uy;
    // f: pressure-based equilibrium with p = 0
    put(QF + i, i, rho * w9[i] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    if (i > 0) {
      const double dev = w9[i] * phi * (1.0 + 3.0 * cu) - 0.5 * w9[i];
      const R st = D.stored(QH + i, (R)(dev - (double)W9F[i] * (double)tref));
      put(QH + i, i, (double)st + 0.5 * w9[i]);
      hrest.sub(h_from(st, i, tref));
    }
  }
  *elem(h0x, (uint32_t)y * kp.pitch + x) = hrest.rest();
  const uint32_t jo = (uint32_t)y * kp.pitch + x;
  // bfloat16 storage: every node's reference momentum starts at 0, so the
  // initial f above are stored relative to 0 as written
  if (LocalF<S>::value) {
    D.put(QJX, D.row(y + 1) + x, R(0));
    D.put(QJY, D.row(y + 1) + x, R(0));
  }
  // g: this node's reference potential psi'~ (16-bit storage; 0 otherwise)
  double tg = 0.0;
  if (LocalG<S>::value) {
    const double psi_lin =
        kp.walls == WALL_PERIODIC ? 0.0 : sp.dpsi * (kp.ny - 0.5 - y) / kp.ny;
    const R t = D.stored(QRG, (R)(psi - psi_lin));
    D.put(QRG, D.row(y + 1) + x, t);
    tg = (double)t;
  }
  if (kp.ion_q9) {  // the ions on D2Q9: nine populations each, weights of Eq. (25)
    for (int i = 0; i < 9; ++i) {
      const double cu = cx[i] * ux + cy[i] * uy;
      put(i < 5 ? QP + i : QP9 + i - 5, i, w9[i] * cp * (1.0 + 3.0 * cu));
      put(i < 5 ? QN + i : QN9 + i - 5, i, w9[i] * cm * (1.0 + 3.0 * cu));
    }
  }
  for (int i = 0; i < 5; ++i) {
    const double cu = cx[i] * ux + cy[i] * uy;
    if (kp.ion_q9) {
      // (ions written above)
    } else if (i == 0 && IonRest<S>::value) {
      if constexpr (IonRest<S>::value) {
        *elem(h0x, kp.cells + jo) = (T0)(w5[0] * (cp - sp.c0));
        *elem(h0x, 2 * kp.cells + jo) = (T0)(w5[0] * (cm - sp.c0));
      }
    } else {
      put(QP + i, i, w5[i] * cp * (1.0 + 3.0 * cu));
      put(QN + i, i, w5[i] * cm * (1.0 + 3.0 * cu));
    }
    put(QG + i, i, i == 0 ? -2.0 / 3.0 * (psi - tg) : (psi - tg) / 6.0);
  }
  *elem(jprev, jo) = (R)(phi * ux);
  *elem(jprev, kp.cells + jo) = (R)(phi * uy);
}

// Sum over the 64 lanes of a wave by a butterfly of lane exchanges, the same
// fixed order in every call (every lane ends with the sum).
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}
// The N sums over a 256-thread workgroup of acc[0..N-1]: each wave's by
// wave_sum, then the four waves' partials (sh: N x 4 doubles of LDS) in a
// fixed order.  Thread j < N returns sum j.
template <int N>
__device__ inline double block_sums(double (*sh)[4], const double acc[N], int t) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const double v = wave_sum(acc[j]);
    if ((t & 63) == 0) sh[j][t >> 6] = v;
  }
  __syncthreads();
  return t < N ? (sh[t][0] + sh[t][1]) + (sh[t][2] + sh[t][3]) : 0.0;
}

// FP64 sums of one row: [phi, rho_e, sum p, sum n, phi x, phi y, nonfinite].
// One 256-thread workgroup per row; wavefront reductions of fixed shape: the
// result depends on nx and ny only.
constexpr int NSUM = 7;
template <class S, class R, class T0>
__global__ __launch_bounds__(256) void k_row_sums(const S* __restrict__ src,
                                                  const T0* __restrict__ h0x,
                                                  double* __restrict__ part, const KP<R> kp) {
  __shared__ double sh[NSUM][4];
  const int y = blockIdx.x, t = threadIdx.x;
  const PopView<S, R> Ph{make_rsrc(src, kp.pop_bytes), &kp};
  double acc[NSUM] = {0, 0, 0, 0, 0, 0, 0};
  const double c0 = (double)kp.c0;
  for (int x = t; x < kp.nx; x += 256) {
    const Cols k = cols_of(x, kp.nx, kp.side_walls);
    R h[9], t4[4], g4[4];
    pull_h(Ph, h0x, k, y, h);
    // the node's phi content in the bookkeeping of the rest type (exact
    // integer sums with the fixed-point rest of FP32 storage)
    RestAcc<T0> content = RestAcc<T0>::from_rest(*elem(h0x, (uint32_t)y * kp.pitch + x));
    for (int i = 1; i < 9; ++i) content.add(h[i]);
    pull4(Ph, QP, k, y, t4);
    const double Pd = ion_rest(Ph, h0x, QP, x, y) + t4[0] + t4[1] + t4[2] + t4[3] +
                      (double)ion_diag_sum(Ph, QP9, k, y);
    pull4(Ph, QN, k, y, t4);
    const double Qd = ion_rest(Ph, h0x, QN, x, y) + t4[0] + t4[1] + t4[2] + t4[3] +
                      (double)ion_diag_sum(Ph, QN9, k, y);
    pull_g(Ph, k, y, g4);
    double phid = content.content();
    // a non-finite population has no fixed-point image
    for (int i = 1; i < 9; ++i)
      if (!isfinite((double)h[i])) phid = (double)h[i];
    const double phi = 0.5 + phid;
    const double psid = (double)psi_of(g4);
    acc[0] += phi;
    acc[1] += (double)kp.q * (Pd - Qd);
    acc[2] += c0 + Pd;
    acc[3] += c0 + Qd;
    acc[4] += phi * x;
    acc[5] += phi * y;
    if (!(isfinite(phid) && isfinite(Pd) && isfinite(Qd) && isfinite(psid))) acc[6] += 1.0;
  }
  const double r = block_sums<NSUM>(sh, acc, t);
  if (t < NSUM) part[(long long)y * NSUM + t] = r;
}

// Column sums of the per-row partial sums [ny][ncol]: one 256-thread
// workgroup per column, thread t summing rows t, t + 256, ... in order, then
// the reductions of block_sums (a fixed shape: the result depends on ny only).
// One thread walking all rows took 270 us at ny = 2048, more than a sweep.
__global__ __launch_bounds__(256) void k_sum_rows(const double* __restrict__ part, int ny,
                                                  int ncol, double* __restrict__ out) {
  __shared__ double sh[1][4];
  const int j = blockIdx.x, t = threadIdx.x;
  double a[1] = {0.0};
  for (int y = t; y < ny; y += 256) a[0] += part[(long long)y * ncol + j];
  const double r = block_sums<1>(sh, a, t);
  if (t == 0) out[j] = r;
}

// FP64 sums of one row for the convergence residual of the g-only sweeps:
// [sum (psi_new - psi_old)^2, sum psi_new^2], psi from the g sets of two
// buffers (the latest sweep and the one before).  Same fixed-shape
// reductions as k_row_sums.
template <class S, class R>
__global__ __launch_bounds__(256) void k_psi_change_rows(const S* __restrict__ gnew,
                                                         const S* __restrict__ gold,
                                                         double* __restrict__ part,
                                                         const KP<R> kp) {
  __shared__ double sh[2][4];
  const int y = blockIdx.x, t = threadIdx.x;
  const PopView<S, R> Pn{make_rsrc(gnew, kp.pop_bytes), &kp};
  const PopView<S, R> Po{make_rsrc(gold, kp.pop_bytes), &kp};
  const double psi_lin =
      kp.walls == WALL_PERIODIC ? 0.0 : (double)kp.dpsi * (kp.ny - 0.5 - y) / kp.ny;
  double dd = 0.0, nn = 0.0;
  for (int x = t; x < kp.nx; x += 256) {
    const Cols k = cols_of(x, kp.nx, kp.side_walls);
    R gn[4], go[4];
    pull_g(Pn, k, y, gn);
    pull_g(Po, k, y, go);
    const double pn = psi_lin + (double)psi_of(gn), po = psi_lin + (double)psi_of(go);
    dd += (pn - po) * (pn - po);
    nn += pn * pn;
  }
  const double acc[2] = {dd, nn};
  const double r = block_sums<2>(sh, acc, t);
  if (t < 2) part[(long long)y * 2 + t] = r;
}

// Plain copy through buffer descriptors (measurement helper).  Each lane
// moves W bytes per iteration; the grid strides over the buffer.
template <int W>
__global__ __launch_bounds__(256) void k_copy(const void* __restrict__ src,
                                              void* __restrict__ dst, uint32_t bytes) {
  const Rsrc rs = make_rsrc(src, bytes), rd = make_rsrc(dst, bytes);
  const uint32_t stride = gridDim.x * blockDim.x * W;
  for (uint32_t o = (blockIdx.x * blockDim.x + threadIdx.x) * W; o < bytes; o += stride) {
    if (W == 4) {
      const unsigned int v = __builtin_amdgcn_raw_buffer_load_b32(rs, o, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b32(v, rd, o, 0, 0);
    } else {
      typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
      const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b128(v, rd, o, 0, 0);
    }
  }
}

}  // namespace lbm
