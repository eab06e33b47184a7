// lbm_ehd_aa.hpp -- the fused sweep with in-place streaming (the AA pattern):
// one population buffer per simulation instead of two.
//
// The buffer keeps the layout of the two-buffer sweep (rows of 33 lines of
// `pitch` elements, ghost rows unused), but the populations of a node sit in
// one of two orientations, alternating step by step:
//   even steps: the population arriving at node x along c_i is at x, line i;
//               the node writes its post-collision population i to x, line
//               opp(i) (its own slots, reversed);
//   odd steps:  the population arriving at x along c_i is at x - c_i, line
//               opp(i) (where its sender left it); the node writes its
//               post-collision population i to x + c_i, line i.
// In both, every location is read and written by exactly one node, so a
// sweep needs no second buffer and no ordering between workgroups.  At an
// electrode the population a node sends through the wall comes back to it
// along the opposite direction: the node writes the wall rule's value (in
// deviation form, as in the two-buffer sweep) to its own line opp(i), which
// at the next step is where it finds that arrival (in the even orientation
// by definition, in the odd one because the wall is the sender).  The rest
// populations stay in place.  The g set has its own orientation (`gpar`),
// so that g-only sweeps (pre-solves, extra Poisson sweeps) work in place too.
//
// The isotropic stencils need phi' and psi' of the eight neighbours at the
// current step, i.e. moments of their arrivals.  The sweep forms them for its
// own rows in an LDS ring one row ahead, as the two-buffer sweep does; but in
// place a neighbouring workgroup may already have overwritten the arrivals of
// the nodes beyond the tile.  A pre-pass (k_aa_hood) therefore writes phi'
// and psi' of every tile's edge nodes (first and last row of each band, first
// and last column of each strip) to two planes first, with the same
// arithmetic, and the sweep takes its halo from them.  The planes are in the
// working type (FP64 with FP32 storage): 16 B per cell of memory; the
// pre-pass reads the h and g arrivals of about 2 / band height of the nodes.
//
// This form covers the plain sweep (no side walls, no local field of Eq. 50)
// with FP64, FP32 and binary16 storage.  With binary16 the node-local
// references stay where the two-buffer layout keeps them: each node's phi'~
// in its own slot of line QH and its psi'~ in its own slot of line QRG (the
// rest populations of h, p and n live in their planes, so those slots are
// free in both orientations), and every population is stored relative to the
// reference of the node it arrives at, which in either orientation is the
// node that reads it.
#pragma once

#include "lbm_ehd_kernels.hpp"

namespace lbm {

// Velocity components and opposite direction of D2Q9 direction i (the D2Q5
// directions 0-4 are the same), as constant expressions.
__host__ __device__ constexpr int cx_of(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int cy_of(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp_of(int i) {
  return i == 0 ? 0 : (i <= 4 ? (i + 1) % 4 + 1 : (i - 3) % 4 + 5);
}

// Stores of the odd steps, which scatter to the neighbours' slots, with 4-
// and 2-byte storage: the non-temporal hint without device scope (SC1),
// where the codec's stores (even steps, a node's own slots, the two-buffer
// sweep, and 8-byte storage) carry both.  Measured on MI355X at 2048^2, a
// step in place: +4.1 % FP32, +3.2 % binary16, +0.5 % FP32 storage with FP64
// arithmetic, -1.1 % FP64 (so FP64 keeps the codec's); the same hint on even
// steps cost 7 %.  The same conversions as the codec's stores.
constexpr int ST_AA_ODD = 2;  // NT
template <class S, class R>
struct OddStore;
template <>
struct OddStore<float, float> {
  __device__ static inline void st(Rsrc r, uint32_t v, uint32_t s, float x) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, v, s,
                                          ST_AA_ODD);
  }
};
template <>
struct OddStore<float, double> {
  __device__ static inline void st(Rsrc r, uint32_t v, uint32_t s, double x) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, (float)x), r, v, s,
                                          ST_AA_ODD);
  }
};
template <>
struct OddStore<__half, float> {
  __device__ static inline void st(Rsrc r, uint32_t v, uint32_t s, float x) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, __float2half_rn(x)),
                                          r, v, s, ST_AA_ODD);
  }
};

// A population buffer in the AA orientations.  The choices between a node's
// own slot and a neighbour's (the orientation, an electrode in the way) are
// selects of the line and the offset, not branches: the row and the
// orientation are uniform, and straight-line code keeps a row's loads in
// flight together (the branched form issued them one group at a time and ran
// the in-place sweep at 0.67x the two-buffer one).
template <class S, class R>
struct AAView {
  PopView<S, R> P;
  // the population of direction i of the set at line q0 that arrives at node
  // (k.c, y) at this step, in orientation `par`: in the even one the node's
  // own slot i; in the odd one the sender's slot opp(i) at x - c_i, or the
  // node's own slot i where the sender lies beyond an electrode (the wall
  // rule wrote the reflected value there)
  template <class K>
  __device__ inline R in(int par, int q0, int i, K k, int y) const {
    const uint32_t own = P.row(y + 1) + k.c;
    const int ny = P.kp->ny;
    const int y1 = y - cy_of(i);
    const bool beyond = y1 < 0 || y1 >= ny;
    const int ys = y1 < 0 ? y1 + ny : (y1 >= ny ? y1 - ny : y1);
    const bool self = par == 0 || i == 0 || (beyond && P.kp->walls != WALL_PERIODIC);
    const int xs = cx_of(i) > 0 ? k.m : (cx_of(i) < 0 ? k.p : k.c);
    return load_as(self ? q0 + i : q0 + opp_of(i), q0 + i, self ? own : P.row(ys + 1) + xs);
  }
  // The same for lanes that may sit in different rows: the line goes into the
  // lane's own offset instead of the wave's scalar one.
  template <class K>
  __device__ inline R in_lane(int par, int q0, int i, K k, int y) const {
    const uint32_t own = P.row(y + 1) + k.c;
    const int ny = P.kp->ny;
    const int y1 = y - cy_of(i);
    const bool beyond = y1 < 0 || y1 >= ny;
    const int ys = y1 < 0 ? y1 + ny : (y1 >= ny ? y1 - ny : y1);
    const bool self = par == 0 || i == 0 || (beyond && P.kp->walls != WALL_PERIODIC);
    const int xs = cx_of(i) > 0 ? k.m : (cx_of(i) < 0 ? k.p : k.c);
    const uint32_t q = self ? q0 + i : q0 + opp_of(i);
    const uint32_t off = (self ? own : P.row(ys + 1) + xs) + q * (uint32_t)P.kp->pitch;
    const int c = q0 + i;
    R v = Codec<S, R>::ld(P.rs, off * (uint32_t)sizeof(S), 0u, P.nt);
    if constexpr (Scaled<S>::value) return v * P.kp->isc[line_set<S>(c)] + P.ofs(c);
    if (P.has_ofs(c)) v += P.kp->iofs[c - QP];
    return v;
  }
  // store the post-collision population v of direction i of the set at line
  // q0 of node (k.c, y), in orientation `par`; `vwall`: the value that comes
  // back along opp(i) when c_i points through an electrode
  template <class K>
  __device__ inline void out(int par, int q0, int i, K k, int y, R v, R vwall) const {
    const uint32_t own = P.row(y + 1) + k.c;
    const int ny = P.kp->ny;
    const int y1 = y + cy_of(i);
    const bool through = (y1 < 0 || y1 >= ny) && P.kp->walls != WALL_PERIODIC;
    const int yd = y1 < 0 ? y1 + ny : (y1 >= ny ? y1 - ny : y1);
    const bool self = par == 0 || i == 0 || through;
    const int xd = cx_of(i) > 0 ? k.p : (cx_of(i) < 0 ? k.m : k.c);
    const int qi = q0 + i, qo = q0 + opp_of(i);
    R x = through ? vwall : v;
    // the reflected value travels along opp(i), the others along i (a line
    // pair of one set: both or neither carry an offset)
    if (P.has_ofs(qi)) x -= through ? P.kp->iofs[qo - QP] : P.kp->iofs[qi - QP];
    if (Scaled<S>::value) x *= P.kp->sc[line_set<S>(qi)];
    const uint32_t vo = (self ? own : P.row(yd + 1) + xd) * (uint32_t)sizeof(S);
    if constexpr (sizeof(S) == 8) {
      Codec<S, R>::st(P.rs, vo, line_bytes(self ? qo : qi), x);
    } else {
      if (par == 0)
        Codec<S, R>::st(P.rs, vo, line_bytes(self ? qo : qi), x);
      else
        OddStore<S, R>::st(P.rs, vo, line_bytes(self ? qo : qi), x);
    }
  }
  // In place a population spends every other step in the slot of the
  // opposite direction, but it keeps the encoding of its own: the per-line
  // offset of the 16-bit ion lines (the drifting bulk, which differs between
  // +y and -y) is that of its direction, so that it rounds as with two
  // buffers and the FP64 rest populations book exactly what is stored.  The
  // same as PopView::at where q == c.
  __device__ inline R load_as(int q, int c, uint32_t off) const {
    R v = Codec<S, R>::ld(P.rs, off * (uint32_t)sizeof(S), line_bytes(q), P.nt);
    if constexpr (Scaled<S>::value) return v * P.kp->isc[line_set<S>(c)] + P.ofs(c);
    if (P.has_ofs(c)) v += P.kp->iofs[c - QP];
    return v;
  }
  // Byte offset of line q, the scalar operand of the buffer access.  The
  // line depends on the orientation, the direction and the row only, which
  // every lane of a wave shares wherever in() and out() are called (one
  // lattice row per wave; the pre-pass, whose lanes sit in different rows,
  // loads through in_lane); without the broadcast the compiler, which sees
  // the line selected inside branches on the lane, wraps each access in a
  // loop over the distinct values.
  __device__ inline uint32_t line_bytes(int q) const {
    return (uint32_t)__builtin_amdgcn_readfirstlane(
        (int)((uint32_t)q * P.kp->pitch * (uint32_t)sizeof(S)));
  }
};

// The arrivals of node (k.c, y) with the node-local references of binary16
// storage added back (h: w_i phi'~, g: psi'~ / 6 of the node itself; see the
// header); a no-op for the other storage types.
template <class S, class R, class K>
__device__ inline void aa_refs_h(const AAView<S, R>& V, K k, int y, R h[9]) {
  if constexpr (LocalH<S>::value) {
    const R t = V.P.at(QH, V.P.row(y + 1) + k.c);
#pragma unroll
    for (int i = 1; i < 9; ++i) h[i] = h_from(h[i], i, t);
  }
}
template <class S, class R, class K>
__device__ inline void aa_refs_g(const AAView<S, R>& V, K k, int y, R g4[4]) {
  if constexpr (LocalG<S>::value) {
    const R t = V.P.at(QRG, V.P.row(y + 1) + k.c) * R(1.0 / 6.0);
#pragma unroll
    for (int i = 0; i < 4; ++i) g4[i] += t;
  }
}
// g0 of node (k.c, y) in orientation gpar, as a deviation (g_rest)
template <class S, class R, class K>
__device__ inline R aa_g0(const AAView<S, R>& V, int gpar, K k, int y) {
  R g0 = V.in(gpar, QG, 0, k, y);
  if constexpr (LocalG<S>::value) g0 -= R(2.0 / 3.0) * V.P.at(QRG, V.P.row(y + 1) + k.c);
  return g0;
}
// The ion content of node (x, y) in orientation par, summed in type A: its
// rest population (the FP64 plane with binary16 storage) plus its four
// arrivals, in the order of the two-buffer helpers.
template <class A, class S, class R, class T0, class K>
__device__ inline A aa_ion(const AAView<S, R>& V, const T0* __restrict__ h0x, int par, int q0,
                           K k, int x, int y) {
  A c;
  if constexpr (IonRest<S>::value)
    c = (A)rest_val(*elem(h0x, (uint32_t)(q0 == QP ? 1 : 2) * V.P.kp->cells +
                                  (uint32_t)y * V.P.kp->pitch + x));
  else
    c = (A)V.in(par, q0, 0, k, y);
#pragma unroll
  for (int i = 1; i < 5; ++i) c += (A)V.in(par, q0, i, k, y);
  return c;
}

// One member of an in-place sweep: its parameters, its population buffer,
// (phi u)(t-1), the rest population of h (one time level, in place), the
// phi' and psi' planes of the pre-pass (in the working type, as the stencil
// ring of the two-buffer sweep) and the two orientations.
template <class S, class R, class T0>
struct SimDescAA {
  KP<R> kp;
  KP<typename WorkOf<S>::type> kpw;
  S* pop;
  R* jprev;
  T0* h0;
  typename WorkOf<S>::type* phiP;
  typename WorkOf<S>::type* psiP;
  int par, gpar;
};

// The pre-pass: phi' and psi' at this step of the nodes that a neighbouring
// tile's stencils reach, i.e. the first and last row of every band and the
// first and last column of every strip (the sweep forms the others itself in
// its LDS ring, one row ahead), with the sums of the two-buffer sweep's
// ring.  In place, a neighbouring workgroup may overwrite such a node's
// arrivals before the stencil needs them.
template <class S, class R, class T0, int NW>
__global__ __launch_bounds__(64 * NW) void k_aa_hood(const SimDescAA<S, R, T0>* __restrict__ sims,
                                                     const BatchTile* __restrict__ tiles,
                                                     int xcd_chunk, int flip, int gflip) {
  typedef typename WorkOf<S>::type W;
  const BatchTile tl = tiles[xcd_tile(xcd_chunk)];
  if (tl.sim < 0) return;
  const SimDescAA<S, R, T0>& sd = sims[tl.sim];
  const KP<R>& kp = sd.kp;
  const int w = min(64 * NW, kp.nx - tl.x0), hb = tl.yend - tl.y0;
  // The tile's edge nodes, each once (also in one-row bands and one-column
  // strips): its first and last row, then the first and last column of the
  // rows between.  A thread takes every (64 NW)-th of them, so that all of
  // them are loaded in a few rounds (a walk down the band, in which only the
  // edge columns' lanes work on the inner rows, made as many dependent
  // rounds as the band has rows).
  const int nrow = hb > 1 ? 2 : 1, ncol = w > 1 ? 2 : 1, inner = max(hb - 2, 0);
  const int count = nrow * w + ncol * inner;
  const int par = (sd.par + flip) & 1, gpar = (sd.gpar + gflip) & 1;
  // cached loads, but for FP32 storage and arithmetic (measured on MI355X at
  // 2048^2, a step in place with non-temporal pre-pass loads: FP32 +1.6 %,
  // FP32 storage with FP64 arithmetic -2.4 %, binary16 and FP64 within noise)
  constexpr bool kLoadNT = sizeof(S) == 4 && sizeof(R) == 4;
  const AAView<S, R> V{PopView<S, R>{make_rsrc(sd.pop, kp.pop_bytes), &kp, kLoadNT}};
  for (int j = (int)threadIdx.x; j < count; j += 64 * NW) {
    int x, y;
    if (j < nrow * w) {
      x = tl.x0 + (j < w ? j : j - w);
      y = j < w ? tl.y0 : tl.yend - 1;
    } else {
      const int r = j - nrow * w;
      x = r < inner ? tl.x0 : tl.x0 + w - 1;
      y = tl.y0 + 1 + (r < inner ? r : r - inner);
    }
    const ColsP k = cols_for<0>(x, kp.nx, 0);
    const uint32_t jo = (uint32_t)y * kp.pitch + x;
    R h[9], g4[4];
#pragma unroll
    for (int i = 1; i < 9; ++i) h[i] = V.in_lane(par, QH, i, k, y);
#pragma unroll
    for (int i = 0; i < 4; ++i) g4[i] = V.in_lane(gpar, QG, i + 1, k, y);
    aa_refs_h(V, k, y, h);
    aa_refs_g(V, k, y, g4);
    *elem(sd.phiP, jo) = phi_of<W>((W)rest_val(*elem(sd.h0, jo)), h);
    *elem(sd.psiP, jo) = psi_as<W>(g4);
  }
}

// Per-node update of the in-place sweep: the arithmetic of update_node (the
// two-buffer sweep, plain form) in the same order, with the stores of the AA
// orientations.
template <class S, class R, class T0, bool STD, class HG, class K>
__device__ inline void update_node_aa(const AAView<S, R>& V, int par, int gpar,
                                      R* __restrict__ jprev, T0* __restrict__ h0x,
                                      const KP<R>& kp, const KP<typename WorkOf<S>::type>& kpw,
                                      int x, int y, K k, const typename WorkOf<S>::type phi9[9],
                                      const typename WorkOf<S>::type psi9[9], R f[9], R p[5],
                                      R n[5], R g0, const HG& hg) {
  typedef typename WorkOf<S>::type W;
  W fw[9], pw[5], nw[5], ps9[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    fw[i] = (W)f[i];
    ps9[i] = (W)psi9[i];
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    pw[i] = (W)p[i];
    nw[i] = (W)n[i];
  }
  const uint32_t jo = (uint32_t)y * kp.pitch + x;
  const uint32_t own = V.P.row(y + 1) + x;
  // exact incoming ion content of the node (FP64 ion rest populations)
  double Pin = 0.0, Qin = 0.0;
  if constexpr (IonRest<S>::value) {
    Pin = rest_val(*elem(h0x, kp.cells + jo));
    Qin = rest_val(*elem(h0x, 2 * kp.cells + jo));
    pw[0] = (W)Pin;
    nw[0] = (W)Qin;
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      Pin += (double)p[i];
      Qin += (double)n[i];
    }
  }
  const W Pd = pw[0] + pw[1] + pw[2] + pw[3] + pw[4];
  const W Qd = nw[0] + nw[1] + nw[2] + nw[3] + nw[4];
  Macro<W> m;
  macro(phi9, ps9, Pd, Qd, fw, kpw, m);
  const bool ins = kp.walls == WALL_INSULATING;
  const R third = R(1) / R(3);

  // f: bounce-back at the electrodes
  collide_f<STD>(fw, m, kpw);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    f[i] = (R)fw[i];
    V.out(par, QF, i, k, y, f[i], f[i]);
  }

  {  // g: Eq. (44)-(47); anti-bounce-back with the electrode potential
    R g[5];
    g[0] = g0;
    hg.g4(g + 1);
    W gw[5] = {(W)g[0], (W)g[1], (W)g[2], (W)g[3], (W)g[4]};
    collide_g<STD>(gw, m.psid, poisson_source<W>(m.rhoe, m.ieps, m.geps, m.gpsi, kpw), kpw);
    if constexpr (LocalG<S>::value) {
      // relative to psi'~ / 6 of the node each population arrives at (the
      // node itself for one reflected at an electrode), g0 relative to
      // -2/3 psi'~ of its own node (store_g of the two-buffer sweep)
      R t[5];
#pragma unroll
      for (int i = 0; i < 5; ++i) t[i] = V.P.stored(QRG, (R)psi9[i]);
      if (kp.walls != WALL_PERIODIC) {
        if (y == 0) t[4] = t[0];
        if (y == kp.ny - 1) t[2] = t[0];
      }
      V.P.put(QRG, own, t[0]);
      const R sixth = R(1.0 / 6.0);
      g[0] = (R)gw[0];
      V.out(gpar, QG, 0, k, y, g[0] + R(2.0 / 3.0) * t[0], g[0]);
#pragma unroll
      for (int i = 1; i < 5; ++i) {
        g[i] = (R)gw[i];
        V.out(gpar, QG, i, k, y, g[i] - t[i] * sixth, -g[i] - t[0] * sixth);
      }
    } else {
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        g[i] = (R)gw[i];
        V.out(gpar, QG, i, k, y, g[i], -g[i]);
      }
    }
  }

  collide_ion<STD>(pw, m.cpd, m.mup, m.itau_p, kpw.mask_p, W(-1), m, kpw);
  collide_ion<STD>(nw, m.cmd, m.mum, m.itau_n, kpw.mask_n, W(1), m, kpw);
  const R cpd = (R)m.cpd, cmd = (R)m.cmd;
  // the rest populations of binary16 storage live in their FP64 planes
  constexpr int I0 = IonRest<S>::value ? 1 : 0;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    p[i] = (R)pw[i];
    n[i] = (R)nw[i];
  }
  // the collision adds the reaction term to each ion's content (Eq. 41); with
  // FP64 rest populations those take what the stored moving ones leave of it
  double Pout = Pin + (double)m.Rr, Qout = Qin + (double)m.Rr;
#pragma unroll
  for (int i = I0; i < 5; ++i) {
    // anode (through it: direction 4): c+ = 0; cathode (direction 2): d c+/dn = 0
    const R wp = ins ? p[i] : (i == 4 ? -p[4] - third * kp.c0 : -p[i] + third * cpd);
    V.out(par, QP, i, k, y, p[i], wp);
    if constexpr (IonRest<S>::value) Pout -= (double)V.P.stored(QP + i, p[i]);
  }
#pragma unroll
  for (int i = I0; i < 5; ++i) {
    // anode: d c-/dn = 0; cathode: c- = 0
    const R wn = ins ? n[i] : (i == 4 ? -n[4] + third * cmd : -n[i] - third * kp.c0);
    V.out(par, QN, i, k, y, n[i], wn);
    if constexpr (IonRest<S>::value) Qout -= (double)V.P.stored(QN + i, n[i]);
  }
  if constexpr (IonRest<S>::value) {
    *elem(h0x, kp.cells + jo) = (T0)Pout;
    *elem(h0x, 2 * kp.cells + jo) = (T0)Qout;
  }

  {  // h: Eq. (27)-(32), with d(phi u)/dt of Eq. (58), in W; bounce-back
    const uint32_t jpl = kp.cells;
    const R Jx = (R)(m.phi * m.u[0]), Jy = (R)(m.phi * m.u[1]);
    const W dJ[2] = {(W)Jx - (W)*elem(jprev, jo), (W)Jy - (W)*elem(jprev, jpl + jo)};
    *elem(jprev, jo) = Jx;
    *elem(jprev, jpl + jo) = Jy;
    const T0 h0in = *elem(h0x, jo);
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
    if constexpr (LocalH<S>::value) {
      // relative to w_i phi'~ of the node each population arrives at (the node
      // itself for one reflected at an electrode)
      R t[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) t[i] = V.P.stored(QH, (R)phi9[i]);
      if (kp.walls != WALL_PERIODIC) {
        if (y == 0) t[4] = t[7] = t[8] = t[0];
        if (y == kp.ny - 1) t[2] = t[5] = t[6] = t[0];
      }
      V.P.put(QH, own, t[0]);  // this node's reference for the next step
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        h[i] = V.P.stored(QH + i, (R)hw[i] - (R)W9F[i] * t[i]);
        V.out(par, QH, i, k, y, h[i], h[i]);
        mass.sub(h_from(h[i], i, t[i]));
      }
    } else {
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        h[i] = V.P.stored(QH + i, (R)hw[i]);
        V.out(par, QH, i, k, y, h[i], h[i]);
        mass.sub(h[i]);
      }
    }
    // the rest population takes what the eight stored ones leave of the content
    *elem(h0x, jo) = mass.rest();
  }
}

// The fused in-place sweep: one workgroup per tile of the list, walking its
// band row by row as the two-buffer sweep does.  phi' and psi' of the
// tile's own rows come from its LDS ring, formed one row ahead from the
// arrivals, whose h1-h8 and g1-g4 are parked in LDS for the row's update;
// those of the rows and columns beyond the tile (its neighbours' edge nodes,
// which they may already have updated in place) from the pre-pass planes.
// A node reads and writes only its own slots of the buffer (the AA
// pattern), so updating a row leaves the arrivals of the next one intact.
// `flip` / `gflip` = 1 turns every member's orientation of f, h, p, n / of g
// (odd steps of a captured block).  STD: the default MRT rates compiled in.
//
// The tile's walk in the orientations PAR (f, h, p, n) and GPAR (g).
template <class S, class R, class T0, int NW, bool STD, int PAR, int GPAR>
__device__ __forceinline__ void sweep_aa_tile(SweepLds<S, R, 64 * NW>& L,
                                              const SimDescAA<S, R, T0>& sd,
                                              const BatchTile& tl) {
  typedef typename WorkOf<S>::type W;
  constexpr int TW = 64 * NW;
  const KP<R>& kp = sd.kp;
  const int nx = kp.nx, ny = kp.ny, x0 = tl.x0, y0 = tl.y0, yend = tl.yend;
  const int w = min(TW, nx - x0);
  const int lane = (int)threadIdx.x;
  const bool valid = lane < w;
  const int x = x0 + (valid ? lane : 0);
  const bool periodic = kp.walls == WALL_PERIODIC;
  constexpr int par = PAR, gpar = GPAR;
  // Loads carry the non-temporal hint of the two-buffer sweep on even steps
  // (a node's own slots): measured on MI355X at 2048^2 against cached loads,
  // +2.4 % FP64, +1.0 % FP32, +0.5 % binary16 per step.  On odd steps, which
  // gather from and scatter to the neighbours' slots, they carry it where the
  // storage is narrower than the arithmetic (with the odd steps' store hint:
  // +5.4 % binary16, +3.0 % FP32 storage with FP64 arithmetic) and are cached
  // otherwise (the hint cost FP32 0.5 % and FP64 3.1 %).
  constexpr bool kLoadNT = PAR == 0 || sizeof(S) < sizeof(R);
  const AAView<S, R> V{PopView<S, R>{make_rsrc(sd.pop, kp.pop_bytes), &kp, kLoadNT}};
  const ColsP k = cols_for<0>(x, nx, 0);
  // halo columns (lanes 0 and 1): x0 - 1 and x0 + w, periodic in x
  const int xh = lane == 0 ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + w == nx ? 0 : x0 + w);
  const int kcol = lane == 0 ? 0 : w + 1;
  auto slot = [&](int yy) { return (yy - y0 + 1) % RING; };
  // phi', psi' of row yy into the ring: the tile's own rows from the
  // arrivals (parked for the update), the rows beyond the band and the halo
  // columns from the planes
  auto ring_row = [&](int yy) {
    const int ys = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
    const int sl = slot(yy);
    const uint32_t jo = (uint32_t)ys * kp.pitch + x;
    const bool own = valid && yy >= y0 && yy < yend;
    // With the pulls in the storage type (FP32, FP64) a thread's own loads
    // are issued before the halo lanes' plane loads, so that the wave holding
    // those lanes waits once for both (measured on MI355X at 2048^2: FP64
    // +3.0 %, FP32 +0.7 %; FP32 storage with FP64 arithmetic -2.6 %).
    constexpr bool kOwnFirst = sizeof(S) == sizeof(R);
    R h[9], g4[4];
    T0 h0v{};
    auto own_loads = [&]() {
#pragma unroll
      for (int i = 1; i < 9; ++i) h[i] = V.in(par, QH, i, k, ys);
#pragma unroll
      for (int i = 0; i < 4; ++i) g4[i] = V.in(gpar, QG, i + 1, k, ys);
      aa_refs_h(V, k, ys, h);
      aa_refs_g(V, k, ys, g4);
      h0v = *elem(sd.h0, jo);
    };
    if (kOwnFirst && own) own_loads();
    if (lane < 2) {
      const uint32_t jh = (uint32_t)ys * kp.pitch + xh;
      L.phi[sl][kcol] = *elem(sd.phiP, jh);
      L.psi.set(sl, kcol, *elem(sd.psiP, jh));
    }
    if (!valid) return;
    if (!own) {
      L.phi[sl][lane + 1] = *elem(sd.phiP, jo);
      L.psi.set(sl, lane + 1, *elem(sd.psiP, jo));
      return;
    }
    if (!kOwnFirst) own_loads();
    L.phi[sl][lane + 1] = phi_of<W>((W)rest_val(h0v), h);
    L.psi.set(sl, lane + 1, psi_as<W>(g4));
    const int b = (yy - y0 + 2) & 1;
#pragma unroll
    for (int i = 1; i < 9; ++i) L.pull[b][i - 1][lane] = (typename ParkOf<S, R>::type)h[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) L.pull[b][8 + i][lane] = (typename ParkOf<S, R>::type)g4[i];
  };

  if (y0 > 0 || periodic) ring_row(y0 - 1);
  ring_row(y0);
  for (int y = y0; y < yend; ++y) {
    const bool up = y + 1 < ny || periodic;
    const bool down = y > 0 || periodic;
    R f[9], p[5], n[5];
    R g0 = R(0);
    __builtin_amdgcn_s_setprio(2);
    if (valid) {
#pragma unroll
      for (int i = 0; i < 9; ++i) f[i] = V.in(par, QF, i, k, y);
      // (with binary16 storage the ion rest populations are read by the update)
      p[0] = IonRest<S>::value ? R(0) : V.in(par, QP, 0, k, y);
      n[0] = IonRest<S>::value ? R(0) : V.in(par, QN, 0, k, y);
#pragma unroll
      for (int i = 1; i < 5; ++i) {
        p[i] = V.in(par, QP, i, k, y);
        n[i] = V.in(par, QN, i, k, y);
      }
      g0 = aa_g0(V, gpar, k, y);
    }
    if (up) ring_row(y + 1);
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    if (valid) {
      const int c = lane + 1, sc = slot(y);
      W phC[3] = {L.phi[sc][c - 1], L.phi[sc][c], L.phi[sc][c + 1]};
      W psC[3] = {L.psi.get(sc, c - 1), L.psi.get(sc, c), L.psi.get(sc, c + 1)};
      W phU[3], phD[3], psU[3], psD[3];
      if (up) {
        const int su = slot(y + 1);
        phU[0] = L.phi[su][c - 1]; phU[1] = L.phi[su][c]; phU[2] = L.phi[su][c + 1];
        psU[0] = L.psi.get(su, c - 1); psU[1] = L.psi.get(su, c); psU[2] = L.psi.get(su, c + 1);
      } else {
        ghost_row(phC, psC, phU, psU);
      }
      if (down) {
        const int sd0 = slot(y - 1);
        phD[0] = L.phi[sd0][c - 1]; phD[1] = L.phi[sd0][c]; phD[2] = L.phi[sd0][c + 1];
        psD[0] = L.psi.get(sd0, c - 1); psD[1] = L.psi.get(sd0, c); psD[2] = L.psi.get(sd0, c + 1);
      } else {
        ghost_row(phC, psC, phD, psD);
      }
      W phi9[9], psi9[9];
      nine(phD, phC, phU, phi9);
      nine(psD, psC, psU, psi9);
      const HGLds<R, typename ParkOf<S, R>::type, TW> hg{L.pull[(y - y0 + 2) & 1], lane};
      update_node_aa<S, R, T0, STD>(V, par, gpar, sd.jprev, sd.h0, kp, sd.kpw, x, y, k, phi9,
                                    psi9, f, p, n, g0, hg);
    }
  }
}

template <class S, class R, class T0, int NW, bool STD>
__global__ __launch_bounds__(64 * NW)
__attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 2))) void k_sweep_aa(
    const SimDescAA<S, R, T0>* __restrict__ sims, const BatchTile* __restrict__ tiles,
    int xcd_chunk, int flip, int gflip) {
  __shared__ SweepLds<S, R, 64 * NW> L;
  const BatchTile tl = tiles[xcd_tile(xcd_chunk)];
  if (tl.sim < 0) return;
  const SimDescAA<S, R, T0>& sd = sims[tl.sim];
  // The orientations are the member's, the same for the whole workgroup:
  // one compiled walk for each pair, in which every line and slot of the AA
  // addressing is a constant.  With the orientation a run-time value, the
  // selects of line and offset in every access cost a third of the binary16
  // sweep's time and a tenth of the FP32 one's (MI355X, 2048^2, a node's
  // own slots: 225 against 157 us, 232 against 204 us).
  const int par = (sd.par + flip) & 1, gpar = (sd.gpar + gflip) & 1;
  if (par == 0) {
    if (gpar == 0)
      sweep_aa_tile<S, R, T0, NW, STD, 0, 0>(L, sd, tl);
    else
      sweep_aa_tile<S, R, T0, NW, STD, 0, 1>(L, sd, tl);
  } else {
    if (gpar == 0)
      sweep_aa_tile<S, R, T0, NW, STD, 1, 0>(L, sd, tl);
    else
      sweep_aa_tile<S, R, T0, NW, STD, 1, 1>(L, sd, tl);
  }
}

// ---------------------------------------------------------------------------
// Helpers of the in-place form outside the hot loop (2-D launches, one
// thread per node).  `par` / `gpar` are the orientations of the state.
// ---------------------------------------------------------------------------

// phi', psi' and rho_e = e0 (P' - Q') of every node into compact planes (as
// k_moments).
template <class S, class R, class T0>
__global__ void k_aa_moments(const S* __restrict__ src, const T0* __restrict__ h0x,
                             R* __restrict__ mom, const KP<R> kp, int par, int gpar) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= kp.nx) return;
  const AAView<S, R> V{PopView<S, R>{make_rsrc(src, kp.pop_bytes), &kp, false}};
  const Cols k = cols_of(x, kp.nx, 0);
  R h[9], g4[4];
  h[0] = (R)rest_val(*elem(h0x, (uint32_t)y * kp.pitch + x));
  for (int i = 1; i < 9; ++i) h[i] = V.in(par, QH, i, k, y);
  for (int i = 0; i < 4; ++i) g4[i] = V.in(gpar, QG, i + 1, k, y);
  aa_refs_h(V, k, y, h);
  aa_refs_g(V, k, y, g4);
  const R Pd = aa_ion<R>(V, h0x, par, QP, k, x, y);
  const R Qd = aa_ion<R>(V, h0x, par, QN, k, x, y);
  const long long c = (long long)y * kp.nx + x, np = (long long)kp.nx * kp.ny;
  mom[c] = sum9(h);
  mom[np + c] = psi_of(g4);
  mom[2 * np + c] = kp.q * (Pd - Qd);
}

// psi' of every node into its moment plane (g-only sweeps).
template <class S, class R>
__global__ void k_aa_psi_plane(const S* __restrict__ src, R* __restrict__ mom, const KP<R> kp,
                               int gpar) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= kp.nx) return;
  const AAView<S, R> V{PopView<S, R>{make_rsrc(src, kp.pop_bytes), &kp, false}};
  const Cols k = cols_of(x, kp.nx, 0);
  R g4[4];
  for (int i = 0; i < 4; ++i) g4[i] = V.in(gpar, QG, i + 1, k, y);
  aa_refs_g(V, k, y, g4);
  mom[(long long)kp.nx * kp.ny + (long long)y * kp.nx + x] = psi_of(g4);
}

// One g-only sweep in place (phi and rho_e held fixed, from the moment
// planes), orientation gpar; the g set then has the other orientation.
template <class S, class R>
__global__ void k_aa_poisson(S* __restrict__ buf, const R* __restrict__ mom, const KP<R> kp,
                             int gpar) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= kp.nx) return;
  const AAView<S, R> V{PopView<S, R>{make_rsrc(buf, kp.pop_bytes), &kp, false}};
  const Cols k = cols_of(x, kp.nx, 0);
  R phi9[9], psi9[9], g[5];
  hood(mom, kp, x, y, phi9, psi9);
  g[0] = aa_g0(V, gpar, k, y);
  for (int i = 1; i < 5; ++i) g[i] = V.in(gpar, QG, i, k, y);
  aa_refs_g(V, k, y, g + 1);
  const long long np = (long long)kp.nx * kp.ny;
  const long long c = (long long)y * kp.nx + x;
  const R eps = (R(0.5) + phi9[0]) * kp.deps + kp.eps_v;
  R gphi[2], gpsi[2];
  grad_lap<R>(phi9, gphi, nullptr);
  grad_lap<R>(psi9, gpsi, nullptr);
  gpsi[1] += kp.psi_slope;
  const R geps[2] = {kp.deps * gphi[0], kp.deps * gphi[1]};
  collide_g(g, psi9[0], poisson_source<R>(mom[2 * np + c], recip(eps), geps, gpsi, kp), kp);
  if constexpr (LocalG<S>::value) {  // the references of the sweep's g store
    R t[5];
    for (int i = 0; i < 5; ++i) t[i] = V.P.stored(QRG, psi9[i]);
    if (kp.walls != WALL_PERIODIC) {
      if (y == 0) t[4] = t[0];
      if (y == kp.ny - 1) t[2] = t[0];
    }
    V.P.put(QRG, V.P.row(y + 1) + x, t[0]);
    const R sixth = R(1.0 / 6.0);
    V.out(gpar, QG, 0, k, y, g[0] + R(2.0 / 3.0) * t[0], g[0]);
    for (int i = 1; i < 5; ++i) V.out(gpar, QG, i, k, y, g[i] - t[i] * sixth, -g[i] - t[0] * sixth);
  } else {
    for (int i = 0; i < 5; ++i) V.out(gpar, QG, i, k, y, g[i], -g[i]);
  }
}

// Macroscopic fields (FP64 output, [10][ny][nx]), as k_fields.
template <class S, class R, class T0>
__global__ void k_aa_fields(const S* __restrict__ src, const T0* __restrict__ h0x,
                            const R* __restrict__ mom, double* __restrict__ out, const KP<R> kp,
                            int par) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= kp.nx) return;
  const AAView<S, R> V{PopView<S, R>{make_rsrc(src, kp.pop_bytes), &kp, false}};
  const Cols k = cols_of(x, kp.nx, 0);
  R phi9[9], psi9[9], f[9];
  hood(mom, kp, x, y, phi9, psi9);
  for (int i = 0; i < 9; ++i) f[i] = V.in(par, QF, i, k, y);
  const R Pd = aa_ion<R>(V, h0x, par, QP, k, x, y);
  const R Qd = aa_ion<R>(V, h0x, par, QN, k, x, y);
  Macro<R> m;
  macro(phi9, psi9, Pd, Qd, f, kp, m);
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

// FP64 sums of one row, as k_row_sums (same layout and tree).
template <class S, class R, class T0>
__global__ __launch_bounds__(256) void k_aa_row_sums(const S* __restrict__ src,
                                                     const T0* __restrict__ h0x,
                                                     double* __restrict__ part, const KP<R> kp,
                                                     int par, int gpar) {
  __shared__ double sh[NSUM][4];
  const int y = blockIdx.x, t = threadIdx.x;
  const AAView<S, R> V{PopView<S, R>{make_rsrc(src, kp.pop_bytes), &kp, false}};
  double acc[NSUM] = {0, 0, 0, 0, 0, 0, 0};
  const double c0 = (double)kp.c0;
  for (int x = t; x < kp.nx; x += 256) {
    const Cols k = cols_of(x, kp.nx, 0);
    RestAcc<T0> content = RestAcc<T0>::from_rest(*elem(h0x, (uint32_t)y * kp.pitch + x));
    R h[9];
    for (int i = 1; i < 9; ++i) h[i] = V.in(par, QH, i, k, y);
    aa_refs_h(V, k, y, h);
    bool finite = true;
    for (int i = 1; i < 9; ++i) {
      content.add(h[i]);
      finite = finite && isfinite((double)h[i]);
    }
    const double phid = finite ? content.content() : NAN;
    const double Pd = aa_ion<double>(V, h0x, par, QP, k, x, y);
    const double Qd = aa_ion<double>(V, h0x, par, QN, k, x, y);
    R g4[4];
    for (int i = 0; i < 4; ++i) g4[i] = V.in(gpar, QG, i + 1, k, y);
    aa_refs_g(V, k, y, g4);
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

}  // namespace lbm
