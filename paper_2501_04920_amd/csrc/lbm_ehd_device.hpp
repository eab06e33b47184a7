// lbm_ehd_device.hpp -- device arithmetic of the five-equation sweep.
//
// Method: Zheng, Wang, Xiong, Huang, Luo, "Phase-field lattice Boltzmann
// method for two-phase electrohydrodynamic flows induced by Onsager-Wien
// effect", arXiv 2501.04920, Sec. 4.
//
// Memory layout (structure of arrays per lattice row; the rest population
// of h lives in the aux buffer, see RestOf):
//   a buffer is ny + 2 lattice rows, each 33 lines of `pitch` elements, one
//   line per population (34 with bfloat16 storage, 41 with the ions on
//   D2Q9; the row stride is `rstride`): population q of row r, column x is
//   element (r * 33 + q) * pitch + x.  Line q of row r = y + 1 holds, at column x,
//   the post-collision population q of node (x, y) from the previous step,
//   so that the population arriving at (x, y) along c_q is read ("pulled")
//   at row y - c_qy + 1, column (x - c_qx) mod nx.  Rows 0 and ny + 1 are
//   ghost rows: at a wall they hold the reflected populations written by the
//   wall node itself, in a y-periodic box the populations leaving the
//   opposite edge.  Populations: f 0-8, h 9-17, p 18-22, n 23-27, g 28-32.
//   Keeping the 33 lines of a row together makes each sweep row one
//   contiguous ~33 * pitch stretch of memory instead of 33 streams a plane
//   apart, which the HBM serves measurably faster.
//
// Deviation form: every plane stores x_q - ref_q with a fixed reference
//   f: 0;  h: w_q / 2;
//   p, n: wbar_q c0.  With 16-bit storage the ion lines are stored relative
//      to the uniform steady bulk instead: concentration c_b = c0 sqrt(1 +
//      2 gamma_v G) (the Onsager-Wien equilibrium in the applied field
//      G = dpsi / ny of the outer phase) drifting at mu_v G, wbar_q c_b
//      (1 +- 3 c_qy mu_v G), so that neither the field-enhanced dissociation
//      nor the ohmic flux of the bulk is carried by the 16-bit values (the
//      collisions still work on deviations from wbar_q c0: loads add and
//      stores subtract the per-line offset);
//   g: the exact steady post-collision populations of the uncharged
//      potential between the electrodes, psi_lin(y) = dpsi (ny - 1/2 - y) / ny
//      (0 in a y-periodic box): -2 psi_lin / 3, psi_lin / 6 (+x, -x),
//      psi_lin / 6 +- a_g (+y, -y), a_g = (tau_g - 1) dpsi / (6 ny).  These
//      are a fixed point of streaming, the g collision of Eq. (44)-(47)
//      without source, and the anti-bounce-back at both electrodes, so the
//      pulled deviations are the stored ones (no reference shift) and the g
//      update is the same MRT collision applied to deviations alone.
//   With 16-bit storage the moving h and g populations are further stored
//   relative to node-local references (LocalH, LocalG) and the rest
//   populations of p and n are kept in FP64 planes (IonRest).
// All arithmetic works on deviations: phi' = phi - 1/2, P' = sum p - c0,
// Q' = sum n - c0, psi' = psi - psi_lin.  The charge density q (P' - Q') and
// the reaction (solved for R directly) never subtract two numbers near c0,
// and the Poisson update never carries the O(dpsi / ny) populations of the
// applied field, which keeps FP32 and 16-bit arithmetic accurate.  Every step
// is the same arithmetic as the paper's up to rounding.
//
// Velocity order (both lattices share the first five): 0 rest, 1 +x, 2 +y,
// 3 -x, 4 -y, 5 (+x,+y), 6 (-x,+y), 7 (-x,-y), 8 (+x,-y)  (Eq. 25-26).
//
// The MRT collisions run in moment space: the raw moments of Eq. (28) / (46)
// are formed with a few additions, each moment is relaxed with its own rate,
// and the populations are rebuilt with the closed-form inverse (entries
// 0, +-1/4, +-1/2, +-1).  Equilibrium and forcing moments are the moments of
// the paper's equilibria and forcing terms, written out in closed form.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int NPOP = 33;
enum { QF = 0, QH = 9, QP = 18, QN = 23, QG = 28 };
enum { WALL_ELECTRODES = 0, WALL_INSULATING = 1, WALL_PERIODIC = 2 };
// rows of phi'/psi' kept in LDS: a row's three, and the next one, written
// before the row's barrier while slower waves may still read the last three
constexpr int RING = 4;

// Kernel constants, in the arithmetic type R.
template <class R>
struct KP {
  int nx, ny, pitch, walls;
  uint32_t rstride;             // elements per lattice row of a buffer, lines * pitch
  uint32_t cells;               // elements per aux plane, ny * pitch
  uint32_t pop_bytes;           // size of a population buffer
  int reaction, poisson_form, flow, ion_force;
  int mask_f, mask_h, mask_p, mask_n, mask_g;
  R rho_v, drho, eta_v, deta, eps_v, deps, mu_v, dmu, m_ratio;
  R three_vth;       // 3 k_B T / e0, so that 1/tau = 1/(1/2 + 3 v_th mu)
  R c0, c0sq, q, gve;  // c0, c0^2, e0, gamma_v * eps_v
  R beta4, kappa;    // 4 beta = 48 zeta / W, kappa = 3 zeta W / 2 (Eq. 13)
  R W, fourW;        // interface width and 4 / W (Eq. 2)
  R s_free, inv_tau_h, inv_tau_g;
  R n_eps2;          // square of the unit normal's regularisation (0: bare form)
  R theta_src;       // theta times the source normalisation
  R dpsi, psi_slope; // anode potential; d psi_lin / dy (0 in a periodic box)
  R a_g;             // (tau_g - 1) dpsi / (6 ny): reference offset of g +-y
  R iofs[10];        // 16-bit storage: offsets of the p and n lines (see above)
  R force_x, force_y;
  R sc[5], isc[5];   // binary16 storage: power-of-two scale of each set (f h p n g)
  int side_walls;    // 1: walls at x = -1/2 and nx - 1/2 (else periodic in x)
  int local_field;   // 1: E from the g populations (Eq. 50), else -grad psi (Eq. 59)
  int ion_q9;        // 1: the ions on D2Q9 (lines QP9, QN9 hold their diagonals)
};

// Population set of plane q: 0 f, 1 h, 2 p, 3 n, 4 g.
__host__ __device__ constexpr int set_of(int q) {
  return q < QH ? 0 : (q < QP ? 1 : (q < QN ? 2 : (q < QG ? 3 : 4)));
}

// ---------------------------------------------------------------------------
// Buffer access.  Population planes are read and written with raw buffer
// instructions: the uniform part of an address (which plane) goes in the
// scalar offset, the per-lane part (row and column) in the vector offset.
// This keeps one vector register per column instead of one per
// (plane, column) pair, and the descriptor's size bounds every access.
// ---------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t Rsrc;

__device__ inline Rsrc make_rsrc(const void* base, uint32_t bytes) {
  // raw buffer (stride 0), range in bytes; word 3 as used for gfx9 raw buffers
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}

// Storage codecs: load/store one element at byte offsets (voff, soff).
// Population stores carry the non-temporal hint: nothing reads them before
// the whole grid has streamed through the caches, and the hint keeps them
// from displacing the lines that neighbouring workgroups are still pulling.
// They also carry device scope (SC1): measured on MI355X at 2048^2 against
// the hint alone, FP32 +1.9 %, FP16 +1 %, FP64 +5 % (device scope without the
// hint: -13 %).
// Population loads carry it too (`nt`), except where a line is known to be
// read again soon: almost every element is read by one node only, so its
// line is best evicted first (measured on MI355X at 2048^2: FP32 16.6 ->
// 17.4 GLUPS, FP16 22.8 -> 23.6).
constexpr int ST_NT = 2 | 16;  // NT | SC1
constexpr int LD_NT = 2;
template <class S, class R>
struct Codec;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <>
struct Codec<double, double> {
  __device__ static inline double ld(Rsrc r, uint32_t v, uint32_t s, bool nt) {
    return __builtin_bit_cast(double, nt ? __builtin_amdgcn_raw_buffer_load_b64(r, v, s, LD_NT)
                                         : __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
  }
  __device__ static inline void st(Rsrc r, uint32_t v, uint32_t s, double x) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, v, s, ST_NT);
  }
};
template <>
struct Codec<float, float> {
  __device__ static inline float ld(Rsrc r, uint32_t v, uint32_t s, bool nt) {
    return __builtin_bit_cast(float, nt ? __builtin_amdgcn_raw_buffer_load_b32(r, v, s, LD_NT)
                                        : __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
  }
  __device__ static inline void st(Rsrc r, uint32_t v, uint32_t s, float x) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, v, s, ST_NT);
  }
};
template <>
struct Codec<float, double> {
  __device__ static inline double ld(Rsrc r, uint32_t v, uint32_t s, bool nt) {
    return (double)__builtin_bit_cast(float, nt ? __builtin_amdgcn_raw_buffer_load_b32(r, v, s, LD_NT)
                                                : __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
  }
  __device__ static inline void st(Rsrc r, uint32_t v, uint32_t s, double x) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, (float)x), r, v, s, ST_NT);
  }
};
template <>
struct Codec<__half, float> {
  __device__ static inline float ld(Rsrc r, uint32_t v, uint32_t s, bool nt) {
    const unsigned short b = nt ? __builtin_amdgcn_raw_buffer_load_b16(r, v, s, LD_NT)
                                : __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0);
    return __half2float(__builtin_bit_cast(__half, b));
  }
  __device__ static inline void st(Rsrc r, uint32_t v, uint32_t s, float x) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, __float2half_rn(x)),
                                          r, v, s, ST_NT);
  }
};
template <>
struct Codec<__hip_bfloat16, float> {
  __device__ static inline float ld(Rsrc r, uint32_t v, uint32_t s, bool nt) {
    const unsigned short b = nt ? __builtin_amdgcn_raw_buffer_load_b16(r, v, s, LD_NT)
                                : __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0);
    return __bfloat162float(__builtin_bit_cast(__hip_bfloat16, b));
  }
  __device__ static inline void st(Rsrc r, uint32_t v, uint32_t s, float x) {
    __builtin_amdgcn_raw_buffer_store_b16(
        __builtin_bit_cast(unsigned short, __float2bfloat16(x)), r, v, s, ST_NT);
  }
};

// The value x takes once converted to the storage type.
template <class S, class R>
__device__ inline R stored_as(R x);
template <>
__device__ inline double stored_as<double, double>(double x) { return x; }
template <>
__device__ inline float stored_as<float, float>(float x) { return x; }
template <>
__device__ inline double stored_as<float, double>(double x) { return (double)(float)x; }
template <>
__device__ inline float stored_as<__half, float>(float x) {
  return __half2float(__float2half_rn(x));
}
template <>
__device__ inline float stored_as<__hip_bfloat16, float>(float x) {
  return __bfloat162float(__float2bfloat16(x));
}

// Type of the rest population of h, kept next to (phi u)(t-1).  It absorbs
// the rounding of the eight moving h populations of its node, so that every
// collision conserves the node's phi.  (In FP32 the per-step changes of
// slowly varying cells would fall below half an ulp of the rest population
// and be lost, always in the same direction.)
//   FP64 (FP64 and 16-bit storage): conserved to FP64 rounding.
//   Fix32 (FP32 storage): 32-bit fixed point, value q 2^-30 (|value| < 2),
//     booked in integers (RestAcc): a node's content is its rest plus the
//     fixed-point images fixq() of its eight incoming populations, and its
//     outgoing rest is that content minus the images of the eight it
//     stores.  Streaming moves stored values unchanged, so the sum of the
//     contents over the grid is conserved exactly, in 4 bytes instead of 8.
//     The phase the collision sees is the rest plus the populations
//     themselves, within 8 2^-31 of the content.
struct Fix32 {
  int32_t q;
};
constexpr double FIX_UNIT = 0x1p-30;
template <class S>
struct RestOf {
  typedef double type;
};
template <>
struct RestOf<float> {
  typedef Fix32 type;
};
__host__ __device__ inline double rest_val(double r) { return r; }
__host__ __device__ inline double rest_val(Fix32 r) { return (double)r.q * FIX_UNIT; }
// fixed-point image of a stored FP32 population: exact power-of-two scaling,
// then the nearest integer
__device__ inline int32_t fixq(float x) { return (int32_t)__builtin_rintf(x * 0x1p30f); }
__device__ inline int32_t fixq(double x) { return (int32_t)__builtin_rint(x * 0x1p30); }

// A node's phi content in the rest type's bookkeeping (see RestOf): built
// from the rest population and the incoming moving ones, then reduced by the
// outgoing ones to the new rest.
template <class T0>
struct RestAcc {
  double m;
  __device__ static RestAcc from_rest(T0 r) { return RestAcc{(double)r}; }
  __device__ static RestAcc from_content(double c) { return RestAcc{c}; }
  template <class X>
  __device__ void add(X x) { m += (double)x; }
  template <class X>
  __device__ void sub(X x) { m -= (double)x; }
  __device__ double content() const { return m; }
  __device__ T0 rest() const { return (T0)m; }
};
template <>
struct RestAcc<Fix32> {
  uint32_t m;  // two's complement, wrapping: the end result fits in 32 bits
  __device__ static RestAcc from_rest(Fix32 r) { return RestAcc{(uint32_t)r.q}; }
  __device__ static RestAcc from_content(double c) {
    return RestAcc{(uint32_t)(int32_t)__builtin_rint(c * 0x1p30)};
  }
  template <class X>
  __device__ void add(X x) { m += (uint32_t)fixq(x); }
  template <class X>
  __device__ void sub(X x) { m -= (uint32_t)fixq(x); }
  __device__ double content() const { return (double)(int32_t)m * FIX_UNIT; }
  __device__ Fix32 rest() const { return Fix32{(int32_t)m}; }
};

// Working type of the sweep for a storage type: the phase ring, the
// macroscopic quantities, the f, p, n, g collisions and the readback.  FP64
// with FP32 or FP64 storage, FP32 with 16-bit storage.
template <class S>
struct WorkOf {
  typedef double type;
};
template <>
struct WorkOf<__half> {
  typedef float type;
};
template <>
struct WorkOf<__hip_bfloat16> {
  typedef float type;
};

// binary16 has a narrow exponent range: its deviations are stored scaled by a
// power of two per set (exact) so that small values stay normal numbers.
template <class S>
struct Scaled {
  static constexpr bool value = false;
};
template <>
struct Scaled<__half> {
  static constexpr bool value = true;
};

// 16-bit storage keeps the moving h populations relative to w_i times the
// phase of the node they arrive at, phi'~ (phi' = phi - 1/2 of that node at
// the step they were sent, rounded to the storage type and stored by the node
// itself in the line of h0, which the population buffers do not otherwise
// use).  The stored deviations are then the O(|u|) and non-equilibrium parts
// only, about a hundred times smaller than phi itself, and 16-bit rounding
// no longer shakes the interface.  Wider storage keeps the fixed reference.
template <class S>
struct LocalH {
  static constexpr bool value = false;
};
template <>
struct LocalH<__half> {
  static constexpr bool value = true;
};
template <>
struct LocalH<__hip_bfloat16> {
  static constexpr bool value = true;
};
// 16-bit storage also keeps the rest populations of the two ions in FP64
// planes beside that of h, and like it they take what the node's four stored
// moving populations leave: each collision then changes a node's ion content
// by exactly the reaction term.  Rounded to 16 bits, the content of slowly
// varying nodes would move by a fraction of an ulp per step, always in the
// same direction, and the charge, which relaxes only over the dielectric
// time, would integrate that drift.
template <class S>
struct IonRest {
  static constexpr bool value = LocalH<S>::value;
};
// FP64 rest planes per time level: h0, then p0 and n0 where kept there
template <class S>
constexpr int rest_planes() {
  return IonRest<S>::value ? 3 : 1;
}
// 16-bit storage keeps the moving g populations relative to w_i times the
// potential psi'~ of the node they arrive at, and g0 relative to its share
// (w_0 - 1) psi'~ of its own node, like h (psi' = psi - psi_lin, rounded to
// the storage type and stored by each node in line QRG, the line of p0,
// which that storage keeps in FP64).  The stored deviations are then the
// non-equilibrium parts only, about a hundred times smaller than psi'/6:
// rounded to 16 bits, psi'/6 itself is a noise source that the Poisson
// iteration amplifies by the condition number of the Laplacian.
template <class S>
struct LocalG {
  static constexpr bool value = IonRest<S>::value;
};
constexpr int QRG = QP;
// bfloat16 storage (an 8-bit significand) also keeps the moving f relative
// to their dominant term, 3 w_i c_i . J~ with J~ = rho u of the node that sent
// them (at the step it sent them, rounded to the storage type and stored by
// that node in lines QJX and QJY): relative to 0 the velocity term of the
// equilibrium, ~3 w_i rho c_i . u, is rounded at ~2e-3 every step, which is
// where that storage's whole deformation error came from.  QJX is the line
// of n0 (kept in FP64 by that storage); QJY is a 34th line.  Populations that
// pass through a ghost row (reflected at an electrode, or wrapped in a
// y-periodic box) are stored relative to 0.
template <class S>
struct LocalF {
  static constexpr bool value = false;
};
template <>
struct LocalF<__hip_bfloat16> {
  static constexpr bool value = true;
};
constexpr int QJX = QN, QJY = NPOP;
// Ions on D2Q9 (the lattice of Eq. 34-38 as printed): directions 0-4 of each
// species keep their lines (QP.., QN..), the diagonals 5-8 take four more
// lines each at the end of the row, 41 lines in all.
constexpr int QP9 = NPOP, QN9 = NPOP + 4, NPOP9 = NPOP + 8;
// lines per lattice row of a buffer
template <class S>
constexpr int lines_of() {
  return LocalF<S>::value ? NPOP + 1 : NPOP;
}
// Reference of moving f population i (1..8) for the momentum (jx, jy) of its
// sender: 3 w_i c_i . J, the same expression for the sender and the receiver.
template <class R>
__device__ inline R f_ref(int i, R jx, R jy) {
  const R a = R(1.0 / 3.0), b = R(1.0 / 12.0);
  switch (i) {
    case 1: return a * jx;
    case 2: return a * jy;
    case 3: return -(a * jx);
    case 4: return -(a * jy);
    case 5: return b * (jx + jy);
    case 6: return b * (jy - jx);
    case 7: return -(b * (jx + jy));
    case 8: return b * (jx - jy);
  }
  return R(0);
}
// Scale set of line a: the reference line of g is scaled like g.
template <class S>
__device__ inline int line_set(int a) {
  return LocalG<S>::value && a == QRG ? 4 : set_of(a);
}
// lattice weights of Eq. (25), for the references above
__device__ constexpr float W9F[9] = {4.f / 9, 1.f / 9, 1.f / 9, 1.f / 9, 1.f / 9,
                                     1.f / 36, 1.f / 36, 1.f / 36, 1.f / 36};
// the moving h population a node reconstructs from a stored deviation and
// its reference phase.  The sender books exactly this value into the rest
// population, so both sides must round alike: one fused multiply-add, never
// left to the compiler's contraction (which differs between call sites).
__device__ inline float h_from(float dev, int i, float phit) {
  return __builtin_fmaf(W9F[i], phit, dev);
}
__device__ inline double h_from(double dev, int i, double phit) {
  return __builtin_fma((double)W9F[i], phit, dev);
}

// A population buffer seen through a buffer descriptor: line q of the row
// at element offset `off` = row(r) + x.  `nt`: loads with the non-temporal
// hint (a constant at every construction, so each load has one form).
template <class S, class R>
struct PopView {
  Rsrc rs;
  const KP<R>* kp;
  bool nt = true;
  __device__ inline uint32_t row(int r) const { return (uint32_t)r * kp->rstride; }
  // whether line q carries an offset: the ion lines with 16-bit storage
  // (see the deviation form).  Decided where q is known at compile time:
  // an add of a zero is no identity in IEEE arithmetic (-0 + 0 = +0), so the
  // compiler keeps it, one vector instruction per load.  Binary16 lines keep
  // the form scale * x + offset throughout, which is one mixed-precision
  // multiply-add with the conversion folded in, offset or not.
  __device__ inline bool has_ofs(int q) const {
    return LocalH<S>::value && q >= QP && q < QG && q != QRG && !(LocalF<S>::value && q == QJX);
  }
  __device__ inline R ofs(int q) const { return has_ofs(q) ? kp->iofs[q - QP] : R(0); }
  __device__ inline R at(int q, uint32_t off) const {
    R v = Codec<S, R>::ld(rs, off * (uint32_t)sizeof(S),
                          (uint32_t)q * kp->pitch * (uint32_t)sizeof(S), nt);
    if constexpr (Scaled<S>::value) return v * kp->isc[line_set<S>(q)] + ofs(q);
    if (has_ofs(q)) v += kp->iofs[q - QP];
    return v;
  }
  __device__ inline void put(int q, uint32_t off, R v) const {
    if (has_ofs(q)) v -= kp->iofs[q - QP];
    if (Scaled<S>::value) v *= kp->sc[line_set<S>(q)];
    Codec<S, R>::st(rs, off * (uint32_t)sizeof(S), (uint32_t)q * kp->pitch * (uint32_t)sizeof(S),
                    v);
  }
  // the 16-bit pattern stored in line q (16-bit storage only)
  __device__ inline unsigned short bits(int q, uint32_t off) const {
    static_assert(sizeof(S) == 2, "a 16-bit storage type");
    const uint32_t v = off * 2u, s = (uint32_t)q * kp->pitch * 2u;
    return nt ? __builtin_amdgcn_raw_buffer_load_b16(rs, v, s, LD_NT)
              : __builtin_amdgcn_raw_buffer_load_b16(rs, v, s, 0);
  }
  // the value v takes once stored in line q (and loaded back)
  __device__ inline R stored(int q, R v) const {
    if constexpr (Scaled<S>::value) {
      const R o = ofs(q);
      const int k = line_set<S>(q);
      return stored_as<S, R>((v - o) * kp->sc[k]) * kp->isc[k] + o;
    }
    if (!has_ofs(q)) return stored_as<S, R>(v);
    const R o = kp->iofs[q - QP];
    return stored_as<S, R>(v - o) + o;
  }
};

// Element `e` of a plain array, addressed as uniform base + 32-bit byte
// offset (scalar-base + vector-offset form).
template <class T>
__device__ inline T* elem(T* base, uint32_t e) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + e * (uint32_t)sizeof(T));
}

// Reference of population q stored at lattice row y (the deviation form
// above), used where absolute values enter or leave: initialisation and
// field output.
__device__ inline double plane_ref(int q, int y, int ny, int walls, double c0, double dpsi,
                                  double a_g, int ion_q9 = 0) {
  const double w9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                        1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  if (q < QH) return 0.0;
  if (q < QP) return 0.5 * w9[q - QH];
  if (q >= QP9) return w9[5] * c0;  // D2Q9 ion diagonals
  if (ion_q9 && q < QG) return w9[q < QN ? q - QP : q - QN] * c0;
  const int k = q < QN ? q - QP : (q < QG ? q - QN : q - QG);
  const double wb = k == 0 ? 1.0 / 3 : 1.0 / 6;
  if (q < QG) return wb * c0;  // the drift offsets are PopView's
  const double psi = walls == WALL_PERIODIC ? 0.0 : dpsi * (ny - 0.5 - y) / ny;
  return k == 0 ? -2.0 / 3 * psi : psi / 6 + (k == 2 ? a_g : (k == 4 ? -a_g : 0.0));
}

// ---------------------------------------------------------------------------
// Moment transforms: Eq. (28) and its inverse, Eq. (46) and its inverse.
// ---------------------------------------------------------------------------
template <class R>
__device__ inline void fwd9(const R x[9], R m[9]) {
  const R d57 = x[5] + x[7], d68 = x[6] + x[8];
  m[0] = x[0] + x[1] + x[2] + x[3] + x[4] + d57 + d68;
  m[1] = x[1] - x[3] + x[5] - x[6] - x[7] + x[8];
  m[2] = x[2] - x[4] + x[5] + x[6] - x[7] - x[8];
  m[8] = d57 + d68;
  m[3] = x[1] + x[3] + m[8];
  m[4] = x[2] + x[4] + m[8];
  m[5] = d57 - d68;
  m[6] = x[5] - x[6] - x[7] + x[8];
  m[7] = x[5] + x[6] - x[7] - x[8];
}

template <class R>
__device__ inline void inv9(const R m[9], R x[9]) {
  const R q = R(0.25);
  x[5] = q * (m[8] + m[5] + m[6] + m[7]);
  x[6] = q * (m[8] - m[5] - m[6] + m[7]);
  x[7] = q * (m[8] + m[5] - m[6] - m[7]);
  x[8] = q * (m[8] - m[5] + m[6] - m[7]);
  const R a = m[3] - m[8], b = m[1] - m[6];
  const R c = m[4] - m[8], d = m[2] - m[7];
  x[1] = R(0.5) * (a + b);
  x[3] = R(0.5) * (a - b);
  x[2] = R(0.5) * (c + d);
  x[4] = R(0.5) * (c - d);
  x[0] = m[0] - m[3] - m[4] + m[8];
}

template <class R>
__device__ inline void fwd5(const R x[5], R m[5]) {
  m[0] = x[0] + x[1] + x[2] + x[3] + x[4];
  m[1] = x[1] - x[3];
  m[2] = x[2] - x[4];
  m[3] = x[1] + x[3];
  m[4] = x[2] + x[4];
}

template <class R>
__device__ inline void inv5(const R m[5], R x[5]) {
  x[1] = R(0.5) * (m[3] + m[1]);
  x[3] = R(0.5) * (m[3] - m[1]);
  x[2] = R(0.5) * (m[4] + m[2]);
  x[4] = R(0.5) * (m[4] - m[2]);
  x[0] = m[0] - m[3] - m[4];
}

// Reciprocals of the per-node rates and properties (positive, O(1e-3..1e3)).
// FP64: the hardware estimate (v_rcp_f64) refined by two Newton steps, each
// of which squares the relative error, so the result is within an ulp or so
// of 1/x; five instructions instead of the ~eleven of the IEEE division
// sequence (scaling for denormal and huge operands, which these never are).
// FP32: the hardware reciprocal (v_rcp_f32, within 1 ulp), far inside the
// FP32 error budget.
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
  return __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
}
__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }

template <class R>
__device__ inline R rate(int mask, int k, R inv_tau, R s_free) {
  return ((mask >> k) & 1) ? inv_tau : s_free;
}

// The default MRT rates (Sec. 6, readings of which rows carry tau): rows
// 3-5 of f and rows 1-2 of h, p, n and g relax with 1/tau, every other row
// with exactly 1.  The collisions below take a compile-time flag STD for
// this case: a row relaxing with 1 becomes its equilibrium plus half its
// source (and its drift term), whatever its pre-collision moment, so that
// moment is never formed and the rate selects disappear.
constexpr int STD_MASK_F = 0x38, STD_MASK_ADE = 0x6;

// ---------------------------------------------------------------------------
// Macroscopic quantities of one node (Sec. 4: Eq. 5-9, 12-14, 33, 41-43, 49,
// 56-57, 59, 61).  phi9 / psi9 hold phi' and psi' of the node (index 0) and
// of its eight neighbours x + c_i, in the velocity order above.
// ---------------------------------------------------------------------------
template <class R>
struct Macro {
  R phi, phid, psid, rho, eps, ieps, mup, mum;  // phi, phi', psi'; ieps = 1/eps
  R itau_f, itau_p, itau_n;
  R gphi[2], lphi, gpsi[2], E[2];
  R cpd, cmd, cp, cm, Rr, rhoe;           // c+', c-', c+, c-, R, rho_e
  R F[2], grho[2], geps[2];
  R u[2], p;
};

template <class R>
__device__ inline void grad_lap(const R c[9], R g[2], R* lap) {
  const R a = R(1) / R(3), b = R(1) / R(12);
  g[0] = a * (c[1] - c[3]) + b * (c[5] - c[6] - c[7] + c[8]);
  g[1] = a * (c[2] - c[4]) + b * (c[5] + c[6] - c[7] - c[8]);
  if (lap)
    *lap = R(2) / R(3) * (c[1] + c[2] + c[3] + c[4] - R(4) * c[0]) +
           R(1) / R(6) * (c[5] + c[6] + c[7] + c[8] - R(4) * c[0]);
}

// Eq. (41)-(43) solved for the reaction rate itself.  With c+ = P + R/2 and
// c- = Q + R/2 (Eq. 41), R = delta (c0^2 F - c+ c-) (Eq. 5) is the root of
//   (delta/4) R^2 + (1 + delta (P + Q)/2) R - delta (c0^2 F - P Q) = 0
// that gives c+ >= 0, the same root as Eq. (42).  c0^2 F - P Q is formed from
// deviations: c0^2 (F - 1) - c0 (P' + Q') - P' Q'.
template <class R>
__device__ inline R reaction_rate(R delta, R c0, R c0sq, R Fm1, R Pd, R Qd) {
  const R Cn = c0sq * Fm1 - c0 * (Pd + Qd) - Pd * Qd;
  const R B = R(1) + R(0.5) * delta * (R(2) * c0 + Pd + Qd);
  const R AC = R(0.25) * delta * delta * Cn;  // (delta/4) (delta Cn)
  return R(2) * delta * Cn * recip(B + sqrt(B * B + R(4) * AC));
}

// Eq. (50): the field from the first moment of the node's incoming g,
// E = sum_i c_i g_i / (c_s^2 tau_g), from its deviations g1'..g4'.  The
// references of the uncharged field carry psi_lin(y -+ 1) / 6 -+ a_g in the
// +-y populations, i.e. a y moment of 2 a_g - psi_slope / 3 (the applied
// field exactly, dpsi / ny, when that moment relaxes with 1 / tau_g).
template <class W, class R>
__device__ inline void field_from_g(const R g4[4], const KP<W>& kp, W E[2]) {
  const W s = W(3) * kp.inv_tau_g;
  E[0] = s * ((W)g4[0] - (W)g4[2]);
  E[1] = s * (((W)g4[1] - (W)g4[3]) + (W(2) * kp.a_g - kp.psi_slope * (W(1) / W(3))));
}

// phi9 comes in the type RP of the phase ring (FP64 with FP32 storage): the
// chemical potential of Eq. (13) is the small difference of a double-well
// term and kappa lap(phi), each ~50 times larger near equilibrium, so phi',
// its stencils and mu_phi are formed in RP and rounded to R afterwards.
template <class R, class RP>
__device__ inline void macro(const RP phi9[9], const R psi9[9], R Pd, R Qd, const R f[9],
                             const KP<R>& kp, Macro<R>& m, const R* Eloc = nullptr) {
  m.phid = (R)phi9[0];
  const RP phiw = RP(0.5) + phi9[0];
  const R phi = (R)phiw;
  m.phi = phi;
  m.psid = psi9[0];
  // Eq. (61)
  m.rho = phi * kp.drho + kp.rho_v;
  const R eta = phi * kp.deta + kp.eta_v;
  m.eps = phi * kp.deps + kp.eps_v;
  m.ieps = recip(m.eps);
  m.mup = phi * kp.dmu + kp.mu_v;
  m.mum = kp.m_ratio * m.mup;
  // Eq. (55), (37)
  const R inv_rho = recip(m.rho);
  m.itau_f = recip(R(0.5) + R(3) * eta * inv_rho);
  m.itau_p = recip(R(0.5) + kp.three_vth * m.mup);
  m.itau_n = recip(R(0.5) + kp.three_vth * m.mum);
  // Eq. (59), (9); the linear part of psi contributes its exact gradient.
  // With the local field (Eq. 50, given in Eloc) grad psi = -E throughout.
  RP gph[2], lph;
  grad_lap<RP>(phi9, gph, &lph);
  m.gphi[0] = (R)gph[0];
  m.gphi[1] = (R)gph[1];
  m.lphi = (R)lph;
  if (Eloc) {
    m.E[0] = Eloc[0];
    m.E[1] = Eloc[1];
    m.gpsi[0] = -Eloc[0];
    m.gpsi[1] = -Eloc[1];
  } else {
    grad_lap<R>(psi9, m.gpsi, nullptr);
    m.gpsi[1] += kp.psi_slope;
    m.E[0] = -m.gpsi[0];
    m.E[1] = -m.gpsi[1];
  }
  // Eq. (5), (6), (41)-(43), (8)
  const R E2 = m.E[0] * m.E[0] + m.E[1] * m.E[1];
  if (kp.reaction) {
    const R delta = kp.q * (m.mup + m.mum) * m.ieps;
    const R gamma = kp.gve * m.ieps;
    m.Rr = reaction_rate(delta, kp.c0, kp.c0sq, R(2) * gamma * sqrt(E2), Pd, Qd);
    m.cpd = Pd + R(0.5) * m.Rr;
    m.cmd = Qd + R(0.5) * m.Rr;
  } else {
    m.Rr = R(0);
    m.cpd = Pd;
    m.cmd = Qd;
  }
  m.cp = kp.c0 + m.cpd;
  m.cm = kp.c0 + m.cmd;
  m.rhoe = kp.q * (Pd - Qd);  // c+ - c- = P - Q
  // Eq. (12)-(14); phi - 1/2 = phi'
  const R mu_phi =
      (R)((RP)kp.beta4 * phiw * (phiw - RP(1)) * phi9[0] - (RP)kp.kappa * lph);
  m.grho[0] = kp.drho * m.gphi[0];
  m.grho[1] = kp.drho * m.gphi[1];
  m.geps[0] = kp.deps * m.gphi[0];
  m.geps[1] = kp.deps * m.gphi[1];
  m.F[0] = mu_phi * m.gphi[0] - R(0.5) * E2 * m.geps[0] + m.rhoe * m.E[0] + kp.force_x;
  m.F[1] = mu_phi * m.gphi[1] - R(0.5) * E2 * m.geps[1] + m.rhoe * m.E[1] + kp.force_y;
  // Eq. (56)-(57)
  if (kp.flow) {
    const R jx = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
    const R jy = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
    m.u[0] = (jx + R(0.5) * m.F[0]) * inv_rho;
    m.u[1] = (jy + R(0.5) * m.F[1]) * inv_rho;
    const R snz = f[1] + f[2] + f[3] + f[4] + f[5] + f[6] + f[7] + f[8];
    const R ugr = m.u[0] * m.grho[0] + m.u[1] * m.grho[1];
    const R uu = m.u[0] * m.u[0] + m.u[1] * m.u[1];
    m.p = R(0.6) * (snz + R(0.5) * ugr - R(2) / R(3) * m.rho * uu);
  } else {
    m.u[0] = m.u[1] = R(0);
    m.p = R(0);
  }
}

// ---------------------------------------------------------------------------
// Collisions (moment space, on deviations).  Each writes post-collision
// deviations.
// ---------------------------------------------------------------------------

// f: Eq. (51)-(55) (reference 0).
template <bool STD = false, class R>
__device__ inline void collide_f(R f[9], const Macro<R>& m, const KP<R>& kp) {
  if (!kp.flow) return;
  R mo[9];
  fwd9(f, mo);
  const R ux = m.u[0], uy = m.u[1], rho = m.rho, p = m.p;
  const R gx = m.grho[0], gy = m.grho[1];
  const R ugr = ux * gx + uy * gy;
  const R third = R(1) / R(3);
  R eq[9], fo[9];
  eq[0] = R(0);
  eq[1] = rho * ux;
  eq[2] = rho * uy;
  eq[3] = p + rho * ux * ux;
  eq[4] = p + rho * uy * uy;
  eq[5] = rho * ux * uy;
  eq[6] = third * rho * ux;
  eq[7] = third * rho * uy;
  eq[8] = third * (p + rho * (ux * ux + uy * uy));
  fo[0] = ugr;
  fo[1] = m.F[0];
  fo[2] = m.F[1];
  fo[3] = ux * gx + third * uy * gy;
  fo[4] = uy * gy + third * ux * gx;
  fo[5] = third * (ux * gy + uy * gx);
  fo[6] = third * m.F[0];
  fo[7] = third * m.F[1];
  fo[8] = third * ugr;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (STD && !((STD_MASK_F >> k) & 1)) {
      mo[k] = eq[k] + R(0.5) * fo[k];
    } else {
      const R s = STD ? m.itau_f : rate(kp.mask_f, k, m.itau_f, kp.s_free);
      mo[k] = mo[k] - s * (mo[k] - eq[k]) + (R(1) - R(0.5) * s) * fo[k];
    }
  }
  inv9(mo, f);
}

// h: Eq. (27)-(32) on deviations from w_i / 2.  dJ = d(phi u)/dt by Eq. (58).
template <bool STD = false, class R, class M>
__device__ inline void collide_h(R h[9], const Macro<M>& m, const R dJ[2], const KP<R>& kp) {
  R mo[9];
  fwd9(h, mo);
  const R phi = (R)m.phi, phid = (R)m.phid, ux = (R)m.u[0], uy = (R)m.u[1];
  const R gx = (R)m.gphi[0], gy = (R)m.gphi[1];
  const R third = R(1) / R(3), ninth = R(1) / R(9);
  // unit normal grad(phi)/|grad(phi)|, regularised where grad(phi) -> 0
  const R g2 = gx * gx + gy * gy;
  R nx = R(0), ny = R(0);
  if (kp.n_eps2 > R(0) || g2 >= R(1e-24)) {
    const R ign = recip(sqrt(g2 + kp.n_eps2));
    nx = gx * ign;
    ny = gy * ign;
  }
  const R lam = kp.fourW * phi * (R(1) - phi);
  const R Ax = R(3) * dJ[0] + lam * nx, Ay = R(3) * dJ[1] + lam * ny;
  R eq[9], fo[9];
  eq[0] = phid;
  eq[1] = phi * ux;
  eq[2] = phi * uy;
  eq[3] = third * phid;
  eq[4] = third * phid;
  eq[5] = R(0);
  eq[6] = third * phi * ux;
  eq[7] = third * phi * uy;
  eq[8] = ninth * phid;
  fo[0] = R(0);
  fo[1] = third * Ax;
  fo[2] = third * Ay;
  fo[3] = R(0);
  fo[4] = R(0);
  fo[5] = R(0);
  fo[6] = ninth * Ax;
  fo[7] = ninth * Ay;
  fo[8] = R(0);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (STD && !((STD_MASK_ADE >> k) & 1)) {
      mo[k] = eq[k] + R(0.5) * fo[k];
    } else {
      const R s = STD ? kp.inv_tau_h : rate(kp.mask_h, k, kp.inv_tau_h, kp.s_free);
      mo[k] = mo[k] - s * (mo[k] - eq[k]) + (R(1) - R(0.5) * s) * fo[k];
    }
  }
  inv9(mo, h);
}

// p and n: Eq. (34)-(40) on D2Q5, deviations from wbar_i c0.  cd is c - c0;
// sign = -1 for cations (- S G), +1 for anions (+ S Gbar).  W is the working
// type (FP64 with FP32 storage: the drift flux mu c grad(psi) is ~10 times
// the deviations that carry the charge, and its FP32 rounding would random-
// walk rho_e); c = c0 + cd is formed in W.
template <bool STD = false, class W, class R>
__device__ inline void collide_ion(W x[5], W cd, R mu, R itau, int mask, W sign,
                                   const Macro<R>& m, const KP<R>& kp) {
  W mo[5];
  fwd5(x, mo);
  const W third = W(1) / W(3);
  const W c = (W)kp.c0 + cd;
  const W Lx = kp.ion_force ? c * (W)m.F[0] : W(0);
  const W Ly = kp.ion_force ? c * (W)m.F[1] : W(0);
  const W Gx = (W)mu * c * (W)m.gpsi[0], Gy = (W)mu * c * (W)m.gpsi[1];
  const W Rr = (W)m.Rr;
  const W eq[5] = {cd, c * (W)m.u[0], c * (W)m.u[1], third * cd, third * cd};
  const W so[5] = {Rr, Lx, Ly, third * Rr, third * Rr};
  const W dr[5] = {W(0), Gx, Gy, W(0), W(0)};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    if (STD && !((STD_MASK_ADE >> k) & 1)) {
      mo[k] = eq[k] + W(0.5) * so[k] + sign * dr[k];
    } else {
      const W s = STD ? (W)itau : (W)rate(mask, k, itau, kp.s_free);
      mo[k] = mo[k] - s * (mo[k] - eq[k]) + (W(1) - W(0.5) * s) * so[k] + sign * s * dr[k];
    }
  }
  inv5(mo, x);
}

// p and n on D2Q9 (Eq. 34-40 with the matrix M of Eq. 28): the same update
// in the nine raw moments, deviations from w_i c0.  The equilibrium
// w_i c (1 + 3 c_i.u) has the moments (c, c u, c/3, c/3, 0, c ux/3, c uy/3,
// c/9); R_i = w_i R has (R, 0, 0, R/3, R/3, 0, 0, 0, R/9); L_i and G_i, of the
// form w_i c_i.v / c_s^2, have v in the first moments and v/3 in moments 6, 7.
template <bool STD = false, class W, class R>
__device__ inline void collide_ion9(W x[9], W cd, R mu, R itau, int mask, W sign,
                                    const Macro<R>& m, const KP<R>& kp) {
  W mo[9];
  fwd9(x, mo);
  const W third = W(1) / W(3), ninth = W(1) / W(9);
  const W c = (W)kp.c0 + cd;
  const W Lx = kp.ion_force ? c * (W)m.F[0] : W(0);
  const W Ly = kp.ion_force ? c * (W)m.F[1] : W(0);
  const W Gx = (W)mu * c * (W)m.gpsi[0], Gy = (W)mu * c * (W)m.gpsi[1];
  const W Rr = (W)m.Rr;
  const W ux = (W)m.u[0], uy = (W)m.u[1];
  const W eq[9] = {cd, c * ux, c * uy, third * cd, third * cd, W(0),
                   third * c * ux, third * c * uy, ninth * cd};
  const W so[9] = {Rr, Lx, Ly, third * Rr, third * Rr, W(0), third * Lx, third * Ly, ninth * Rr};
  const W dr[9] = {W(0), Gx, Gy, W(0), W(0), W(0), third * Gx, third * Gy, W(0)};
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (STD && !((STD_MASK_ADE >> k) & 1)) {
      mo[k] = eq[k] + W(0.5) * so[k] + sign * dr[k];
    } else {
      const W s = STD ? (W)itau : (W)rate(mask, k, itau, kp.s_free);
      mo[k] = mo[k] - s * (mo[k] - eq[k]) + (W(1) - W(0.5) * s) * so[k] + sign * s * dr[k];
    }
  }
  inv9(mo, x);
}

// Poisson source S_psi of Eq. (44) (or its variable-eps form), in W;
// ieps = 1 / eps.
template <class W, class R>
__device__ inline W poisson_source(R rhoe, R ieps, const R geps[2], const R gpsi[2],
                                   const KP<R>& kp) {
  W s = (W)rhoe;
  if (kp.poisson_form) s += (W)geps[0] * (W)gpsi[0] + (W)geps[1] * (W)gpsi[1];
  return s * (W)ieps;
}

// g: Eq. (44)-(47) on deviations from the uncharged steady state (see the
// deviation form above): the collision is affine in g and psi, and the
// reference is its fixed point, so the deviations obey the same collision
// with the equilibrium of psi' and the source.
// W is the working type: FP64 with FP32 storage, because the Poisson LBE is
// an iterative solve whose rounding noise is amplified by the condition
// number of the Laplacian (~ny^2); in FP32 it limits psi' to ~1e-6.
template <bool STD = false, class W, class R>
__device__ inline void collide_g(W g[5], W psid, W Spsi, const KP<R>& kp) {
  W mo[5];
  fwd5(g, mo);
  const W third = W(1) / W(3);
  const W eq[5] = {W(0), W(0), W(0), third * psid, third * psid};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    if (STD && !((STD_MASK_ADE >> k) & 1)) {
      mo[k] = eq[k];
    } else {
      const W s = STD ? (W)kp.inv_tau_g : (W)rate(kp.mask_g, k, kp.inv_tau_g, kp.s_free);
      mo[k] = mo[k] - s * (mo[k] - eq[k]);
    }
  }
  inv5(mo, g);
  const W src = (W)kp.theta_src * Spsi;
  g[0] += src * (W(1) / W(3));
#pragma unroll
  for (int k = 1; k < 5; ++k) g[k] += src * (W(1) / W(6));
}

}  // namespace lbm
