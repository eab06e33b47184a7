// lbm_ehd_device.hpp -- device code of the fused five-equation sweep.
//
// Method: Zheng, Wang, Xiong, Huang, Luo, "Phase-field lattice Boltzmann
// method for two-phase electrohydrodynamic flows induced by Onsager-Wien
// effect", arXiv 2501.04920, Sec. 4.
//
// Memory layout (structure of arrays, one plane per population):
//   plane q of buffer B holds, at row r = y + 1 and column x, the
//   post-collision population q of node (x, y) from the previous step, so
//   that the population arriving at (x, y) along c_q is read ("pulled") at
//   row y - c_qy + 1, column (x - c_qx) mod nx.  Rows 0 and ny + 1 are ghost
//   rows: at a wall they hold the reflected populations written by the wall
//   node itself, in a y-periodic box the populations leaving the opposite
//   edge.  33 planes: f 0-8, h 9-17, p 18-22, n 23-27, g 28-32.
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
constexpr int TILE_W = 64;  // one wavefront of columns per workgroup
constexpr int RING = 5;     // rows of phi/psi kept in LDS

// Kernel constants, in the arithmetic type R.
template <class R>
struct KP {
  int nx, ny, pitch, walls;
  uint32_t plane;   // elements per population plane, (ny + 2) * pitch
  uint32_t pop_bytes, g_bytes;  // sizes of a population buffer and of a g set
  int reaction, poisson_form, flow, ion_force;
  int mask_f, mask_h, mask_p, mask_n, mask_g;
  R rho_v, drho, eta_v, deta, eps_v, deps, mu_v, dmu, m_ratio;
  R three_vth;       // 3 k_B T / e0, so that 1/tau = 1/(1/2 + 3 v_th mu)
  R c0sq, q, gve;    // c0^2, e0, gamma_v * eps_v
  R beta4, kappa;    // 4 beta = 48 zeta / W, kappa = 3 zeta W / 2 (Eq. 13)
  R W, fourW;        // interface width and 4 / W (Eq. 2)
  R s_free, inv_tau_h, inv_tau_g;
  R theta_src;       // theta times the source normalisation
  R dpsi, force_x, force_y;
  // reference states of the 16-bit storage forms (zero otherwise)
  R ref_p, ref_n;    // concentration whose rest equilibrium is subtracted
};

// ---------------------------------------------------------------------------
// Buffer access.  Population planes are read and written with raw buffer
// instructions: the uniform part of an address (which plane) goes in the
// scalar offset, the per-lane part (row and column) in the vector offset.
// This keeps one vector register per column instead of one per
// (plane, column) pair, and the descriptor's size bounds every access.
// ---------------------------------------------------------------------------
typedef __amdgpu_buffer_rsrc_t Rsrc;

// cache policy of population stores (gfx940+ encoding: bit 1 = nt)
#ifndef LBM_STORE_POLICY
#define LBM_STORE_POLICY 0
#endif

__device__ inline Rsrc make_rsrc(const void* base, uint32_t bytes) {
  // raw buffer (stride 0), range in bytes; word 3 as used for gfx9 raw buffers
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}

// Storage codecs: load/store one element at byte offsets (voff, soff).
// FP64/FP32 store the populations as they are; the 16-bit forms store
// x - ref, ref a fixed reference state per plane.
template <class S, class R>
struct Codec;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <>
struct Codec<double, double> {
  __device__ static inline double ld(Rsrc r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
  }
  __device__ static inline void st(Rsrc r, uint32_t v, uint32_t s, double x) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, v, s, LBM_STORE_POLICY);
  }
};
template <>
struct Codec<float, float> {
  __device__ static inline float ld(Rsrc r, uint32_t v, uint32_t s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
  }
  __device__ static inline void st(Rsrc r, uint32_t v, uint32_t s, float x) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, v, s, LBM_STORE_POLICY);
  }
};
template <>
struct Codec<float, double> {
  __device__ static inline double ld(Rsrc r, uint32_t v, uint32_t s) {
    return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
  }
  __device__ static inline void st(Rsrc r, uint32_t v, uint32_t s, double x) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, (float)x), r, v, s, LBM_STORE_POLICY);
  }
};
template <>
struct Codec<__half, float> {
  __device__ static inline float ld(Rsrc r, uint32_t v, uint32_t s) {
    const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0);
    return __half2float(__builtin_bit_cast(__half, b));
  }
  __device__ static inline void st(Rsrc r, uint32_t v, uint32_t s, float x) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, __float2half_rn(x)),
                                          r, v, s, LBM_STORE_POLICY);
  }
};
template <>
struct Codec<__hip_bfloat16, float> {
  __device__ static inline float ld(Rsrc r, uint32_t v, uint32_t s) {
    const unsigned short b = __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0);
    return __bfloat162float(__builtin_bit_cast(__hip_bfloat16, b));
  }
  __device__ static inline void st(Rsrc r, uint32_t v, uint32_t s, float x) {
    __builtin_amdgcn_raw_buffer_store_b16(
        __builtin_bit_cast(unsigned short, __float2bfloat16(x)), r, v, s, LBM_STORE_POLICY);
  }
};

// Reference of plane q for the 16-bit storage forms: the rest equilibrium of
// a uniform state.  f: 0; h: w_q / 2; p, n: wbar_q c_ref; g: the populations of
// the uncharged linear potential of row y.
template <class R>
__device__ inline R plane_ref(int q, int y, const KP<R>& kp) {
  const R w9[9] = {R(4) / R(9), R(1) / R(9), R(1) / R(9), R(1) / R(9), R(1) / R(9),
                   R(1) / R(36), R(1) / R(36), R(1) / R(36), R(1) / R(36)};
  if (q < QH) return R(0);
  if (q < QP) return R(0.5) * w9[q - QH];
  const int k = q < QN ? q - QP : (q < QG ? q - QN : q - QG);
  const R wb = k == 0 ? R(1) / R(3) : R(1) / R(6);
  if (q < QN) return wb * kp.ref_p;
  if (q < QG) return wb * kp.ref_n;
  if (kp.walls == WALL_PERIODIC) return R(0);
  // linear potential between psi(-1/2) = dpsi and psi(ny - 1/2) = 0; the
  // population of plane q stored at row y is the post-collision value of node
  // y, i.e. the equilibrium of the linear potential there
  const R psi = kp.dpsi * (R(kp.ny) - R(0.5) - R(y)) / R(kp.ny);
  return k == 0 ? -R(2) / R(3) * psi : psi / R(6);
}

// Element `e` of a plain array, addressed as uniform base + 32-bit byte
// offset (scalar-base + vector-offset form).
template <class T>
__device__ inline T* elem(T* base, uint32_t e) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + e * (uint32_t)sizeof(T));
}
template <class T>
__device__ inline const T* elem(const T* base, uint32_t e) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + e * (uint32_t)sizeof(T));
}

// A population buffer (or the g set of one) seen through a buffer
// descriptor.  Element `off` of plane q (counted from the first plane of the
// view, population index q + qoff) lies at lattice row `yrow`.
template <class S, class R, bool DEV>
struct PopView {
  Rsrc rs;
  int qoff;
  const KP<R>* kp;
  __device__ inline R at(int q, uint32_t off, int yrow) const {
    R v = Codec<S, R>::ld(rs, off * (uint32_t)sizeof(S),
                          (uint32_t)q * kp->plane * (uint32_t)sizeof(S));
    if (DEV) v += plane_ref<R>(q + qoff, yrow, *kp);
    return v;
  }
  __device__ inline void put(int q, uint32_t off, int yrow, R v) const {
    if (DEV) v -= plane_ref<R>(q + qoff, yrow, *kp);
    Codec<S, R>::st(rs, off * (uint32_t)sizeof(S), (uint32_t)q * kp->plane * (uint32_t)sizeof(S),
                    v);
  }
};

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

template <class R>
__device__ inline R rate(int mask, int k, R inv_tau, R s_free) {
  return ((mask >> k) & 1) ? inv_tau : s_free;
}

// ---------------------------------------------------------------------------
// Macroscopic quantities of one node (Sec. 4: Eq. 5-9, 12-14, 33, 41-43, 49,
// 56-57, 59, 61).  chi9 arrays hold the node (index 0) and its eight
// neighbours x + c_i in the velocity order above.
// ---------------------------------------------------------------------------
template <class R>
struct Macro {
  R phi, psi, rho, eps, mup, mum;
  R itau_f, itau_p, itau_n;
  R gphi[2], lphi, gpsi[2], E[2];
  R cp, cm, Rr, rhoe;
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

// Cation root of Eq. (42) in a cancellation-free form (same root).
template <class R>
__device__ inline void ion_roots(R cbp, R cbm, R lam0, R* cp, R* cm) {
  const R b = R(1) - lam0 * (cbp - cbm);
  const R root = sqrt(b * b + R(4) * lam0 * cbp);
  *cp = b >= R(0) ? R(2) * cbp / (b + root) : (root - b) / (R(2) * lam0);
  *cm = *cp - cbp + cbm;
}

template <class R>
__device__ inline void macro(const R phi9[9], const R psi9[9], R P, R Q, const R f[9],
                             const KP<R>& kp, Macro<R>& m) {
  const R phi = phi9[0];
  m.phi = phi;
  m.psi = psi9[0];
  // Eq. (61)
  m.rho = phi * kp.drho + kp.rho_v;
  const R eta = phi * kp.deta + kp.eta_v;
  m.eps = phi * kp.deps + kp.eps_v;
  m.mup = phi * kp.dmu + kp.mu_v;
  m.mum = kp.m_ratio * m.mup;
  // Eq. (55), (37)
  m.itau_f = R(1) / (R(0.5) + R(3) * eta / m.rho);
  m.itau_p = R(1) / (R(0.5) + kp.three_vth * m.mup);
  m.itau_n = R(1) / (R(0.5) + kp.three_vth * m.mum);
  // Eq. (59), (9)
  grad_lap(phi9, m.gphi, &m.lphi);
  grad_lap<R>(psi9, m.gpsi, nullptr);
  m.E[0] = -m.gpsi[0];
  m.E[1] = -m.gpsi[1];
  // Eq. (5), (6), (41)-(43), (8)
  const R E2 = m.E[0] * m.E[0] + m.E[1] * m.E[1];
  if (kp.reaction) {
    const R delta = kp.q * (m.mup + m.mum) / m.eps;
    const R gamma = kp.gve / m.eps;
    const R Fo = R(1) + R(2) * gamma * sqrt(E2);
    const R lam0 = R(0.5) * delta;
    const R gen = lam0 * kp.c0sq * Fo;
    const R cbp = P + gen, cbm = Q + gen;
    ion_roots(cbp, cbm, lam0, &m.cp, &m.cm);
    m.Rr = delta * (kp.c0sq * Fo - m.cp * m.cm);
  } else {
    m.cp = P;
    m.cm = Q;
    m.Rr = R(0);
  }
  m.rhoe = kp.q * (m.cp - m.cm);
  // Eq. (12)-(14)
  const R mu_phi = kp.beta4 * phi * (phi - R(1)) * (phi - R(0.5)) - kp.kappa * m.lphi;
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
    const R inv_rho = R(1) / m.rho;
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
// Collisions (moment space).  Each writes post-collision populations.
// ---------------------------------------------------------------------------

// f: Eq. (51)-(55).
template <class R>
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
    const R s = rate(kp.mask_f, k, m.itau_f, kp.s_free);
    mo[k] = mo[k] - s * (mo[k] - eq[k]) + (R(1) - R(0.5) * s) * fo[k];
  }
  inv9(mo, f);
}

// h: Eq. (27)-(32).  dJ = d(phi u)/dt by Eq. (58).
template <class R>
__device__ inline void collide_h(R h[9], const Macro<R>& m, const R dJ[2], const KP<R>& kp) {
  R mo[9];
  fwd9(h, mo);
  const R phi = m.phi, ux = m.u[0], uy = m.u[1];
  const R third = R(1) / R(3), ninth = R(1) / R(9);
  const R gn = sqrt(m.gphi[0] * m.gphi[0] + m.gphi[1] * m.gphi[1]);
  R nx = R(0), ny = R(0);
  if (gn >= R(1e-12)) {
    nx = m.gphi[0] / gn;
    ny = m.gphi[1] / gn;
  }
  const R lam = kp.fourW * phi * (R(1) - phi);
  const R Ax = R(3) * dJ[0] + lam * nx, Ay = R(3) * dJ[1] + lam * ny;
  R eq[9], fo[9];
  eq[0] = phi;
  eq[1] = phi * ux;
  eq[2] = phi * uy;
  eq[3] = third * phi;
  eq[4] = third * phi;
  eq[5] = R(0);
  eq[6] = third * phi * ux;
  eq[7] = third * phi * uy;
  eq[8] = ninth * phi;
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
    const R s = rate(kp.mask_h, k, kp.inv_tau_h, kp.s_free);
    mo[k] = mo[k] - s * (mo[k] - eq[k]) + (R(1) - R(0.5) * s) * fo[k];
  }
  inv9(mo, h);
}

// p and n: Eq. (34)-(40) on D2Q5.  sign = -1 for cations (- S G),
// +1 for anions (+ S Gbar).
template <class R>
__device__ inline void collide_ion(R x[5], R c, R mu, R itau, int mask, R sign,
                                   const Macro<R>& m, const KP<R>& kp) {
  R mo[5];
  fwd5(x, mo);
  const R third = R(1) / R(3);
  const R Lx = kp.ion_force ? c * m.F[0] : R(0);
  const R Ly = kp.ion_force ? c * m.F[1] : R(0);
  const R Gx = mu * c * m.gpsi[0], Gy = mu * c * m.gpsi[1];
  const R eq[5] = {c, c * m.u[0], c * m.u[1], third * c, third * c};
  const R so[5] = {m.Rr, Lx, Ly, third * m.Rr, third * m.Rr};
  const R dr[5] = {R(0), Gx, Gy, R(0), R(0)};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const R s = rate(mask, k, itau, kp.s_free);
    mo[k] = mo[k] - s * (mo[k] - eq[k]) + (R(1) - R(0.5) * s) * so[k] + sign * s * dr[k];
  }
  inv5(mo, x);
}

// Poisson source S_psi of Eq. (44) (or its variable-eps form).
template <class R>
__device__ inline R poisson_source(R rhoe, R eps, const R geps[2], const R gpsi[2],
                                   const KP<R>& kp) {
  R s = rhoe;
  if (kp.poisson_form) s += geps[0] * gpsi[0] + geps[1] * gpsi[1];
  return s / eps;
}

// g: Eq. (44)-(47).
template <class R>
__device__ inline void collide_g(R g[5], R psi, R Spsi, const KP<R>& kp) {
  R mo[5];
  fwd5(g, mo);
  const R third = R(1) / R(3);
  const R eq[5] = {R(0), R(0), R(0), third * psi, third * psi};
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const R s = rate(kp.mask_g, k, kp.inv_tau_g, kp.s_free);
    mo[k] = mo[k] - s * (mo[k] - eq[k]);
  }
  inv5(mo, g);
  const R src = kp.theta_src * Spsi;
  g[0] += src / R(3);
#pragma unroll
  for (int k = 1; k < 5; ++k) g[k] += src / R(6);
}

}  // namespace lbm
