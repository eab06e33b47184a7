// lbm_ehd.hip -- host runtime and C ABI of the five-equation phase-field
// EHD lattice Boltzmann library (declarations and documentation in
// include/lbm_ehd.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm_ehd.h"
#include "lbm_ehd_aa.hpp"

using namespace lbm;

// Scratch of lbm_ehd_invariants_noalloc, which allocates nothing: the
// per-row partial sums [ny][NSUM] and their total [NSUM], for grids of up to
// NOALLOC_MAX_ROWS rows (0.9 MB).  Every GPU the library runs on holds its
// own copy until the process ends.  In host code `scratch` names a host-side
// stand-in: its device address on each GPU comes from hipGetSymbolAddress
// (noalloc_scratch) and only that address is ever passed on.
constexpr int NOALLOC_MAX_ROWS = 16384;
static __device__ __align__(256) double scratch[(NOALLOC_MAX_ROWS + 1) * NSUM];

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
  } while (0)

size_t elem_size(int prec) {
  switch (prec) {
    case LBM_FP64: return 8;
    case LBM_FP32: return 4;
    case LBM_FP32_F64: return 4;
    case LBM_FP16_STORE:
    case LBM_BF16_STORE: return 2;
    default: return 0;
  }
}
size_t arith_size(int prec) { return (prec == LBM_FP64 || prec == LBM_FP32_F64) ? 8 : 4; }
// 16-bit storage also reads and writes the line of h0 in the population
// buffers (the reference phase of the moving h, see LocalH)
bool local_h(int prec) { return elem_size(prec) == 2; }
// bytes per cell and time level of the rest populations (see RestOf and
// IonRest): h0 (FP64; 32-bit fixed point with FP32 storage), and with
// 16-bit storage also p0 and n0 (FP64)
size_t rest_bytes(int prec) {
  if (local_h(prec)) return 3 * 8;
  return elem_size(prec) == 4 ? 4 : 8;
}

int pitch_of(int nx) { return (nx + 63) / 64 * 64; }
// lines per lattice row of a population buffer: 33, a 34th with bfloat16
// storage (the second line of the reference momentum of f, see LocalF), 41
// with the ions on D2Q9 (the diagonals of both species)
int lines_of(const lbm_ehd_params& p) {
  if (p.ion_q9) return NPOP9;
  return p.precision == LBM_BF16_STORE ? NPOP + 1 : NPOP;
}
int lines_of(int prec) { return prec == LBM_BF16_STORE ? NPOP + 1 : NPOP; }

bool finite_all(std::initializer_list<double> v) {
  for (double d : v)
    if (!std::isfinite(d)) return false;
  return true;
}

}  // namespace

struct lbm_ehd {
  lbm_ehd_params P;
  int device = 0;
  hipStream_t stream = nullptr;
  void* pop[2] = {nullptr, nullptr};
  size_t pop_bytes = 0;
  void* aux = nullptr;
  size_t aux_bytes = 0;
  bool own = false;
  int cur = 0;          // buffer holding the current state
  int64_t step = 0;
  bool ready = false;   // initial state written
  int pitch = 0;
  // scratch owned by the library
  void* mom = nullptr;      // phi, psi, rho_e planes (arithmetic type), [3][ny][nx]
  double* fld = nullptr;    // [10][ny][nx]
  double* part = nullptr;   // [ny][NSUM]
  int64_t presolve_iters = 0;     // g-only sweeps of the last pre-solve
  double presolve_residual = NAN; // its convergence residual (NaN: not measured)
  double* red = nullptr;    // [NSUM]
  double* line = nullptr;   // [2 ny + 2 nx]
  double* upl = nullptr;    // uploaded initial fields [6][ny][nx]
  int tile_rows = 16;
  int waves = 1;        // wavefronts per sweep workgroup (strip of 64 * waves columns)
  // The sweep runs as a batch of one (the same kernel as lbm_ehd_batch_run,
  // so a simulation gives bitwise the same results alone and in a batch):
  // its descriptor, written with cur = desc_cur, and its tile list.
  void* d_desc = nullptr;
  BatchTile* d_tiles = nullptr;
  int ntiles = 0;
  int desc_cur = 0;
  // In-place streaming (P.inplace): the orientation of f, h, p, n (par) and
  // of g (gpar), and those the uploaded descriptor was written with.
  int par = 0, gpar = 0;
  int desc_par = 0, desc_gpar = 0;
  // g-only sweeps replayed from a captured graph (pre-solves): a block of
  // sweeps starting from the state buffer, per state buffer, captured on a
  // private stream (never the legacy default one)
  hipGraphExec_t pre_exec[2] = {nullptr, nullptr};
  hipStream_t cap = nullptr;
  // Blocks of RUN_BLOCK fused sweeps replayed from a captured graph
  // (lbm_ehd_run), one per parity of cur against desc_cur (in place: of par
  // and of gpar against the descriptor's); dropped when the launch shape
  // changes.
  hipGraphExec_t run_exec[4] = {nullptr, nullptr, nullptr, nullptr};
  // The batch this simulation belongs to (NULL: none).  A member is stepped
  // by its batch only.
  lbm_ehd_batch* batch = nullptr;
};

namespace {

// The default MRT rates: rows 3-5 of f and rows 1-2 of h, p, n, g relax
// with 1/tau, every other row with exactly 1 (s_free = 1, Sec. 6).
bool std_rates(const lbm_ehd_params& p) {
  return p.mask_f == 0x38 && p.mask_h == 0x6 && p.mask_p == 0x6 && p.mask_n == 0x6 &&
         p.mask_g == 0x6 && p.s_free == 1.0;
}

// Form of the sweep a simulation runs on, each compiled separately: 0 plain,
// 1 with side walls, 2 with side walls and the local field of Eq. (50), 3
// in-place streaming (plain), 4 plain with the ions on D2Q9, 5 side walls
// with the ions on D2Q9; all but 2 with the default MRT rates compiled in
// are NFORM higher.
constexpr int NFORM = 6;
int sweep_form(const lbm_ehd_params& p) {
  const int base = p.inplace ? 3
                 : p.ion_q9  ? (p.side_walls ? 5 : 4)
                             : (p.local_field ? 2 : (p.side_walls ? 1 : 0));
  return base + (base != 2 && std_rates(p) ? NFORM : 0);
}

// Tile list of a set of simulations: larger ones first, each band by band
// across its strips of 64 * waves columns, padded with empty tiles to a
// multiple of 8 (the sweep gives each XCD one contiguous run of tiles).
// `form` -1 takes every simulation (and never returns an empty list); 0 to
// 2 NFORM - 1 only those on that form of the sweep (possibly none).
std::vector<BatchTile> tile_list(const std::vector<const lbm_ehd*>& sims, int waves,
                                 int tile_rows, int form = -1) {
  std::vector<int> order;
  for (size_t i = 0; i < sims.size(); ++i)
    if (form < 0 || sweep_form(sims[i]->P) == form) order.push_back((int)i);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    return (long long)sims[a]->P.nx * sims[a]->P.ny > (long long)sims[c]->P.nx * sims[c]->P.ny;
  });
  const int tw = 64 * waves;
  std::vector<BatchTile> tl;
  for (int i : order) {
    const lbm_ehd_params& P = sims[i]->P;
    const int tr = std::min(tile_rows, P.ny);
    for (int y0 = 0; y0 < P.ny; y0 += tr)
      for (int x0 = 0; x0 < P.nx; x0 += tw) tl.push_back({i, x0, y0, std::min(y0 + tr, P.ny)});
  }
  while ((form < 0 && tl.empty()) || tl.size() % 8) tl.push_back({-1, 0, 0, 0});
  return tl;
}

// Offset of the +y / -y g references from psi_lin / 6: the steady
// post-collision g of the uncharged potential carries (1/s_2 - 1) G / 6 in
// the +y population and minus that in the -y one, with s_2 the rate of the
// y first moment and G = dpsi / ny the applied field.
double a_g_of(const lbm_ehd_params& p) {
  if (p.walls == LBM_PERIODIC) return 0.0;
  const double s2 = ((p.mask_g >> 2) & 1) ? 1.0 / (0.5 + 3.0 * p.theta) : p.s_free;
  return (1.0 / s2 - 1.0) * p.dpsi / p.ny / 6.0;
}

// Offsets of the ion lines stored in 16 bits: the uniform steady bulk of the
// outer phase in the applied field G = dpsi / ny (0 in a y-periodic box) has
// c_b = c0 sqrt(1 + 2 gamma_v G) (reaction on) and drifts at +mu_+ G
// (cations) and -mu_- G (anions), i.e. populations wbar_q c_b (1 +- 3 c_qy
// mu G), given as offsets from wbar_q c0.
void ion_offsets(const lbm_ehd_params& p, double out[10]) {
  const double G = p.walls == LBM_PERIODIC ? 0.0 : p.dpsi / p.ny;
  const double cb = p.reaction ? p.c0 * std::sqrt(1.0 + 2.0 * p.gamma_v * G) : p.c0;
  const double wb[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
  for (int s = 0; s < 2; ++s) {
    const double drift = s == 0 ? p.mu_v * G : -p.mu_v * p.m_ratio * G;
    for (int k = 0; k < 5; ++k) {
      const double cy = k == 2 ? 1.0 : (k == 4 ? -1.0 : 0.0);
      out[5 * s + k] = wb[k] * (cb * (1.0 + 3.0 * cy * drift) - p.c0);
    }
  }
}

template <class R>
KP<R> make_kp(const lbm_ehd* h) {
  const lbm_ehd_params& p = h->P;
  KP<R> k;
  std::memset(&k, 0, sizeof k);
  k.nx = p.nx;
  k.ny = p.ny;
  k.pitch = h->pitch;
  k.walls = p.walls;
  k.side_walls = p.side_walls;
  k.local_field = p.local_field;
  k.rstride = (uint32_t)(lines_of(p) * h->pitch);
  k.ion_q9 = p.ion_q9;
  k.cells = (uint32_t)((long long)p.ny * h->pitch);
  k.pop_bytes = (uint32_t)h->pop_bytes;
  k.reaction = p.reaction;
  k.poisson_form = p.poisson_form;
  k.flow = p.flow;
  k.ion_force = p.ion_force;
  k.mask_f = p.mask_f;
  k.mask_h = p.mask_h;
  k.mask_p = p.mask_p;
  k.mask_n = p.mask_n;
  k.mask_g = p.mask_g;
  k.rho_v = (R)p.rho_v;
  k.drho = (R)(p.rho_v * p.rho_r - p.rho_v);
  k.eta_v = (R)p.eta_v;
  k.deta = (R)(p.eta_v * p.eta_r - p.eta_v);
  k.eps_v = (R)p.eps_v;
  k.deps = (R)(p.eps_v * p.eps_r - p.eps_v);
  k.mu_v = (R)p.mu_v;
  k.dmu = (R)(p.mu_v * p.mu_r - p.mu_v);
  k.m_ratio = (R)p.m_ratio;
  k.three_vth = (R)(3.0 * p.v_th);
  k.c0 = (R)p.c0;
  k.c0sq = (R)(p.c0 * p.c0);
  k.q = (R)p.q;
  k.gve = (R)(p.gamma_v * p.eps_v);
  k.beta4 = (R)(48.0 * p.zeta / p.W);
  k.kappa = (R)(1.5 * p.zeta * p.W);
  k.W = (R)p.W;
  k.fourW = (R)(4.0 / p.W);
  k.s_free = (R)p.s_free;
  k.n_eps2 = (R)(p.n_eps * p.n_eps);
  k.inv_tau_h = (R)(1.0 / (0.5 + 3.0 * p.M_phi));
  k.inv_tau_g = (R)(1.0 / (0.5 + 3.0 * p.theta));
  k.theta_src = (R)(p.poisson_norm ? p.theta * 1.5 : p.theta);  // 1/(1 - wbar_0) = 3/2
  k.dpsi = (R)p.dpsi;
  const bool per = p.walls == LBM_PERIODIC;
  k.psi_slope = per ? (R)0 : (R)(-p.dpsi / p.ny);
  k.a_g = (R)a_g_of(p);
  double io[10];
  ion_offsets(p, io);
  for (int i = 0; i < 10; ++i) k.iofs[i] = (R)io[i];
  k.force_x = (R)p.force_x;
  k.force_y = (R)p.force_y;
  // binary16: keep the deviations of each set well inside the normal range
  // (largest magnitudes: f ~ 1, h ~ 1/4, ions ~ c0, g ~ dpsi)
  for (int i = 0; i < 5; ++i) k.sc[i] = k.isc[i] = (R)1;
  if (p.precision == LBM_FP16_STORE) {
    auto pow2_below = [](double v) { return std::ldexp(1.0, (int)std::floor(std::log2(v))); };
    const double c0 = std::max(std::fabs(p.c0), 1e-6);
    // h: the deviations from the node-local references are ~1e-3 and the
    // references themselves lie in [-1/2, 1/2]
    const double sets[5] = {4096.0, 64.0, pow2_below(4096.0 / c0), pow2_below(4096.0 / c0),
                            pow2_below(4096.0 / std::max(std::fabs(p.dpsi), 1e-3))};
    for (int i = 0; i < 5; ++i) {
      k.sc[i] = (R)sets[i];
      k.isc[i] = (R)(1.0 / sets[i]);
    }
  }
  return k;
}

// Launch helpers, one instantiation per storage form.
template <class S, class R>
struct Form {
  typedef typename RestOf<S>::type T0;
  typedef typename WorkOf<S>::type W;
  static S* buf(lbm_ehd* h, int i) { return static_cast<S*>(h->pop[i]); }
  static R* jp(lbm_ehd* h) { return static_cast<R*>(h->aux); }
  // FP64 rest populations of time level i, after the two (phi u) planes:
  // h0 (then p0, n0 with 16-bit storage), one plane each.  Like the
  // populations they ping-pong between time levels (neighbouring workgroups
  // read h0 for their phi halo).
  // In place there is one time level, which the sweep updates in place
  // (neighbours take phi' from the pre-pass planes instead).
  static T0* h0(lbm_ehd* h, int i) {
    if (h->P.inplace) i = 0;
    return reinterpret_cast<T0*>(static_cast<char*>(h->aux) +
                                 2 * (size_t)h->P.ny * h->pitch * sizeof(R)) +
           (size_t)i * rest_planes<S>() * h->P.ny * h->pitch;
  }
  // In place: the phi' and psi' planes of the pre-pass (type W), after the
  // rest population.
  static W* phiP(lbm_ehd* h) {
    return reinterpret_cast<W*>(h0(h, 0) + rest_planes<S>() * (size_t)h->P.ny * h->pitch);
  }
  static W* psiP(lbm_ehd* h) { return phiP(h) + (size_t)h->P.ny * h->pitch; }

  typedef SimDesc<S, R, T0> Desc;
  typedef SimDescAA<S, R, T0> DescAA;

  // Descriptor of an in-place simulation.
  static DescAA desc_aa(lbm_ehd* h) {
    DescAA d;
    std::memset(&d, 0, sizeof d);
    d.kp = make_kp<R>(h);
    d.kpw = make_kp<W>(h);
    d.pop = buf(h, 0);
    d.jprev = jp(h);
    d.h0 = h0(h, 0);
    d.phiP = phiP(h);
    d.psiP = psiP(h);
    d.par = h->par;
    d.gpar = h->gpar;
    return d;
  }
  // the storage types that have the in-place sweep (not bfloat16)
  static constexpr bool kAA = !LocalF<S>::value;
  // ... and the sweep with the ions on D2Q9 (4- and 8-byte storage)
  static constexpr bool kQ9 = sizeof(S) >= 4;

  // Descriptor of a simulation for the tile kernel.
  static Desc desc(lbm_ehd* h) {
    Desc d;
    std::memset(&d, 0, sizeof d);
    d.kp = make_kp<R>(h);
    d.kpw = make_kp<W>(h);
    d.pop[0] = buf(h, 0);
    d.pop[1] = buf(h, 1);
    d.jprev = jp(h);
    d.h0[0] = h0(h, 0);
    d.h0[1] = h0(h, 1);
    d.cur = h->cur;
    return d;
  }

  // Upload the simulation's descriptor and tile list (at creation and when
  // the launch shape changes; never inside a step).
  static lbm_status prepare_sweep(lbm_ehd* h) {
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (hipGraphExec_t& e : h->run_exec) {
      if (e) (void)hipGraphExecDestroy(e);
      e = nullptr;
    }
    const std::vector<BatchTile> tl = tile_list({h}, h->waves, h->tile_rows);
    (void)hipFree(h->d_tiles);
    h->d_tiles = nullptr;
    if (!h->d_desc) HIP_TRY(hipMalloc(&h->d_desc, std::max(sizeof(Desc), sizeof(DescAA))));
    HIP_TRY(hipMalloc(&h->d_tiles, tl.size() * sizeof(BatchTile)));
    if (h->P.inplace) {
      const DescAA d = desc_aa(h);
      HIP_TRY(hipMemcpy(h->d_desc, &d, sizeof d, hipMemcpyHostToDevice));
    } else {
      const Desc d = desc(h);
      HIP_TRY(hipMemcpy(h->d_desc, &d, sizeof d, hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(h->d_tiles, tl.data(), tl.size() * sizeof(BatchTile),
                      hipMemcpyHostToDevice));
    h->ntiles = (int)tl.size();
    h->desc_cur = h->cur;
    h->desc_par = h->par;
    h->desc_gpar = h->gpar;
    return LBM_OK;
  }

  template <int NW, int EXT, bool STD>
  static void launch_nw(const void* descs, const BatchTile* tiles, int ntiles, int flip,
                        hipStream_t st) {
    hipLaunchKernelGGL((k_sweep_batch<S, R, T0, NW, EXT, STD>), dim3(ntiles), dim3(64 * NW), 0,
                       st, static_cast<const Desc*>(descs), tiles, ntiles / 8, flip);
  }

  template <int EXT, bool STD = false>
  static void launch_ext(int waves, const void* descs, const BatchTile* tiles, int ntiles,
                        int flip, hipStream_t st) {
    switch (waves) {
      case 8: launch_nw<8, EXT, STD>(descs, tiles, ntiles, flip, st); break;
      case 4: launch_nw<4, EXT, STD>(descs, tiles, ntiles, flip, st); break;
      case 2: launch_nw<2, EXT, STD>(descs, tiles, ntiles, flip, st); break;
      default: launch_nw<1, EXT, STD>(descs, tiles, ntiles, flip, st); break;
    }
  }

  // One fused sweep over the tiles `tiles` (a multiple of 8) of the members
  // described by `descs`, all on sweep form `form`; `flip` = 1 swaps every
  // member's buffers.
  static lbm_status launch_tiles(int waves, int form, const void* descs,
                                 const BatchTile* tiles, int ntiles, int flip, hipStream_t st) {
    switch (form) {
      case 4:
      case 4 + NFORM:
      case 5:
      case 5 + NFORM:
        if constexpr (kQ9) {
          if (form == 4)
            launch_ext<3>(waves, descs, tiles, ntiles, flip, st);
          else if (form == 4 + NFORM)
            launch_ext<3, true>(waves, descs, tiles, ntiles, flip, st);
          else if (form == 5)
            launch_ext<4>(waves, descs, tiles, ntiles, flip, st);
          else
            launch_ext<4, true>(waves, descs, tiles, ntiles, flip, st);
        }
        break;
      case 2: launch_ext<2>(waves, descs, tiles, ntiles, flip, st); break;
      case 1: launch_ext<1>(waves, descs, tiles, ntiles, flip, st); break;
      case 1 + NFORM: launch_ext<1, true>(waves, descs, tiles, ntiles, flip, st); break;
      case NFORM: launch_ext<0, true>(waves, descs, tiles, ntiles, flip, st); break;
      default: launch_ext<0>(waves, descs, tiles, ntiles, flip, st); break;
    }
    HIP_TRY(hipGetLastError());
    return LBM_OK;
  }

  // One in-place step over the tiles `tiles` of the members described by
  // `descs` (DescAA): the phi'/psi' pre-pass, then the sweep.  `flip` /
  // `gflip` = 1 turns every member's orientation of f, h, p, n / of g.
  template <int NW, bool STD>
  static void launch_aa_nw(const void* descs, const BatchTile* tiles, int ntiles, int flip,
                           int gflip, hipStream_t st) {
    if constexpr (kAA) {
      hipLaunchKernelGGL((k_aa_hood<S, R, T0, NW>), dim3(ntiles), dim3(64 * NW), 0, st,
                         static_cast<const DescAA*>(descs), tiles, ntiles / 8, flip, gflip);
      hipLaunchKernelGGL((k_sweep_aa<S, R, T0, NW, STD>), dim3(ntiles), dim3(64 * NW), 0, st,
                         static_cast<const DescAA*>(descs), tiles, ntiles / 8, flip, gflip);
    }
  }
  template <bool STD>
  static void launch_aa_std(int waves, const void* descs, const BatchTile* tiles, int ntiles,
                            int flip, int gflip, hipStream_t st) {
    switch (waves) {
      case 8: launch_aa_nw<8, STD>(descs, tiles, ntiles, flip, gflip, st); break;
      case 4: launch_aa_nw<4, STD>(descs, tiles, ntiles, flip, gflip, st); break;
      case 2: launch_aa_nw<2, STD>(descs, tiles, ntiles, flip, gflip, st); break;
      default: launch_aa_nw<1, STD>(descs, tiles, ntiles, flip, gflip, st); break;
    }
  }
  // `std`: the members have the default MRT rates (sweep form 3 + NFORM)
  static lbm_status launch_aa(int waves, bool std, const void* descs, const BatchTile* tiles,
                              int ntiles, int flip, int gflip, hipStream_t st) {
    if (!kAA) return fail(LBM_EINVAL, "in-place streaming needs FP64, FP32 or FP16 storage");
    if (std)
      launch_aa_std<true>(waves, descs, tiles, ntiles, flip, gflip, st);
    else
      launch_aa_std<false>(waves, descs, tiles, ntiles, flip, gflip, st);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
  }

  static lbm_status sweep(lbm_ehd* h) {
    if (h->P.inplace) {
      lbm_status st = launch_aa(h->waves, std_rates(h->P), h->d_desc, h->d_tiles, h->ntiles,
                                h->par ^ h->desc_par, h->gpar ^ h->desc_gpar, h->stream);
      if (st) return st;
      h->par ^= 1;
      h->gpar ^= 1;
      return LBM_OK;
    }
    lbm_status st = launch_tiles(h->waves, sweep_form(h->P), h->d_desc, h->d_tiles,
                                 h->ntiles, h->cur ^ h->desc_cur, h->stream);
    if (st) return st;
    h->cur = 1 - h->cur;
    return LBM_OK;
  }

  static dim3 grid2(const lbm_ehd* h) { return dim3((h->P.nx + 63) / 64, h->P.ny); }

  // phi', psi', rho_e planes in type RF (R for the Poisson sweeps, the wide
  // type T0 for readback).  Scratch is allocated on first use (room for
  // FP64 planes): a simulation that only steps holds its state and nothing
  // else.
  // `gsrc` is the buffer holding the current g set (NULL: the state buffer).
  template <class RF>
  static lbm_status moments_as(lbm_ehd* h, const S* gsrc) {
    if (!h->mom) HIP_TRY(hipMalloc(&h->mom, 3 * (size_t)h->P.nx * h->P.ny * sizeof(double)));
    const KP<RF> kp = make_kp<RF>(h);
    const S* src = buf(h, h->cur);
    if (!gsrc) gsrc = src;
    hipLaunchKernelGGL((k_moments<S, RF, T0>), grid2(h), dim3(64), 0, h->stream, src, gsrc,
                       h0(h, h->cur), static_cast<RF*>(h->mom), kp);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
  }
  static lbm_status moments(lbm_ehd* h, const S* gsrc) { return moments_as<R>(h, gsrc); }

  // One g-only sweep on stream `st`: the moment planes of the state with g
  // from `from` (all of phi', psi', rho_e if `full`, else psi' alone: phi and
  // rho_e do not change in g-only sweeps), then g from `from` into `to`.
  static lbm_status g_sweep(lbm_ehd* h, const S* from, S* to, hipStream_t st, bool full) {
    const KP<R> kp = make_kp<R>(h);
    if (full)
      hipLaunchKernelGGL((k_moments<S, R, T0>), grid2(h), dim3(64), 0, st, buf(h, h->cur), from,
                         h0(h, h->cur), static_cast<R*>(h->mom), kp);
    else
      hipLaunchKernelGGL((k_psi_plane<S, R>), grid2(h), dim3(64), 0, st, from,
                         static_cast<R*>(h->mom), kp);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL((k_poisson<S, R>), grid2(h), dim3(64), 0, st, from, to,
                       static_cast<const R*>(h->mom), kp);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
  }

  // `n` g-only sweeps from the g in `from`, which is left pointing at the
  // buffer holding the latest g.  The g set (its five lines and, with 16-bit
  // storage, the line of its reference potential) ping-pongs between the
  // state buffer and the same lines of the other buffer, which the next
  // sweep overwrites anyway.  Each sweep is two small kernels, launch-bound
  // on small grids (3-4 us per launch at 256^2), so from the state buffer
  // whole blocks of PRE_BLOCK sweeps (even: a block ends in the buffer it
  // started from) are replayed from a graph captured once per state buffer.
  static constexpr int PRE_BLOCK = 64;
  static lbm_status g_sweeps(lbm_ehd* h, const S*& from, int n) {
    S* A = buf(h, h->cur);
    S* B = buf(h, 1 - h->cur);
    if (!h->mom) HIP_TRY(hipMalloc(&h->mom, 3 * (size_t)h->P.nx * h->P.ny * sizeof(double)));
    // the first sweep refreshes every moment plane, the later ones psi' alone
    for (int first = 0; first < 2 && n > 0; ++first, --n) {
      S* to = from == A ? B : A;
      lbm_status st = g_sweep(h, from, to, h->stream, first == 0);
      if (st) return st;
      from = to;
    }
    if (from == A && n >= 2 * PRE_BLOCK) {
      hipGraphExec_t& exec = h->pre_exec[h->cur];
      if (!exec) {
        if (!h->cap) HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
        const S* f = A;
        lbm_status cst = LBM_OK;
        for (int i = 0; i < PRE_BLOCK && !cst; ++i) {
          S* to = f == A ? B : A;
          cst = g_sweep(h, f, to, h->cap, false);
          f = to;
        }
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(h->cap, &g);
        if (!cst && e == hipSuccess) {
          const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
          if (ie != hipSuccess) {
            exec = nullptr;
            cst = fail(LBM_EDEVICE, std::string("graph instantiation: ") + hipGetErrorString(ie));
          }
        } else if (!cst) {
          cst = fail(LBM_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        }
        if (g) (void)hipGraphDestroy(g);
        if (cst) return cst;
      }
      for (; n >= PRE_BLOCK; n -= PRE_BLOCK) HIP_TRY(hipGraphLaunch(exec, h->stream));
    }
    for (int it = 0; it < n; ++it) {
      S* to = from == A ? B : A;
      lbm_status st = g_sweep(h, from, to, h->stream, false);
      if (st) return st;
      from = to;
    }
    return LBM_OK;
  }

  // `iters` g-only sweeps from the state; returns (in *gsrc) the buffer
  // holding the latest g.
  static lbm_status poisson(lbm_ehd* h, int iters, const S** gsrc) {
    const S* from = buf(h, h->cur);
    lbm_status st = g_sweeps(h, from, iters);
    *gsrc = from;
    return st;
  }

  // Bring the latest g back into the state buffer: the five g lines of
  // every row, and the reference line with 16-bit storage.
  static lbm_status settle_g(lbm_ehd* h, const S* gsrc) {
    S* A = buf(h, h->cur);
    if (gsrc != A) {
      const size_t row = (size_t)lines_of(h->P) * h->pitch * sizeof(S);
      const size_t line = (size_t)h->pitch;
      HIP_TRY(hipMemcpy2DAsync(A + QG * line, row, gsrc + QG * line, row,
                               5 * line * sizeof(S), (size_t)h->P.ny + 2,
                               hipMemcpyDeviceToDevice, h->stream));
      if (LocalG<S>::value)
        HIP_TRY(hipMemcpy2DAsync(A + QRG * line, row, gsrc + QRG * line, row, line * sizeof(S),
                                 (size_t)h->P.ny + 2, hipMemcpyDeviceToDevice, h->stream));
    }
    return LBM_OK;
  }

  static lbm_status step(lbm_ehd* h) {
    if (h->P.poisson_tol > 0) {
      // converged-Poisson mode: g-only sweeps to the tolerance first
      int done = 0;
      double r = NAN;
      lbm_status st = presolve_to(h, h->P.poisson_tol, h->P.poisson_max, h->P.poisson_iters,
                                  &done, &r);
      if (st) return st;
      h->presolve_iters = done;
      h->presolve_residual = r;
    } else if (h->P.poisson_iters > 0) {
      if (h->P.inplace) {
        lbm_status st = g_sweeps_aa(h, h->P.poisson_iters);
        if (st) return st;
        return sweep(h);
      }
      const S* g = nullptr;
      lbm_status st = poisson(h, h->P.poisson_iters, &g);
      if (st) return st;
      st = settle_g(h, g);
      if (st) return st;
    }
    return sweep(h);
  }

  // `n` g-only sweeps in place (phi and rho_e held fixed), each turning the
  // orientation of g.  The first refreshes every moment plane, the later ones
  // psi' alone.
  static lbm_status g_sweeps_aa(lbm_ehd* h, int n) {
    if constexpr (kAA) {
      if (!h->mom) HIP_TRY(hipMalloc(&h->mom, 3 * (size_t)h->P.nx * h->P.ny * sizeof(double)));
      const KP<R> kp = make_kp<R>(h);
      S* A = buf(h, 0);
      R* mom = static_cast<R*>(h->mom);
      for (int it = 0; it < n; ++it) {
        if (it == 0)
          hipLaunchKernelGGL((k_aa_moments<S, R, T0>), grid2(h), dim3(64), 0, h->stream, A,
                             h0(h, 0), mom, kp, h->par, h->gpar);
        else
          hipLaunchKernelGGL((k_aa_psi_plane<S, R>), grid2(h), dim3(64), 0, h->stream, A, mom,
                             kp, h->gpar);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL((k_aa_poisson<S, R>), grid2(h), dim3(64), 0, h->stream, A, mom, kp,
                           h->gpar);
        HIP_TRY(hipGetLastError());
        h->gpar ^= 1;
      }
      return LBM_OK;
    }
    return fail(LBM_EINVAL, "in-place streaming needs FP64, FP32 or FP16 storage");
  }

  // `n` time steps.  Steps without extra g-only sweeps are fused sweeps
  // alone: whole blocks of RUN_BLOCK of them (even, so a block ends in the
  // buffer it started from) are replayed from a graph captured once per
  // parity of the state buffer; on small grids a step is a few microseconds
  // of kernel and launch-bound otherwise.
  static constexpr int RUN_BLOCK = 16;
  static lbm_status steps(lbm_ehd* h, int64_t n) {
    if (h->P.poisson_tol > 0 || h->P.poisson_iters > 0) {
      for (int64_t i = 0; i < n; ++i) {
        lbm_status st = step(h);
        if (st) return st;
      }
      return LBM_OK;
    }
    if (n >= RUN_BLOCK) {
      const bool aa = h->P.inplace;
      const int par = aa ? h->par ^ h->desc_par : h->cur ^ h->desc_cur;
      const int gpar = aa ? h->gpar ^ h->desc_gpar : 0;
      hipGraphExec_t& exec = h->run_exec[par | (gpar << 1)];
      if (!exec) {
        // captured (not run) on a private stream: the handle's stream may be
        // the legacy default one, which cannot be captured
        if (!h->cap) HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
        lbm_status cst = LBM_OK;
        for (int i = 0; i < RUN_BLOCK && !cst; ++i)
          cst = aa ? launch_aa(h->waves, std_rates(h->P), h->d_desc, h->d_tiles, h->ntiles,
                               par ^ (i & 1), gpar ^ (i & 1), h->cap)
                   : launch_tiles(h->waves, sweep_form(h->P), h->d_desc, h->d_tiles,
                                  h->ntiles, par ^ (i & 1), h->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(h->cap, &g);
        if (!cst && e == hipSuccess) {
          const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
          if (ie != hipSuccess) {
            exec = nullptr;
            cst = fail(LBM_EDEVICE, std::string("graph instantiation: ") + hipGetErrorString(ie));
          }
        } else if (!cst) {
          cst = fail(LBM_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        }
        if (g) (void)hipGraphDestroy(g);
        if (cst) return cst;
      }
      for (; n >= RUN_BLOCK; n -= RUN_BLOCK) HIP_TRY(hipGraphLaunch(exec, h->stream));
    }
    for (int64_t i = 0; i < n; ++i) {
      lbm_status st = sweep(h);
      if (st) return st;
    }
    return LBM_OK;
  }

  static lbm_status presolve(lbm_ehd* h, int iters) {
    if (h->P.inplace) return g_sweeps_aa(h, iters);
    const S* g = nullptr;
    lbm_status st = poisson(h, iters, &g);
    if (st) return st;
    return settle_g(h, g);
  }

  static lbm_status init(lbm_ehd* h, const InitSpec& sp) {
    const KP<R> kp = make_kp<R>(h);
    h->cur = 0;
    h->par = h->gpar = 0;
    if (h->P.inplace) {
      if constexpr (kAA)
        hipLaunchKernelGGL((k_init<S, R, T0, true>), grid2(h), dim3(64), 0, h->stream, buf(h, 0),
                           jp(h), h0(h, 0), kp, sp);
    } else {
      hipLaunchKernelGGL((k_init<S, R, T0>), grid2(h), dim3(64), 0, h->stream, buf(h, 0), jp(h),
                         h0(h, 0), kp, sp);
    }
    HIP_TRY(hipGetLastError());
    return LBM_OK;
  }

  // Readback in the working type W (FP64 for FP32 and FP64 storage): the
  // derived fields (u, p, E, ...) are formed from the stored state without
  // adding FP32 rounding of their own.
  static lbm_status fields(lbm_ehd* h) {
    if (h->P.inplace) {
      if constexpr (kAA) {
        if (!h->mom) HIP_TRY(hipMalloc(&h->mom, 3 * (size_t)h->P.nx * h->P.ny * sizeof(double)));
        if (!h->fld)
          HIP_TRY(hipMalloc(&h->fld, 10 * (size_t)h->P.nx * h->P.ny * sizeof(double)));
        const KP<W> kpw = make_kp<W>(h);
        hipLaunchKernelGGL((k_aa_moments<S, W, T0>), grid2(h), dim3(64), 0, h->stream,
                           buf(h, 0), h0(h, 0), static_cast<W*>(h->mom), kpw, h->par, h->gpar);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL((k_aa_fields<S, W, T0>), grid2(h), dim3(64), 0, h->stream, buf(h, 0),
                           h0(h, 0), static_cast<const W*>(h->mom), h->fld, kpw, h->par);
        HIP_TRY(hipGetLastError());
      }
      return LBM_OK;
    }
    lbm_status st = moments_as<W>(h, nullptr);
    if (st) return st;
    if (!h->fld) HIP_TRY(hipMalloc(&h->fld, 10 * (size_t)h->P.nx * h->P.ny * sizeof(double)));
    const KP<W> kp = make_kp<W>(h);
    const S* src = buf(h, h->cur);
    hipLaunchKernelGGL((k_fields<S, W, T0>), grid2(h), dim3(64), 0, h->stream, src,
                       h0(h, h->cur), static_cast<const W*>(h->mom), h->fld, kp);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
  }

  // FP64 sums of the current state: per-row partials into `part` [ny][NSUM],
  // their column sums in row order into `red` [NSUM].
  static lbm_status sums_into(lbm_ehd* h, double* part, double* red) {
    const KP<R> kp = make_kp<R>(h);
    const S* src = buf(h, h->cur);
    if (h->P.inplace) {
      if constexpr (kAA)
        hipLaunchKernelGGL((k_aa_row_sums<S, R, T0>), dim3(h->P.ny), dim3(256), 0, h->stream,
                           src, h0(h, 0), part, kp, h->par, h->gpar);
    } else {
      hipLaunchKernelGGL((k_row_sums<S, R, T0>), dim3(h->P.ny), dim3(256), 0, h->stream, src,
                         h0(h, h->cur), part, kp);
    }
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_sum_rows, dim3(NSUM), dim3(256), 0, h->stream, part, h->P.ny, NSUM, red);
    HIP_TRY(hipGetLastError());
    return LBM_OK;
  }

  // g-only sweeps until the convergence residual falls below tol (checked
  // every `every` sweeps) or max_iters sweeps are done.  The residual is the
  // FP64 relative change of psi over the last sweep, ||psi_k+1 - psi_k|| /
  // ||psi_k+1||, divided by the per-sweep decay rate of the slowest mode of
  // the Poisson LBE (a diffusion with coefficient theta between electrodes a
  // distance ny apart: pi^2 theta / ny^2), which estimates the distance to
  // the converged potential.  Both g sets are at hand: the sweeps ping-pong
  // between the buffers, so the other one holds the sweep before.
  static lbm_status presolve_to(lbm_ehd* h, double tol, int max_iters, int every, int* done,
                                double* residual) {
    const KP<W> kpw = make_kp<W>(h);
    S* A = buf(h, h->cur);
    S* B = buf(h, 1 - h->cur);
    const S* from = A;
    const double theta = h->P.theta > 0 ? h->P.theta : 0.3;
    const double rate = M_PI * M_PI * theta / ((double)h->P.ny * h->P.ny);
    int k = 0;
    double r = NAN;
    while (k < max_iters) {
      const int n = std::min(every, max_iters - k);
      lbm_status st = g_sweeps(h, from, n);
      if (st) return st;
      k += n;
      const S* older = from == A ? B : A;
      hipLaunchKernelGGL((k_psi_change_rows<S, W>), dim3(h->P.ny), dim3(256), 0, h->stream,
                         from, older, h->part, kpw);
      HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL(k_sum_rows, dim3(2), dim3(256), 0, h->stream, h->part, h->P.ny, 2,
                         h->red);
      HIP_TRY(hipGetLastError());
      double sums[2];
      HIP_TRY(hipMemcpyAsync(sums, h->red, sizeof sums, hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(hipStreamSynchronize(h->stream));
      // (checked before the ratio: a NaN sum would fail `sums[1] > 0` and read
      // as a converged potential)
      if (!std::isfinite(sums[0]) || !std::isfinite(sums[1]))
        return fail(LBM_ENONFINITE, "potential contains NaN or Inf");
      r = sums[1] > 0 ? std::sqrt(sums[0] / sums[1]) / rate : 0.0;
      if (!std::isfinite(r)) return fail(LBM_ENONFINITE, "potential contains NaN or Inf");
      if (r < tol) break;
    }
    lbm_status st = settle_g(h, from);
    if (st) return st;
    *done = k;
    *residual = r;
    return LBM_OK;
  }
};

// ---------------------------------------------------------------------------
// Batched sweeps: several simulations advanced by one launch per step over the
// tiles of all members (k_sweep_batch).
// ---------------------------------------------------------------------------
}  // namespace

struct lbm_ehd_batch {
  std::vector<lbm_ehd*> sims;
  int precision = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;        // created by the library (graphs need a stream other
                                  // than the legacy default one)
  int waves = 2, tile_rows = 8;
  int graph_steps = 16;           // steps per captured block (even)
  // device copies of the member descriptors and of the tile list
  void* d_desc = nullptr;
  size_t desc_cap = 0;            // bytes
  void* h_desc = nullptr;         // pinned staging of the descriptors
  BatchTile* d_tiles = nullptr;
  size_t tiles_cap = 0;           // tiles
  BatchTile* h_tiles = nullptr;   // pinned staging of the tile list
  int ntiles[2 * NFORM] = {};  // tiles of the members on each sweep form, in the order of
                               // the forms (each padded to a multiple of 8)
  // descriptors of the in-place members (form 3), indexed like the members
  void* d_aadesc = nullptr;
  size_t aadesc_cap = 0;          // bytes
  void* h_aadesc = nullptr;
  bool dirty = true;              // descriptors / tiles / graph must be rebuilt
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

template <class S, class R>
struct BatchForm {
  typedef Form<S, R> F;
  typedef typename F::Desc Desc;

  // Descriptors and tile list of the current members and launch shape.
  static lbm_status rebuild(lbm_ehd_batch* b) {
    HIP_TRY(hipStreamSynchronize(b->stream));  // staging buffers may still be in use
    const size_t n = b->sims.size();
    const size_t dbytes = std::max<size_t>(1, n) * sizeof(Desc);
    if (dbytes > b->desc_cap) {
      (void)hipFree(b->d_desc);
      (void)hipHostFree(b->h_desc);
      b->d_desc = b->h_desc = nullptr;
      b->desc_cap = 0;
      HIP_TRY(hipMalloc(&b->d_desc, dbytes));
      HIP_TRY(hipHostMalloc(&b->h_desc, dbytes, hipHostMallocDefault));
      b->desc_cap = dbytes;
    }
    Desc* hd = static_cast<Desc*>(b->h_desc);
    bool any_aa = false;
    for (size_t i = 0; i < n; ++i) {
      hd[i] = F::desc(b->sims[i]);
      any_aa = any_aa || b->sims[i]->P.inplace;
    }
    if (any_aa) {
      const size_t abytes = n * sizeof(typename F::DescAA);
      if (abytes > b->aadesc_cap) {
        (void)hipFree(b->d_aadesc);
        (void)hipHostFree(b->h_aadesc);
        b->d_aadesc = b->h_aadesc = nullptr;
        b->aadesc_cap = 0;
        HIP_TRY(hipMalloc(&b->d_aadesc, abytes));
        HIP_TRY(hipHostMalloc(&b->h_aadesc, abytes, hipHostMallocDefault));
        b->aadesc_cap = abytes;
      }
      typename F::DescAA* ha = static_cast<typename F::DescAA*>(b->h_aadesc);
      for (size_t i = 0; i < n; ++i)
        if (b->sims[i]->P.inplace) ha[i] = F::desc_aa(b->sims[i]);
      HIP_TRY(hipMemcpyAsync(b->d_aadesc, b->h_aadesc, abytes, hipMemcpyHostToDevice,
                             b->stream));
    }
    // members on each form of the sweep get a launch of their own, so that
    // every member runs the code it runs alone (bitwise the same results)
    const std::vector<const lbm_ehd*> ms(b->sims.begin(), b->sims.end());
    std::vector<BatchTile> tl;
    for (int form = 0; form < 2 * NFORM; ++form) {
      const std::vector<BatchTile> t = tile_list(ms, b->waves, b->tile_rows, form);
      b->ntiles[form] = (int)t.size();
      tl.insert(tl.end(), t.begin(), t.end());
    }
    if (tl.empty()) tl.push_back({-1, 0, 0, 0});
    if (tl.size() > b->tiles_cap) {
      (void)hipFree(b->d_tiles);
      (void)hipHostFree(b->h_tiles);
      b->d_tiles = b->h_tiles = nullptr;
      b->tiles_cap = 0;
      HIP_TRY(hipMalloc(&b->d_tiles, tl.size() * sizeof(BatchTile)));
      HIP_TRY(hipHostMalloc(&b->h_tiles, tl.size() * sizeof(BatchTile), hipHostMallocDefault));
      b->tiles_cap = tl.size();
    }
    std::copy(tl.begin(), tl.end(), b->h_tiles);
    HIP_TRY(hipMemcpyAsync(b->d_desc, b->h_desc, n * sizeof(Desc), hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(hipMemcpyAsync(b->d_tiles, b->h_tiles, tl.size() * sizeof(BatchTile),
                           hipMemcpyHostToDevice, b->stream));
    return LBM_OK;
  }

  static lbm_status launch(lbm_ehd_batch* b, int flip) {
    int first = 0;
    for (int form = 0; form < 2 * NFORM; ++form) {
      if (b->ntiles[form] > 0) {
        const lbm_status st =
            form % NFORM == 3
                ? F::launch_aa(b->waves, form >= NFORM, b->d_aadesc, b->d_tiles + first,
                               b->ntiles[form],
                                     flip, flip, b->stream)
                      : F::launch_tiles(b->waves, form, b->d_desc, b->d_tiles + first,
                                        b->ntiles[form], flip, b->stream);
        if (st) return st;
      }
      first += b->ntiles[form];
    }
    return LBM_OK;
  }
};

template <class F>
lbm_status dispatch_prec(int precision, F&& fn) {
  switch (precision) {
    case LBM_FP64: return fn(BatchForm<double, double>{});
    case LBM_FP32: return fn(BatchForm<float, float>{});
    case LBM_FP32_F64: return fn(BatchForm<float, double>{});
    case LBM_FP16_STORE: return fn(BatchForm<__half, float>{});
    case LBM_BF16_STORE: return fn(BatchForm<__hip_bfloat16, float>{});
  }
  return fail(LBM_EINVAL, "unknown precision");
}

template <class F>
lbm_status dispatch(lbm_ehd* h, F&& fn) {
  switch (h->P.precision) {
    case LBM_FP64: return fn(Form<double, double>{});
    case LBM_FP32: return fn(Form<float, float>{});
    case LBM_FP32_F64: return fn(Form<float, double>{});
    case LBM_FP16_STORE: return fn(Form<__half, float>{});
    case LBM_BF16_STORE: return fn(Form<__hip_bfloat16, float>{});
  }
  return fail(LBM_EINVAL, "unknown precision");
}

lbm_status validate(const lbm_ehd_params* p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->nx < 2 || p->ny < 2) return fail(LBM_EINVAL, "nx and ny must be >= 2");
  if ((long long)p->nx * p->ny > (1LL << 31)) return fail(LBM_EINVAL, "grid too large");
  // the helper kernels launch one row of workgroups per lattice row
  if (p->ny > 65536) return fail(LBM_EINVAL, "ny must be at most 65536");
  if (!elem_size(p->precision)) return fail(LBM_EINVAL, "unknown precision");
  // kernels address a population buffer with 32-bit byte offsets
  if ((double)lines_of(*p) * (p->ny + 2) * pitch_of(p->nx) * elem_size(p->precision) >=
      4294967296.0)
    return fail(LBM_EINVAL, "grid too large: a population buffer must stay below 4 GiB");
  if (p->walls < 0 || p->walls > 2) return fail(LBM_EINVAL, "unknown walls");
  if (p->side_walls != 0 && p->side_walls != 1) return fail(LBM_EINVAL, "side_walls: 0 or 1");
  if (p->local_field != 0 && p->local_field != 1) return fail(LBM_EINVAL, "local_field: 0 or 1");
  if (!(p->poisson_tol >= 0)) return fail(LBM_EINVAL, "poisson_tol must be >= 0");
  if (p->poisson_tol > 0 && (p->poisson_iters < 1 || p->poisson_max < 1))
    return fail(LBM_EINVAL, "poisson_tol > 0 needs poisson_iters >= 1 and poisson_max >= 1");
  if (p->poisson_iters < 0) return fail(LBM_EINVAL, "poisson_iters < 0");
  if (p->diag_every < 0) return fail(LBM_EINVAL, "diag_every < 0");
  if (p->inplace != 0 && p->inplace != 1) return fail(LBM_EINVAL, "inplace: 0 or 1");
  if (p->ion_q9 != 0 && p->ion_q9 != 1) return fail(LBM_EINVAL, "ion_q9: 0 or 1");
  if (p->ion_q9 && (elem_size(p->precision) == 2 || p->local_field || p->inplace))
    return fail(LBM_EINVAL,
                "ions on D2Q9: FP64 or FP32 storage, two buffers, no local field");
  if (p->inplace && p->precision == LBM_BF16_STORE)
    return fail(LBM_EINVAL, "in-place streaming needs FP64, FP32 or FP16 storage");
  if (p->inplace && (p->side_walls || p->local_field || p->poisson_tol > 0))
    return fail(LBM_EINVAL,
                "in-place streaming covers the plain sweep: no side walls, no local field, "
                "no converged-Poisson mode");
  if (!finite_all({p->rho_v, p->rho_r, p->eta_v, p->eta_r, p->M_phi, p->W, p->zeta, p->theta,
                   p->dpsi, p->eps_v, p->eps_r, p->mu_v, p->mu_r, p->m_ratio, p->v_th, p->c0,
                   p->q, p->gamma_v, p->force_x, p->force_y, p->s_free, p->n_eps}))
    return fail(LBM_EINVAL, "non-finite coefficient");
  if (p->rho_v <= 0 || p->rho_r <= 0 || p->eps_v <= 0 || p->eps_r <= 0 || p->W <= 0)
    return fail(LBM_EINVAL, "density, permittivity and W must be positive");
  if (p->s_free <= 0 || p->s_free >= 2) return fail(LBM_EINVAL, "s_free must lie in (0, 2)");
  if (p->n_eps < 0) return fail(LBM_EINVAL, "n_eps must be >= 0");
  // every relaxation time > 1/2 for phi in [0, 1] (the properties are linear)
  for (double phi : {0.0, 1.0}) {
    const double rho = p->rho_v + phi * (p->rho_v * p->rho_r - p->rho_v);
    const double eta = p->eta_v + phi * (p->eta_v * p->eta_r - p->eta_v);
    const double mu = p->mu_v + phi * (p->mu_v * p->mu_r - p->mu_v);
    if (p->flow && !(eta / rho > 0)) return fail(LBM_EINVAL, "tau_f <= 1/2");
    if (!(p->v_th * mu > 0) || !(p->v_th * mu * p->m_ratio > 0))
      return fail(LBM_EINVAL, "tau_+ or tau_- <= 1/2 (v_th mu must be > 0)");
    if (!(p->eps_v + phi * (p->eps_v * p->eps_r - p->eps_v) > 0))
      return fail(LBM_EINVAL, "permittivity <= 0");
  }
  if (!(p->M_phi > 0)) return fail(LBM_EINVAL, "tau_h <= 1/2 (M_phi must be > 0)");
  if (!(p->theta > 0)) return fail(LBM_EINVAL, "tau_g <= 1/2 (theta must be > 0)");
  return LBM_OK;
}

void free_scratch(lbm_ehd* h) {
  for (hipGraphExec_t& e : h->pre_exec)
    if (e) (void)hipGraphExecDestroy(e);
  for (hipGraphExec_t& e : h->run_exec)
    if (e) (void)hipGraphExecDestroy(e);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  (void)hipFree(h->d_desc);
  (void)hipFree(h->d_tiles);
  (void)hipFree(h->mom);
  (void)hipFree(h->fld);
  (void)hipFree(h->part);
  (void)hipFree(h->red);
  (void)hipFree(h->line);
  (void)hipFree(h->upl);
  if (h->own) {
    (void)hipFree(h->pop[0]);
    (void)hipFree(h->pop[1]);
    (void)hipFree(h->aux);
  }
}

// Default launch shape of the sweep for a grid.  Strips are 64 columns per
// wave: one wave on grids narrower than 512 columns, four waves (256
// columns) on wider ones, eight (512) where eight-wave workgroups fit twice
// on a CU
// (FP32 arithmetic, or FP32 storage with its pulls parked in LDS as FP32 in
// the plain two-buffer sweep with the default MRT rates; the other forms
// take more than 128 registers with FP64 arithmetic, three waves per SIMD).
// Bands are the tallest (the h and g rows just outside a band are read
// twice) that still put four wavefronts per SIMD in flight (4096 on the 256
// CUs), eight per SIMD with FP32 storage.  Measured on
// MI355X at 2048^2 (GLUPS; waves x rows per band): FP32 20.1 (8 x 8), 19.9
// (8 x 16), 19.9 (4 x 8), 19.6 (4 x 4), 19.3 (8 x 4), 17.4 (2 x 8); FP32
// storage with FP64 arithmetic 19.6 (8 x 8), 19.4 (8 x 16), 19.3 (4 x 8),
// 19.0 (4 x 16), in place 17.1 (4 x 8), 17.0 (8 x 8), 17.0 (4 x 16); FP16
// 26.5 (8 x 16), 25.9 (8 x 8), 24.5 (4 x 16), 20.0 (4 x 32); BF16 25.9
// (8 x 16), 25.1 (8 x 8), 23.1 (4 x 16); FP64 10.8 (4 x 16), 10.8 (8 x 16),
// 10.7 (4 x 8), 10.6 (8 x 8).  On narrow grids many small tiles fill the
// chip first (MLUPS at 256^2, FP32 / FP16 / FP64: 5158 / 5080 / 4923 with
// (1 x 2) against 4908 / 5057 / 4541 with (4 x 2); at 128^2 1378 / 1399 /
// 1544 against 1335 / 1348 / 1438 with (2 x 2)).
void default_launch(const lbm_ehd_params* p, int* waves, int* tile_rows) {
  *waves = p->nx >= 512 ? 4 : 1;
  const bool fp32_store = elem_size(p->precision) == 4;
  if (p->nx >= 512 && (arith_size(p->precision) == 4 || (fp32_store && sweep_form(*p) == NFORM)))
    *waves = 8;
  const long long strips = (p->nx + 64 * *waves - 1) / (64 * *waves);
  // FP32 storage and arithmetic in place takes the taller bands of four
  // wavefronts per SIMD (18.3 GLUPS with 8 x 16 against 17.9 with 8 x 8 at
  // 2048^2; its pre-pass covers the band edges)
  const bool fp32_inplace = p->inplace && fp32_store && arith_size(p->precision) == 4;
  const long long want = fp32_store && !fp32_inplace ? 8192 : 4096;
  int rows = 32;
  while (rows > 2 && strips * *waves * ((p->ny + rows - 1) / rows) < want) rows /= 2;
  *tile_rows = std::min(rows, p->ny);
}

void fill_init_params(const lbm_ehd* h, InitSpec* sp) {
  sp->W = h->P.W;
  sp->c0 = h->P.c0;
  sp->dpsi = h->P.dpsi;
  sp->rho_v = h->P.rho_v;
  sp->drho = h->P.rho_v * h->P.rho_r - h->P.rho_v;
  sp->a_g = a_g_of(h->P);
}

// Length between the two phi = 1/2 crossings of a profile, walking out from
// index `start` (linear interpolation between the bracketing nodes).
bool span(const double* v, int n, double start, double* len) {
  int i0 = (int)std::floor(start);
  i0 = std::min(std::max(i0, 0), n - 1);
  if (!(v[i0] >= 0.5)) return false;
  double hi = NAN, lo = NAN;
  for (int i = i0; i < n - 1; ++i)
    if (v[i] >= 0.5 && v[i + 1] < 0.5) {
      hi = i + (v[i] - 0.5) / (v[i] - v[i + 1]);
      break;
    }
  for (int i = i0; i > 0; --i)
    if (v[i] >= 0.5 && v[i - 1] < 0.5) {
      lo = i - (v[i] - 0.5) / (v[i] - v[i - 1]);
      break;
    }
  if (std::isnan(hi) || std::isnan(lo)) return false;
  *len = hi - lo;
  return true;
}

// Entry points that move or replace a simulation's state refuse members of
// a batch: the batch holds uploaded descriptors (current buffer, step) and a
// captured graph of them, which such a call would make stale.
lbm_status not_member(const lbm_ehd* h, const char* what) {
  if (h->batch)
    return fail(LBM_ESTATE, std::string(what) + ": the simulation is a member of a batch "
                                                "(remove it from the batch first)");
  return LBM_OK;
}

// FP64 invariant sums of the current state into out[NSUM] (the layout of
// k_row_sums), with the per-row partials in `part` [ny][NSUM] and the
// result in `red` [NSUM]; synchronises.
lbm_status read_sums(lbm_ehd* h, double* part, double* red, double out[NSUM]) {
  lbm_status st = dispatch(h, [&](auto F) { return decltype(F)::sums_into(h, part, red); });
  if (st) return st;
  HIP_TRY(hipMemcpyAsync(out, red, NSUM * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};

// Device address of `scratch` on device `dev`, looked up once per device
// with that device current.
lbm_status noalloc_scratch(int dev, double** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(LBM_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    int prev = -1;
    HIP_TRY(hipGetDevice(&prev));
    if (prev != dev) HIP_TRY(hipSetDevice(dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev != dev) (void)hipSetDevice(prev);
    if (e != hipSuccess || !ptr)
      return fail(LBM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                   hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch[dev];
  return LBM_OK;
}

// The watchdog of lbm_ehd_params.diag_every: check the state when the step
// count is a multiple of diag_every.
lbm_status watchdog(lbm_ehd* h) {
  if (h->P.diag_every <= 0 || h->step % h->P.diag_every) return LBM_OK;
  double r[NSUM];
  lbm_status st = read_sums(h, h->part, h->red, r);
  if (st) return st;
  if (r[6] != 0 || !std::isfinite(r[0]) || !std::isfinite(r[1]))
    return fail(LBM_ENONFINITE, "watchdog: " + std::to_string((long long)r[6]) +
                                    " cells not finite at step " + std::to_string(h->step));
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_ehd_params_default(lbm_ehd_params* o) {
  if (!o) return fail(LBM_EINVAL, "out is NULL");
  std::memset(o, 0, sizeof *o);
  o->nx = o->ny = 128;
  o->precision = LBM_FP32;
  o->walls = LBM_ELECTRODES;
  o->reaction = 1;
  o->poisson_form = 1;
  o->poisson_norm = 1;
  o->flow = 1;
  o->ion_force = 1;
  o->mask_f = (1 << 3) | (1 << 4) | (1 << 5);
  o->mask_h = o->mask_p = o->mask_n = o->mask_g = (1 << 1) | (1 << 2);
  o->rho_v = 1.0;
  o->rho_r = 1.0;
  o->eta_v = 0.1;
  o->eta_r = 1.0;
  o->M_phi = 0.1;
  o->W = 4.0;
  o->zeta = 1e-3;
  o->theta = 0.3;
  o->eps_v = 1.0;
  o->eps_r = 1.0;
  o->mu_v = 1.0;
  o->mu_r = 1.0;
  o->m_ratio = 1.0;
  o->v_th = 0.01;
  o->c0 = 1.0;
  o->s_free = 1.0;
  o->n_eps = 1e-4;
  return LBM_OK;
}

lbm_status lbm_ehd_params_from_groups(const lbm_ehd_groups* g, lbm_ehd_params* o) {
  if (!g || !o) return fail(LBM_EINVAL, "NULL argument");
  lbm_ehd_params_default(o);
  const double U = g->U > 0 ? g->U : 0.01, alpha = g->alpha > 0 ? g->alpha : 0.01;
  const double zeta = g->zeta > 0 ? g->zeta : 1e-3, M_phi = g->M_phi > 0 ? g->M_phi : 0.1;
  const double eta_v = g->eta_v > 0 ? g->eta_v : 0.1, eps_v = g->eps_v > 0 ? g->eps_v : 1.0;
  const double n = g->n;
  if (g->n < 8 || !(g->radius > 0) || !(g->W > 0) || !(g->Ca_E > 0) || !(g->eps_r > 0) ||
      !(g->rho_r > 0) || !(g->eta_r > 0) || !(g->m_ratio > 0))
    return fail(LBM_EINVAL, "groups: n >= 8 and positive radius, W, Ca_E, ratios required");
  if (2 * g->radius + 2 * g->W >= n) return fail(LBM_EINVAL, "droplet does not fit the gap");
  if (g->reaction && (!(g->W0 > 0) || !(g->beta > 0)))
    return fail(LBM_EINVAL, "W0 and beta must be positive with the reaction on");
  if (g->sigma_r > 0 && g->reaction)
    return fail(LBM_EINVAL, "sigma_r applies to the leaky model only (reaction = 0)");
  o->nx = o->ny = g->n;
  o->precision = g->precision;
  o->reaction = g->reaction;
  o->W = g->W;
  o->zeta = zeta;
  o->M_phi = M_phi;
  o->eta_v = eta_v;
  o->eta_r = g->eta_r;
  o->rho_r = g->rho_r;
  o->eps_v = eps_v;
  o->eps_r = g->eps_r;
  o->m_ratio = g->m_ratio;
  o->mu_r = g->sigma_r > 0 ? g->sigma_r : g->mu_r;
  if (!(o->mu_r > 0)) return fail(LBM_EINVAL, "mu_r must be positive");
  o->dpsi = n * std::sqrt(g->Ca_E * zeta / (eps_v * g->radius));
  const double mu_bar = U * n / o->dpsi;
  o->mu_v = mu_bar / std::sqrt(g->m_ratio);
  o->v_th = alpha * o->dpsi;
  o->c0 = 1.0;
  o->q = g->W0 > 0 ? g->W0 * eps_v * o->dpsi / (n * n) : 0.0;
  o->gamma_v = g->reaction ? (g->beta * g->beta / g->W0) * n / o->dpsi : 0.0;
  return validate(o);
}

lbm_status lbm_ehd_required_bytes(const lbm_ehd_params* p, size_t* pop_bytes,
                                  size_t* aux_bytes) {
  lbm_status st = validate(p);
  if (st) return st;
  const size_t pitch = pitch_of(p->nx);
  if (pop_bytes)
    *pop_bytes = (size_t)lines_of(*p) * (p->ny + 2) * pitch * elem_size(p->precision);
  if (aux_bytes) {
    if (p->inplace)  // (phi u), one level of the rest of h, the phi' and psi' planes (FP64)
      *aux_bytes =
          (size_t)p->ny * pitch * (2 * arith_size(p->precision) + rest_bytes(p->precision) + 16);
    else
      *aux_bytes =
          (size_t)p->ny * pitch * (2 * arith_size(p->precision) + 2 * rest_bytes(p->precision));
  }
  return LBM_OK;
}

lbm_status lbm_ehd_footprint_bytes(const lbm_ehd_params* p, size_t* bytes) {
  if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
  size_t pb = 0, ab = 0;
  lbm_status st = lbm_ehd_required_bytes(p, &pb, &ab);
  if (st) return st;
  const size_t nc = (size_t)p->nx * p->ny;
  // state + moment and field scratch (allocated on first use) + sums, lines
  // and the sweep's tile list at its largest (one wave, bands of one row)
  *bytes = (p->inplace ? 1 : 2) * pb + ab + 3 * nc * sizeof(double) + 10 * nc * sizeof(double) +
           (size_t)p->ny * NSUM * sizeof(double) + NSUM * sizeof(double) +
           (2 * (size_t)p->ny + 2 * (size_t)p->nx) * sizeof(double) +
           ((size_t)p->ny * ((p->nx + 63) / 64) + 8) * sizeof(BatchTile) + 4096;
  return LBM_OK;
}

lbm_status lbm_ehd_create(const lbm_ehd_params* p, const lbm_ehd_device* dev, lbm_ehd** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm_status st = validate(p);
  if (st) return st;
  size_t pb = 0, ab = 0;
  lbm_ehd_required_bytes(p, &pb, &ab);
  lbm_ehd* h = new (std::nothrow) lbm_ehd;
  if (!h) return fail(LBM_ENOMEM, "host allocation failed");
  h->P = *p;
  h->pitch = pitch_of(p->nx);
  default_launch(p, &h->waves, &h->tile_rows);
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(LBM_EDEVICE, "no HIP device");
  }
  auto cleanup = [&](lbm_status code, const std::string& msg) {
    free_scratch(h);
    delete h;
    return fail(code, msg);
  };
  if (dev) {
    if (!dev->pop[0] || !dev->aux || (!p->inplace && (!dev->pop[1] || dev->pop[0] == dev->pop[1])))
      return cleanup(LBM_EINVAL, "device buffers missing or aliased");
    if (dev->pop_bytes < pb || dev->aux_bytes < ab)
      return cleanup(LBM_ERANGE, "device buffers too small (need " + std::to_string(pb) +
                                     " and " + std::to_string(ab) + " bytes)");
    h->pop[0] = dev->pop[0];
    h->pop[1] = p->inplace ? nullptr : dev->pop[1];
    h->aux = dev->aux;
    h->stream = static_cast<hipStream_t>(dev->stream);
    h->own = false;
  } else {
    h->own = true;
    if (hipMalloc(&h->pop[0], pb) != hipSuccess ||
        (!p->inplace && hipMalloc(&h->pop[1], pb) != hipSuccess) ||
        hipMalloc(&h->aux, ab) != hipSuccess)
      return cleanup(LBM_ENOMEM, "device allocation of the state failed");
  }
  h->pop_bytes = pb;
  h->aux_bytes = ab;
  if (hipMalloc(&h->part, (size_t)p->ny * NSUM * sizeof(double)) != hipSuccess ||
      hipMalloc(&h->red, NSUM * sizeof(double)) != hipSuccess ||
      hipMalloc(&h->line, (2 * (size_t)p->ny + 2 * (size_t)p->nx) * sizeof(double)) !=
          hipSuccess)
    return cleanup(LBM_ENOMEM, "device allocation of scratch failed");
  st = dispatch(h, [&](auto F) { return decltype(F)::prepare_sweep(h); });
  if (st) {
    const std::string msg = g_err;
    return cleanup(st, msg);
  }
  *out = h;
  return LBM_OK;
}

lbm_status lbm_ehd_init_droplet(lbm_ehd* h, double xc, double yc, double radius, double noise,
                                uint64_t seed) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (lbm_status ms = not_member(h, "init")) return ms;
  if (!finite_all({xc, yc, radius, noise})) return fail(LBM_EINVAL, "non-finite argument");
  if (noise < 0 || noise >= 1) return fail(LBM_EINVAL, "noise must lie in [0, 1)");
  if (h->P.walls != LBM_PERIODIC && radius > 0 &&
      (yc - radius < -0.5 || yc + radius > h->P.ny - 0.5))
    return fail(LBM_EINVAL, "droplet crosses an electrode");
  if (h->P.side_walls && radius > 0 && (xc - radius < -0.5 || xc + radius > h->P.nx - 0.5))
    return fail(LBM_EINVAL, "droplet crosses a side wall");
  InitSpec sp;
  std::memset(&sp, 0, sizeof sp);
  sp.xc = xc;
  sp.yc = yc;
  sp.radius = radius;
  sp.noise = noise;
  sp.seed = seed;
  fill_init_params(h, &sp);
  lbm_status st = dispatch(h, [&](auto F) { return decltype(F)::init(h, sp); });
  if (st) return st;
  h->step = 0;
  h->presolve_iters = 0;
  h->presolve_residual = NAN;
  h->ready = true;
  return LBM_OK;
}

lbm_status lbm_ehd_init_fields(lbm_ehd* h, const double* phi, const double* cp,
                               const double* cm, const double* psi, const double* ux,
                               const double* uy) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (lbm_status ms = not_member(h, "init")) return ms;
  if (!phi || !cp || !cm || !psi) return fail(LBM_EINVAL, "phi, cp, cm and psi are required");
  const size_t nc = (size_t)h->P.nx * h->P.ny;
  if (!h->upl) HIP_TRY(hipMalloc(&h->upl, 6 * nc * sizeof(double)));
  const double* srcs[6] = {phi, cp, cm, psi, ux, uy};
  for (int i = 0; i < 6; ++i)
    if (srcs[i])
      HIP_TRY(hipMemcpyAsync(h->upl + i * nc, srcs[i], nc * sizeof(double),
                             hipMemcpyHostToDevice, h->stream));
  InitSpec sp;
  std::memset(&sp, 0, sizeof sp);
  sp.phi = h->upl;
  sp.cp = h->upl + nc;
  sp.cm = h->upl + 2 * nc;
  sp.psi = h->upl + 3 * nc;
  sp.ux = ux ? h->upl + 4 * nc : nullptr;
  sp.uy = uy ? h->upl + 5 * nc : nullptr;
  fill_init_params(h, &sp);
  lbm_status st = dispatch(h, [&](auto F) { return decltype(F)::init(h, sp); });
  if (st) return st;
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->step = 0;
  h->presolve_iters = 0;
  h->presolve_residual = NAN;
  h->ready = true;
  return LBM_OK;
}

lbm_status lbm_ehd_presolve(lbm_ehd* h, int32_t iters) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (lbm_status ms = not_member(h, "presolve")) return ms;
  if (!h->ready) return fail(LBM_ESTATE, "presolve before init");
  if (iters < 0) return fail(LBM_EINVAL, "iters < 0");
  if (iters == 0) return LBM_OK;
  h->presolve_iters = iters;
  h->presolve_residual = NAN;
  return dispatch(h, [&](auto F) { return decltype(F)::presolve(h, iters); });
}

lbm_status lbm_ehd_presolve_to(lbm_ehd* h, double tol, int32_t max_iters, int32_t check_every,
                               int32_t* iters, double* residual) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (lbm_status ms = not_member(h, "presolve")) return ms;
  if (!h->ready) return fail(LBM_ESTATE, "presolve before init");
  if (!(tol > 0) || max_iters < 1 || check_every < 1)
    return fail(LBM_EINVAL, "need tol > 0, max_iters >= 1, check_every >= 1");
  if (h->P.inplace)
    return fail(LBM_EINVAL, "presolve_to: the convergence residual needs two buffers "
                            "(not available with in-place streaming)");
  int done = 0;
  double r = NAN;
  lbm_status st = dispatch(
      h, [&](auto F) { return decltype(F)::presolve_to(h, tol, max_iters, check_every, &done, &r); });
  if (st) return st;
  h->presolve_iters = done;
  h->presolve_residual = r;
  if (iters) *iters = done;
  if (residual) *residual = r;
  return LBM_OK;
}

lbm_status lbm_ehd_step(lbm_ehd* h) { return lbm_ehd_run(h, 1); }

lbm_status lbm_ehd_run(lbm_ehd* h, int64_t nsteps) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
  if (!h->ready) return fail(LBM_ESTATE, "step before init");
  lbm_status st = not_member(h, "step");
  if (st) return st;
  while (nsteps > 0) {
    // up to the next multiple of diag_every, where the watchdog checks
    int64_t n = nsteps;
    if (h->P.diag_every > 0) n = std::min<int64_t>(n, h->P.diag_every - h->step % h->P.diag_every);
    st = dispatch(h, [&](auto F) { return decltype(F)::steps(h, n); });
    if (st) return st;
    h->step += n;
    nsteps -= n;
    st = watchdog(h);
    if (st) return st;
  }
  return LBM_OK;
}

lbm_status lbm_ehd_get_fields(lbm_ehd* h, uint32_t mask, double* out, size_t n_doubles) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (!h->ready) return fail(LBM_ESTATE, "get_fields before init");
  if (mask & ~LBM_FIELD_ALL) return fail(LBM_EINVAL, "unknown field bits");
  const size_t nc = (size_t)h->P.nx * h->P.ny;
  size_t nsel = 0;
  for (int b = 0; b < 10; ++b) nsel += (mask >> b) & 1;
  if (n_doubles < nsel * nc) return fail(LBM_ERANGE, "output buffer too small");
  if (nsel && !out) return fail(LBM_EINVAL, "out is NULL");
  lbm_status st = dispatch(h, [&](auto F) { return decltype(F)::fields(h); });
  if (st) return st;
  size_t k = 0;
  for (int b = 0; b < 10; ++b)
    if ((mask >> b) & 1) {
      HIP_TRY(hipMemcpyAsync(out + k * nc, h->fld + b * nc, nc * sizeof(double),
                             hipMemcpyDeviceToHost, h->stream));
      ++k;
    }
  HIP_TRY(hipStreamSynchronize(h->stream));
  return LBM_OK;
}

lbm_status lbm_ehd_diagnostics(lbm_ehd* h, lbm_ehd_diag* out) {
  if (!h || !out) return fail(LBM_EINVAL, "NULL argument");
  if (!h->ready) return fail(LBM_ESTATE, "diagnostics before init");
  double r[NSUM];
  lbm_status st = read_sums(h, h->part, h->red, r);
  if (st) return st;
  out->step = h->step;
  out->sum_phi = r[0];
  out->sum_rhoe = r[1];
  out->sum_p = r[2];
  out->sum_n = r[3];
  out->nonfinite = (int64_t)r[6];
  out->presolve_iters = h->presolve_iters;
  out->presolve_residual = h->presolve_residual;
  out->D = out->L = out->H = NAN;
  if (out->nonfinite) return fail(LBM_ENONFINITE, "state contains NaN or Inf");
  if (r[0] > 0) {
    // deformation: phi on the lines through the centroid
    const int nx = h->P.nx, ny = h->P.ny;
    const double xb = r[4] / r[0], yb = r[5] / r[0];
    st = dispatch(h, [&](auto F) { return decltype(F)::fields(h); });
    if (st) return st;
    const int j = (int)std::floor(xb), i = (int)std::floor(yb);
    const int j1 = (j + 1) % nx, i1 = std::min(i + 1, ny - 1);
    std::vector<double> c0(ny), c1(ny), r0(nx), r1(nx);
    HIP_TRY(hipMemcpy2DAsync(c0.data(), sizeof(double), h->fld + j, nx * sizeof(double),
                             sizeof(double), ny, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpy2DAsync(c1.data(), sizeof(double), h->fld + j1, nx * sizeof(double),
                             sizeof(double), ny, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(r0.data(), h->fld + (size_t)i * nx, nx * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(r1.data(), h->fld + (size_t)i1 * nx, nx * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const double tx = xb - j, ty = yb - i;
    std::vector<double> col(ny), row(nx);
    for (int y = 0; y < ny; ++y) col[y] = (1 - tx) * c0[y] + tx * c1[y];
    for (int x = 0; x < nx; ++x) row[x] = (1 - ty) * r0[x] + ty * r1[x];
    double L, H;
    if (span(col.data(), ny, yb, &L) && span(row.data(), nx, xb, &H)) {
      out->L = L;
      out->H = H;
      out->D = (L - H) / (L + H);
    }
  }
  return LBM_OK;
}

lbm_status lbm_ehd_invariants_noalloc(lbm_ehd* h, lbm_ehd_diag* out) {
  if (!h || !out) return fail(LBM_EINVAL, "NULL argument");
  if (!h->ready) return fail(LBM_ESTATE, "invariants before init");
  if (h->P.ny > NOALLOC_MAX_ROWS)
    return fail(LBM_ERANGE, "lbm_ehd_invariants_noalloc: ny = " + std::to_string(h->P.ny) +
                                " exceeds its scratch of " + std::to_string(NOALLOC_MAX_ROWS) +
                                " rows (use lbm_ehd_diagnostics)");
  double* sc = nullptr;
  lbm_status st = noalloc_scratch(h->device, &sc);
  if (st) return st;
  double r[NSUM];
  st = read_sums(h, sc, sc + (size_t)NOALLOC_MAX_ROWS * NSUM, r);
  if (st) return st;
  out->step = h->step;
  out->sum_phi = r[0];
  out->sum_rhoe = r[1];
  out->sum_p = r[2];
  out->sum_n = r[3];
  out->nonfinite = (int64_t)r[6];
  out->D = out->L = out->H = NAN;
  out->presolve_iters = h->presolve_iters;
  out->presolve_residual = h->presolve_residual;
  if (out->nonfinite) return fail(LBM_ENONFINITE, "state contains NaN or Inf");
  return LBM_OK;
}

int64_t lbm_ehd_time(const lbm_ehd* h) { return h ? h->step : -1; }

lbm_status lbm_ehd_set_launch(lbm_ehd* h, int32_t waves, int32_t tile_rows) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (lbm_status ms = not_member(h, "set_launch")) return ms;
  if (waves != 1 && waves != 2 && waves != 4 && waves != 8)
    return fail(LBM_EINVAL, "waves must be 1, 2, 4 or 8");
  if (tile_rows < 1) return fail(LBM_EINVAL, "tile_rows must be >= 1");
  h->waves = waves;
  h->tile_rows = std::min<int32_t>(tile_rows, h->P.ny);
  return dispatch(h, [&](auto F) { return decltype(F)::prepare_sweep(h); });
}

lbm_status lbm_ehd_get_launch(const lbm_ehd* h, int32_t* waves, int32_t* tile_rows) {
  if (!h || !waves || !tile_rows) return fail(LBM_EINVAL, "NULL argument");
  *waves = h->waves;
  *tile_rows = h->tile_rows;
  return LBM_OK;
}

namespace {

// What the stored deviations of a state are measured against: the wall
// types (which also fix the reference potential's shape), the anode
// potential, c0, the offset a_g of the g references, the ion line offsets
// and the binary16 scales.  A state read with other values would stand for
// another physical state.
struct RefSig {
  int32_t walls, side_walls, inplace, ion_q9;
  double dpsi, c0, a_g;
  double iofs[10], sc[5];
};

RefSig ref_sig(const lbm_ehd* h) {
  RefSig r;
  std::memset(&r, 0, sizeof r);
  const KP<double> k = make_kp<double>(h);
  r.walls = h->P.walls;
  r.side_walls = h->P.side_walls;
  r.inplace = h->P.inplace;
  r.ion_q9 = h->P.ion_q9;
  r.dpsi = h->P.dpsi;
  r.c0 = h->P.c0;
  r.a_g = k.a_g;
  if (elem_size(h->P.precision) == 2)  // the offsets and scales are used by 16-bit storage only
    for (int i = 0; i < 10; ++i) r.iofs[i] = k.iofs[i];
  for (int i = 0; i < 5; ++i) r.sc[i] = k.sc[i];
  return r;
}

// Header of a saved state.
struct SavedState {
  uint64_t magic;
  int32_t nx, ny, precision, pitch;
  int64_t step;
  int32_t cur, gpar;  // the current buffer, or in place the two orientations
  uint64_t pop_bytes, aux_bytes;
  RefSig ref;
};
constexpr uint64_t STATE_MAGIC = 0x3430455441545345ull;  // "ESTATE04"

}  // namespace

lbm_status lbm_ehd_state_bytes(const lbm_ehd* h, size_t* bytes) {
  if (!h || !bytes) return fail(LBM_EINVAL, "NULL argument");
  *bytes = sizeof(SavedState) + h->pop_bytes + h->aux_bytes;
  return LBM_OK;
}

lbm_status lbm_ehd_save_state(lbm_ehd* h, void* buffer, size_t bytes) {
  if (!h || !buffer) return fail(LBM_EINVAL, "NULL argument");
  if (!h->ready) return fail(LBM_ESTATE, "save before init");
  const size_t need = sizeof(SavedState) + h->pop_bytes + h->aux_bytes;
  if (bytes < need) return fail(LBM_ERANGE, "state buffer too small");
  SavedState hd;
  std::memset(&hd, 0, sizeof hd);
  hd.magic = STATE_MAGIC;
  hd.nx = h->P.nx;
  hd.ny = h->P.ny;
  hd.precision = h->P.precision;
  hd.pitch = h->pitch;
  hd.step = h->step;
  hd.cur = h->P.inplace ? h->par : h->cur;
  hd.gpar = h->P.inplace ? h->gpar : 0;
  hd.pop_bytes = h->pop_bytes;
  hd.aux_bytes = h->aux_bytes;
  hd.ref = ref_sig(h);
  char* out = static_cast<char*>(buffer);
  std::memcpy(out, &hd, sizeof hd);
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipMemcpy(out + sizeof hd, h->pop[h->cur], h->pop_bytes, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(out + sizeof hd + h->pop_bytes, h->aux, h->aux_bytes, hipMemcpyDeviceToHost));
  return LBM_OK;
}

lbm_status lbm_ehd_load_state(lbm_ehd* h, const void* buffer, size_t bytes) {
  if (!h || !buffer) return fail(LBM_EINVAL, "NULL argument");
  if (lbm_status ms = not_member(h, "load_state")) return ms;
  if (bytes < sizeof(SavedState)) return fail(LBM_ERANGE, "state buffer too small");
  SavedState hd;
  std::memcpy(&hd, buffer, sizeof hd);
  if (hd.magic != STATE_MAGIC) return fail(LBM_EINVAL, "not a saved state");
  if (hd.nx != h->P.nx || hd.ny != h->P.ny || hd.precision != h->P.precision ||
      hd.pitch != h->pitch || hd.pop_bytes != h->pop_bytes || hd.aux_bytes != h->aux_bytes ||
      (hd.cur != 0 && hd.cur != 1) || (hd.gpar != 0 && hd.gpar != 1))
    return fail(LBM_EINVAL, "state of another grid, precision or layout");
  const RefSig mine = ref_sig(h);
  if (std::memcmp(&hd.ref, &mine, sizeof mine) != 0)
    return fail(LBM_EINVAL,
                "state stored against other references (walls, side walls, dpsi, c0, theta and "
                "the g rates, or the 16-bit ion offsets and scales differ)");
  if (bytes < sizeof hd + hd.pop_bytes + hd.aux_bytes)
    return fail(LBM_ERANGE, "state buffer too small");
  const char* in = static_cast<const char*>(buffer);
  HIP_TRY(hipStreamSynchronize(h->stream));
  const int into = h->P.inplace ? 0 : hd.cur;
  HIP_TRY(hipMemcpy(h->pop[into], in + sizeof hd, hd.pop_bytes, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->aux, in + sizeof hd + hd.pop_bytes, hd.aux_bytes, hipMemcpyHostToDevice));
  h->cur = into;
  if (h->P.inplace) {
    h->par = hd.cur;
    h->gpar = hd.gpar & 1;
  }
  h->step = hd.step;
  h->ready = true;
  return LBM_OK;
}

lbm_status lbm_ehd_synchronize(lbm_ehd* h) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  HIP_TRY(hipStreamSynchronize(h->stream));
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

lbm_status lbm_ehd_destroy(lbm_ehd* h) {
  if (!h) return LBM_OK;
  if (h->batch) (void)lbm_ehd_batch_remove(h->batch, h);  // waits for the batch's work
  (void)hipStreamSynchronize(h->stream);
  free_scratch(h);
  delete h;
  return LBM_OK;
}

const char* lbm_ehd_last_error(void) { return g_err.c_str(); }

lbm_status lbm_ehd_stream_copy(const void* src, void* dst, size_t bytes, void* stream,
                               int32_t width) {
  if (!src || !dst || bytes == 0 || bytes % 16 || bytes >= 4294967296ull)
    return fail(LBM_EINVAL, "copy size must be a positive multiple of 16 below 4 GiB");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int blocks = 256 * 16;
  if (width == 4)
    hipLaunchKernelGGL(k_copy<4>, dim3(blocks), dim3(256), 0, st, src, dst, (uint32_t)bytes);
  else if (width == 16)
    hipLaunchKernelGGL(k_copy<16>, dim3(blocks), dim3(256), 0, st, src, dst, (uint32_t)bytes);
  else
    return fail(LBM_EINVAL, "width must be 4 or 16");
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

// ---------------------------------------------------------------------------
// Batched sweeps.
// ---------------------------------------------------------------------------
namespace {

void batch_drop_graph(lbm_ehd_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

lbm_status batch_prepare(lbm_ehd_batch* b) {
  if (!b->dirty) return LBM_OK;
  batch_drop_graph(b);
  lbm_status st = dispatch_prec(b->precision, [&](auto F) { return decltype(F)::rebuild(b); });
  if (st) return st;
  b->dirty = false;
  return LBM_OK;
}

lbm_status batch_check_member(const lbm_ehd_batch* b, const lbm_ehd* h) {
  if (!h) return fail(LBM_EINVAL, "NULL member");
  if (!h->ready) return fail(LBM_ESTATE, "batch member not initialised");
  if (h->batch && h->batch != b) return fail(LBM_EINVAL, "simulation is a member of another batch");
  if (h->P.precision != b->precision) return fail(LBM_EINVAL, "batch members differ in precision");
  if (h->P.poisson_iters != 0 || h->P.poisson_tol > 0)
    return fail(LBM_EINVAL, "batch members need poisson_iters = 0 and poisson_tol = 0");
  if (std::find(b->sims.begin(), b->sims.end(), h) != b->sims.end())
    return fail(LBM_EINVAL, "simulation is already a batch member");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != h->device)
    return fail(LBM_EINVAL, "batch members must live on the current device");
  return LBM_OK;
}

// `n` steps launched directly (no graph); members' state moves n times.
lbm_status batch_direct(lbm_ehd_batch* b, int64_t n) {
  for (int64_t i = 0; i < n; ++i) {
    lbm_status st =
        dispatch_prec(b->precision, [&](auto F) { return decltype(F)::launch(b, (int)(i & 1)); });
    if (st) return st;
  }
  if (n & 1) {  // every member's current buffer (or orientation) changed: record it
    for (lbm_ehd* h : b->sims) {
      if (h->P.inplace) {
        h->par ^= 1;
        h->gpar ^= 1;
      } else {
        h->cur = 1 - h->cur;
      }
    }
    b->dirty = true;
  }
  for (lbm_ehd* h : b->sims) h->step += n;
  return LBM_OK;
}

}  // namespace

lbm_status lbm_ehd_batch_create(lbm_ehd* const* sims, int32_t n, void* stream,
                                lbm_ehd_batch** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 0 || (n > 0 && !sims)) return fail(LBM_EINVAL, "bad member list");
  lbm_ehd_batch* b = new (std::nothrow) lbm_ehd_batch;
  if (!b) return fail(LBM_ENOMEM, "host allocation failed");
  b->precision = n > 0 && sims[0] ? sims[0]->P.precision : -1;
  if (stream) {
    b->stream = static_cast<hipStream_t>(stream);
  } else {
    // a blocking stream of default priority: ordered with the legacy default
    // stream that members may use
    if (hipStreamCreate(&b->stream) != hipSuccess) {
      delete b;
      return fail(LBM_EDEVICE, "hipStreamCreate failed");
    }
    b->own_stream = true;
  }
  for (int32_t i = 0; i < n; ++i) {
    lbm_status st = batch_check_member(b, sims[i]);
    if (st) {
      const std::string msg = g_err;
      lbm_ehd_batch_destroy(b);
      return fail(st, msg);
    }
    b->sims.push_back(sims[i]);
    sims[i]->batch = b;
  }
  *out = b;
  return LBM_OK;
}

lbm_status lbm_ehd_batch_add(lbm_ehd_batch* b, lbm_ehd* h) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (b->sims.empty() && h) b->precision = h->P.precision;
  lbm_status st = batch_check_member(b, h);
  if (st) return st;
  // the member's own pending work must be done before the batch stream uses it
  if (h->stream != b->stream) HIP_TRY(hipStreamSynchronize(h->stream));
  b->sims.push_back(h);
  h->batch = b;
  b->dirty = true;
  return LBM_OK;
}

lbm_status lbm_ehd_batch_remove(lbm_ehd_batch* b, lbm_ehd* h) {
  if (!b || !h) return fail(LBM_EINVAL, "NULL argument");
  auto it = std::find(b->sims.begin(), b->sims.end(), h);
  if (it == b->sims.end()) return fail(LBM_EINVAL, "not a member of the batch");
  // the member's state must be complete before it is used on its own stream
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->sims.erase(it);
  h->batch = nullptr;
  b->dirty = true;
  return LBM_OK;
}

int32_t lbm_ehd_batch_size(const lbm_ehd_batch* b) { return b ? (int32_t)b->sims.size() : -1; }

lbm_status lbm_ehd_batch_set_launch(lbm_ehd_batch* b, int32_t waves, int32_t tile_rows) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (waves != 1 && waves != 2 && waves != 4 && waves != 8)
    return fail(LBM_EINVAL, "waves must be 1, 2, 4 or 8");
  if (tile_rows < 1) return fail(LBM_EINVAL, "tile_rows must be >= 1");
  if (waves != b->waves || tile_rows != b->tile_rows) b->dirty = true;
  b->waves = waves;
  b->tile_rows = tile_rows;
  return LBM_OK;
}

lbm_status lbm_ehd_batch_get_launch(const lbm_ehd_batch* b, int32_t* waves, int32_t* tile_rows) {
  if (!b || !waves || !tile_rows) return fail(LBM_EINVAL, "NULL argument");
  *waves = b->waves;
  *tile_rows = b->tile_rows;
  return LBM_OK;
}

lbm_status lbm_ehd_batch_set_graph_steps(lbm_ehd_batch* b, int32_t steps) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (steps < 0 || (steps & 1)) return fail(LBM_EINVAL, "graph steps must be even and >= 0");
  if (steps != b->graph_steps) batch_drop_graph(b);
  b->graph_steps = steps;
  return LBM_OK;
}

lbm_status lbm_ehd_batch_run(lbm_ehd_batch* b, int64_t nsteps) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
  if (b->sims.empty() || nsteps == 0) return LBM_OK;
  lbm_status st = batch_prepare(b);
  if (st) return st;
  const int G = b->graph_steps;
  int64_t blocks = G > 0 ? nsteps / G : 0;
  if (blocks > 0 && !b->exec) {
    // capture one block of G steps (flip 0, 1, 0, ...): an even number of
    // steps leaves every member's state in the buffer it started in, so the
    // block can be replayed as it is
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    lbm_status cst = LBM_OK;
    for (int i = 0; i < G && !cst; ++i)
      cst = dispatch_prec(b->precision, [&](auto F) { return decltype(F)::launch(b, i & 1); });
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (cst) {
      if (g) (void)hipGraphDestroy(g);
      return cst;
    }
    HIP_TRY(e);
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  for (int64_t k = 0; k < blocks; ++k) HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  for (lbm_ehd* h : b->sims) h->step += blocks * G;
  return batch_direct(b, nsteps - blocks * G);
}

lbm_status lbm_ehd_batch_autotune(lbm_ehd_batch* b, int32_t steps_per_trial, int32_t* waves,
                                  int32_t* tile_rows, int64_t* steps_taken) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (steps_per_trial < 2 || (steps_per_trial & 1))
    return fail(LBM_EINVAL, "steps_per_trial must be even and >= 2");
  int64_t taken = 0;
  if (b->sims.empty()) {
    if (steps_taken) *steps_taken = 0;
    return LBM_OK;
  }
  int maxn = 0;
  for (lbm_ehd* h : b->sims) maxn = std::max(maxn, h->P.nx);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best = 1e30f;
  int bw = b->waves, br = b->tile_rows;
  lbm_status st = LBM_OK;
  for (int w : {1, 2, 4, 8}) {
    if (w > 1 && 64 * w > 2 * maxn) continue;  // strips mostly empty
    for (int r : {2, 4, 8, 16, 32}) {
      st = lbm_ehd_batch_set_launch(b, w, r);
      if (!st) st = batch_prepare(b);
      if (!st) st = batch_direct(b, 2);  // warm-up at this shape
      if (!st) st = batch_prepare(b);
      if (st) break;
      (void)hipEventRecord(e0, b->stream);
      st = batch_direct(b, steps_per_trial);
      (void)hipEventRecord(e1, b->stream);
      if (st) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        st = fail(LBM_EDEVICE, "autotune: kernel failed");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      taken += steps_per_trial + 2;
      if (ms < best) {
        best = ms;
        bw = w;
        br = r;
      }
    }
    if (st) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  st = lbm_ehd_batch_set_launch(b, bw, br);
  if (st) return st;
  if (waves) *waves = bw;
  if (tile_rows) *tile_rows = br;
  if (steps_taken) *steps_taken = taken;
  return LBM_OK;
}

lbm_status lbm_ehd_batch_synchronize(lbm_ehd_batch* b) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (b->stream) HIP_TRY(hipStreamSynchronize(b->stream));
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

lbm_status lbm_ehd_batch_destroy(lbm_ehd_batch* b) {
  if (!b) return LBM_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (lbm_ehd* h : b->sims) h->batch = nullptr;
  batch_drop_graph(b);
  (void)hipFree(b->d_desc);
  (void)hipFree(b->d_tiles);
  (void)hipHostFree(b->h_desc);
  (void)hipHostFree(b->h_tiles);
  (void)hipFree(b->d_aadesc);
  (void)hipHostFree(b->h_aadesc);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return LBM_OK;
}

double lbm_ehd_bytes_per_lup(int32_t precision) {
  const size_t s = elem_size(precision);
  if (!s) return 0.0;
  // the moving populations (32; with 16-bit storage 30, plus the lines of
  // the reference phase of h and the reference potential of g, and with
  // bfloat16 storage the two lines of the reference momentum of f), the
  // FP64 rest populations and (phi u)(t-1), each read once and written once
  const double lines = local_h(precision) ? NPOP - 3 + 2 + (lines_of(precision) - NPOP) * 2
                                          : NPOP - 1;
  return 2.0 * lines * s + 2.0 * rest_bytes(precision) + 2.0 * 2.0 * arith_size(precision);
}

}  // extern "C"
