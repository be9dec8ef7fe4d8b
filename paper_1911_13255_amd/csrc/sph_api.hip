// C-ABI of the multi-resolution SPH FSI library (declared in include/mrsph.h):
// arena planning, scene set-up, the Algorithm 1 entry points, graph capture
// of one acoustic step, and FP64 state I/O in original particle order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mlp_internal.h"
#include "mrsph.h"
#include "mrsph_mlp.h"
#include "sph_kernels.h"

using namespace mrsph;

struct sph_ctx {
  Dev D;
  hipStream_t stream;
  int n_scenes, dim;
  std::vector<ScenePar> par;
  LaunchCfg cfg;
  hipGraph_t graph;
  hipGraphExec_t graph_exec;
  int graph_failed;
  int prebin;        // a rebuild set from the host may await binning (sph_advance bins it first)
  hipStream_t side;  // second stream for the concurrent continuity pass (graph capture only)
  hipEvent_t ev_fork, ev_join;
  // streamed solid: the scene states copied to pinned host memory at the end
  // of each step, after the next step's kappa is computed (kappa_next); the
  // next step waits on ev_kappa while its fluid passes run, instead of
  // stopping the stream to read kappa at its solid phase
  SceneState *st_host;
  hipEvent_t ev_kappa;
  int kappa_ready;  // 1: st_host's kappa_next belongs to the step about to be enqueued
  size_t stage_doubles;
  mlp_ctx *net;  // sub-step surrogate (nullptr: plain sub-steps only)
  // position in Algorithm 1's sequence of one acoustic step: 0 at a step
  // boundary, 1 after neighbor_build, 2 after fluid_step, 3 after couple
  // (solid_substeps returns it to 0)
  int phase;
  int features_taken;  // sph_solid_features ran in the current step (its scales await the targets)
  unsigned long long fallback_seen;  // surrogate fall-backs already reported by sph_sync
  double *red_scratch;  // device address of the static reduction scratch on this context's device
  char err[512];
};

namespace {

const size_t kAlign = 256;

struct Plan {
  int dim = 0, n_scenes = 0;
  int nf = 0, nw = 0, ns = 0, nb = 0, ncell = 0, maxn = 0;
  int max_count = 0;
  int capf = 0, capb = 0, lw = 1;  // pair-list capacities per particle and chunk width
  int tile_gp = 0;                 // particles per neighbour tile (0: per-pair gathers)
  std::vector<ScenePar> par;
  std::vector<int> rank_to_cell, cell_scene, bs_scene;
  std::vector<int4> parts_map;  // split form of the block-resident solid kernel: (scene, part, parts, 0)
  // lattice blocks of the streamed solid passes (3D; empty: none): the grid,
  // per scene (grid offset, L0, L1, L2), the blocks, each particle's cell and
  // the lattice axes slowest to fastest in storage
  std::vector<int> lat_grid, lat_cell;
  std::vector<float> lat_jit;  // each particle's offset from its lattice point (3 per particle, FP32)
  double lat_jit_max = 0.0;    // the largest of them, in spacings
  std::vector<int4> lat_scene, lat_blocks;
  int lat_axis[3] = {0, 1, 2};
  LaunchCfg cfg{256, 256, 256};
};

double psi0_lattice(int d, double h_ratio) {
  // number density of an unbounded lattice of unit spacing at h = h_ratio
  double h = h_ratio, s = 0.0;
  double alpha = d == 2 ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
  int R = (int)std::ceil(2.0 * h_ratio) + 1;
  for (int i = -R; i <= R; ++i)
    for (int j = -R; j <= R; ++j)
      for (int k = (d == 3 ? -R : 0); k <= (d == 3 ? R : 0); ++k) {
        double r = std::sqrt((double)(i * i + j * j + k * k));
        double q = r / h;
        if (q >= 2.0) continue;
        double t = 1.0 - 0.5 * q;
        s += alpha * t * t * t * t * (1.0 + 2.0 * q);
      }
  return s;
}

uint64_t morton_code(int d, const int *c) {
  uint64_t code = 0;
  for (int bit = 0; bit < 21; ++bit)
    for (int k = 0; k < d; ++k) code |= (uint64_t)((c[k] >> bit) & 1) << (bit * d + k);
  return code;
}

// Lattice blocks of the streamed solid passes (3D).  Every scene's solid must
// sit near one lattice of spacing dp_S (each axis's coordinate within a
// quarter spacing of an integer number of spacings from the scene's minimum,
// one particle per cell) in a bounding box of at most 4 cells per particle;
// otherwise P keeps no blocks.  Each particle's offset from its lattice
// point is kept (zero to 1e-6 of a spacing on an exact lattice).  Whether the reference neighbours are exactly
// the lattice points within 2 h_S is checked by sph_init once the table is
// built.
void plan_lattice(const sph_scene *sc, int n, Plan &P) {
  std::vector<int> cell((size_t)3 * P.ns);
  std::vector<float> jit((size_t)3 * P.ns, 0.0f);
  double jmax = 0.0;
  long long changes[3] = {0, 0, 0};
  for (int s = 0; s < n; ++s) {
    const sph_scene &S = sc[s];
    const int base = P.par[s].s_begin;
    if (S.n_solid == 0) continue;
    double lo[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = S.x_solid[k];
      for (int i = 1; i < S.n_solid; ++i) lo[k] = std::min(lo[k], S.x_solid[3 * (size_t)i + k]);
    }
    for (int i = 0; i < S.n_solid; ++i)
      for (int k = 0; k < 3; ++k) {
        const double d = (S.x_solid[3 * (size_t)i + k] - lo[k]) / S.dp_s;
        const double r = std::rint(d);
        if (!(std::fabs(d - r) <= 0.25) || r > 1e6) return;
        cell[3 * (size_t)(base + i) + k] = (int)r;
        jit[3 * (size_t)(base + i) + k] = (float)(S.x_solid[3 * (size_t)i + k] - (lo[k] + r * S.dp_s));
        jmax = std::max(jmax, std::fabs(d - r));
        if (i > 0 && cell[3 * (size_t)(base + i) + k] != cell[3 * (size_t)(base + i - 1) + k]) ++changes[k];
      }
  }
  // the axis that changes least often between consecutive particles first
  int ax[3] = {0, 1, 2};
  std::stable_sort(ax, ax + 3, [&](int x, int y) { return changes[x] < changes[y]; });
  std::vector<int> grid;
  std::vector<int4> scene(n), blocks;
  const int B[3] = {kLatB0, kLatB1, kLatB2};
  for (int s = 0; s < n; ++s) {
    const ScenePar &p = P.par[s];
    scene[s] = make_int4((int)grid.size(), 0, 0, 0);
    if (p.s_count == 0) continue;
    int L[3] = {0, 0, 0};
    for (int i = 0; i < p.s_count; ++i)
      for (int k = 0; k < 3; ++k) L[k] = std::max(L[k], cell[3 * (size_t)(p.s_begin + i) + ax[k]] + 1);
    const long long cells = (long long)L[0] * L[1] * L[2];
    if (cells > 4LL * p.s_count + 4096 || (long long)grid.size() + cells > (1LL << 30)) return;
    const size_t g0 = grid.size();
    grid.resize(g0 + (size_t)cells, -1);
    auto at = [&](int c0, int c1, int c2) { return g0 + ((size_t)c0 * L[1] + c1) * L[2] + c2; };
    for (int i = 0; i < p.s_count; ++i) {
      const int *c = &cell[3 * (size_t)(p.s_begin + i)];
      int &g = grid[at(c[ax[0]], c[ax[1]], c[ax[2]])];
      if (g >= 0) return;
      g = p.s_begin + i;
    }
    scene[s] = make_int4((int)g0, L[0], L[1], L[2]);
    const int nfree = p.s_count - p.s_nclamp;
    for (int b0 = 0; b0 < L[0]; b0 += B[0])
      for (int b1 = 0; b1 < L[1]; b1 += B[1])
        for (int b2 = 0; b2 < L[2]; b2 += B[2]) {
          bool any = false;
          for (int c0 = b0; c0 < std::min(L[0], b0 + B[0]) && !any; ++c0)
            for (int c1 = b1; c1 < std::min(L[1], b1 + B[1]) && !any; ++c1)
              for (int c2 = b2; c2 < std::min(L[2], b2 + B[2]) && !any; ++c2) {
                const int a = grid[at(c0, c1, c2)];
                any = a >= 0 && a - p.s_begin < nfree;
              }
          if (any) blocks.push_back(make_int4(s, b0, b1, b2));
        }
  }
  if (blocks.empty()) return;
  P.lat_grid = std::move(grid);
  P.lat_cell = std::move(cell);
  P.lat_jit = std::move(jit);
  P.lat_jit_max = jmax;
  P.lat_scene = std::move(scene);
  P.lat_blocks = std::move(blocks);
  for (int k = 0; k < 3; ++k) P.lat_axis[k] = ax[k];
}

bool make_plan(const sph_scene *sc, int n, const sph_options *opt, Plan &P, std::string &err) {
  if (!sc || n <= 0) {
    err = "no scenes";
    return false;
  }
  P.dim = sc[0].dim;
  P.n_scenes = n;
  if (P.dim != 2 && P.dim != 3) {
    err = "dim must be 2 or 3";
    return false;
  }
  sph_options o{1, 1, 0, 0, 0, 0, 0};
  if (opt) o = *opt;
  P.maxn = o.max_solid_nbr > 0 ? o.max_solid_nbr : (P.dim == 2 ? 40 : 128);
  int max_solid_scene = 0;
  for (int s = 0; s < n; ++s) {
    const sph_scene &S = sc[s];
    if (S.dim != P.dim) {
      err = "all scenes must share dim";
      return false;
    }
    if (S.n_fluid < 0 || S.n_wall < 0 || S.n_solid < 0 || S.n_clamp < 0 || S.n_clamp > S.n_solid) {
      err = "invalid particle counts";
      return false;
    }
    if ((S.n_fluid && !S.x_fluid) || (S.n_wall && (!S.x_wall || !S.nrm_wall)) || (S.n_solid && !S.x_solid)) {
      err = "missing particle arrays";
      return false;
    }
    if (!(S.dp_f > 0) || !(S.dp_s > 0) || !(S.h_ratio > 0) || !(S.rho0_f > 0) || !(S.c_f > 0) ||
        !(S.gamma > 0) || !(S.rho0_s > 0) || !(S.E > 0) || !(S.nu > -1.0 && S.nu < 0.5)) {
      err = "invalid material or resolution parameters";
      return false;
    }
    if ((S.material != 0 && S.material != 1) || (S.single_step != 0 && S.single_step != 1)) {
      err = "material must be 0 or 1 and single_step 0 or 1";
      return false;
    }
    ScenePar p;
    std::memset(&p, 0, sizeof p);
    double hf = S.h_ratio * S.dp_f, hs = S.h_ratio * S.dp_s;
    int nc = 1;
    for (int k = 0; k < 3; ++k) {
      if (k < P.dim) {
        double ext = S.hi[k] - S.lo[k];
        if (!(ext > 0)) {
          err = "empty box";
          return false;
        }
        int m = (int)std::floor(ext / (2.0 * hf));
        if (m < 1) m = 1;
        if (S.periodic[k] && m < 3) {
          err = "periodic axis needs at least 3 cells of 2 h_F";
          return false;
        }
        if (m > 1048576) {
          err = "grid too large";
          return false;
        }
        p.ncell[k] = m;
        p.csd[k] = ext / m;
        p.lo[k] = S.lo[k];
        p.len[k] = ext;
        p.periodic[k] = S.periodic[k] ? 1 : 0;
      } else {
        p.ncell[k] = 1;
        p.csd[k] = 1.0;
        p.lo[k] = 0.0;
        p.len[k] = 1.0;
      }
      p.cs[k] = (float)p.csd[k];
      nc *= p.ncell[k];
    }
    if ((double)P.ncell + nc > 2.0e9) {
      err = "too many cells";
      return false;
    }
    p.f_begin = P.nf;
    p.f_count = S.n_fluid;
    p.w_begin = P.nw;
    p.w_count = S.n_wall;
    p.s_begin = P.ns;
    p.s_count = S.n_solid;
    p.s_nclamp = S.n_clamp;
    p.b_begin = P.nb;
    p.b_count = S.n_wall + S.n_solid - S.n_clamp;
    p.cell_begin = P.ncell;
    p.ncell_total = nc;
    double d = P.dim;
    p.hf = (float)hf;
    p.inv_hf = (float)(1.0 / hf);
    p.r2max_f = (float)(4.0 * hf * hf);
    p.alpha_f = (float)(P.dim == 2 ? 7.0 / (4.0 * M_PI * hf * hf) : 21.0 / (16.0 * M_PI * hf * hf * hf));
    p.hs = (float)hs;
    p.inv_hs = (float)(1.0 / hs);
    p.r2max_s = (float)(4.0 * hs * hs);
    p.alpha_s = (float)(P.dim == 2 ? 7.0 / (4.0 * M_PI * hs * hs) : 21.0 / (16.0 * M_PI * hs * hs * hs));
    p.rho0 = (float)S.rho0_f;
    p.c = (float)S.c_f;
    p.eta = (float)S.eta;
    p.gamma = (float)S.gamma;
    p.p_coef = (float)(S.rho0_f * S.c_f * S.c_f / S.gamma);
    p.gam_inv_rho0c2 = (float)(S.gamma / (S.rho0_f * S.c_f * S.c_f));
    for (int k = 0; k < 3; ++k) p.g[k] = k < P.dim ? (float)S.g[k] : 0.0f;
    p.Vf = (float)std::pow(S.dp_f, d);
    p.Vs = (float)std::pow(S.dp_s, d);
    p.psi0d = psi0_lattice(P.dim, S.h_ratio);
    p.psi0 = (float)p.psi0d;
    p.dpf = S.dp_f;
    p.dps = S.dp_s;
    // Lame parameters from E and nu (E = 2 mu (1 + nu) = 3 K (1 - 2 nu))
    double mu = S.E / (2.0 * (1.0 + S.nu));
    double lam = S.E * S.nu / ((1.0 + S.nu) * (1.0 - 2.0 * S.nu));
    double K = lam + 2.0 * mu / 3.0;
    p.rho0s = (float)S.rho0_s;
    p.mu = (float)mu;
    p.lam = (float)lam;
    p.c_s = (float)std::sqrt(K / S.rho0_s);
    p.cfl_ac = (float)S.cfl_ac;
    p.cfl_ad = (float)S.cfl_ad;
    p.cfl_s = (float)S.cfl_s;
    p.u_ref = (float)S.u_ref;
    p.dt_visc = S.eta > 0 ? S.cfl_ad * hf * hf * S.rho0_f / S.eta : 0.0;
    p.in_U0 = (float)S.inflow_U0;
    p.in_ts = (float)S.inflow_ts;
    p.in_H = (float)S.inflow_H;
    p.in_len = (float)S.inflow_len;
    p.riemann = o.riemann ? 1 : 0;
    p.reinit = o.density_reinit;
    p.material = S.material;
    p.single_step = S.single_step;
    // Morton order of the scene's cells
    std::vector<std::pair<uint64_t, int>> codes(nc);
    for (int lin = 0; lin < nc; ++lin) {
      int c[3] = {lin % p.ncell[0], (lin / p.ncell[0]) % p.ncell[1], lin / (p.ncell[0] * p.ncell[1])};
      codes[lin] = {morton_code(P.dim, c), lin};
    }
    std::sort(codes.begin(), codes.end());
    for (int r = 0; r < nc; ++r) {
      P.rank_to_cell.push_back(p.cell_begin + codes[r].second);
      P.cell_scene.push_back(s);
    }
    for (int q = 0; q < p.b_count; ++q) P.bs_scene.push_back(s);
    P.nf += S.n_fluid;
    P.nw += S.n_wall;
    P.ns += S.n_solid;
    P.nb += p.b_count;
    P.ncell += nc;
    P.max_count = std::max(P.max_count, std::max(S.n_fluid, std::max(S.n_wall, S.n_solid)));
    max_solid_scene = std::max(max_solid_scene, S.n_solid);
    P.par.push_back(p);
  }
  int max_free_scene = 0;
  for (int s = 0; s < n; ++s) max_free_scene = std::max(max_free_scene, sc[s].n_solid - sc[s].n_clamp);
  int bs = o.solid_block;
  if (bs != 0 && (bs < 64 || bs > 1024 || (bs & (bs - 1)))) {
    err = "solid_block must be a power of two in [64, 1024]";
    return false;
  }
  // register-resident solid kernel (2D) when every scene's free solid fits
  // 2048 particles (at most 4 per thread); otherwise streamed passes
  P.cfg.solid_ppt = 0;
  // (and its reference table fits the 31-bit range of a buffer resource)
  const bool table_fits = (size_t)(P.maxn + kSolidBatch) * P.ns * sizeof(float4) < (size_t)INT_MAX;
  if (o.solid_lds != 1 && P.dim == 2 && max_free_scene > 0 && max_free_scene <= 2048 && table_fits) {
    // block limits of the register-resident kernel: 1024, 768, 512 threads
    int ppt = max_free_scene <= 1024 ? 1 : (max_free_scene <= 1536 ? 2 : 4);
    int limit = ppt == 1 ? 1024 : (ppt == 2 ? 768 : 512);
    P.cfg.solid_ppt = ppt;
    int need = (max_free_scene + ppt - 1) / ppt;
    int want = std::max(64, (need + 63) / 64 * 64);
    if (bs == 0 || bs > limit) bs = std::min(limit, want);
  }
  if (bs == 0) {
    bs = 64;
    while (bs < max_solid_scene && bs < 1024) bs *= 2;
  }
  if (P.cfg.solid_ppt && (long long)bs * P.cfg.solid_ppt < max_free_scene) P.cfg.solid_ppt = 0;
  P.cfg.block_solid = bs;
  // lanes per particle: enough lanes in flight to keep about eight waves per
  // CU, and in 3D at least 4 (about 80 neighbours per particle: four lanes
  // share a row's loads; measured on the 2.0M-particle dam break, 1 lane per
  // particle ran the force pass in 0.94 ms, 2 in 0.72, 4 in 0.63, 8 in 0.64)
  const int dim3_min = P.dim == 3 ? 4 : 1;
  auto pick_lpp = [dim3_min](long long nparticles) {
    const long long target = 256LL * 8 * 64;
    int l = dim3_min;
    while (l < 16 && nparticles * l < target) l *= 2;
    return l;
  };
  int lpp = o.lanes_per_particle;
  if (lpp != 0 && lpp != 1 && lpp != 2 && lpp != 4 && lpp != 8 && lpp != 16) {
    err = "lanes_per_particle must be 1, 2, 4, 8 or 16";
    return false;
  }
  P.cfg.lpp_force = P.cfg.lpp_cont = P.cfg.lpp_reinit = lpp ? lpp : pick_lpp(P.nf);
  P.cfg.lpp_couple = lpp ? lpp : pick_lpp(P.ns);
  int bp = o.block_pair;
  if (bp != 0 && bp != 64 && bp != 128 && bp != 256) {
    err = "block_pair must be 64, 128 or 256";
    return false;
  }
  P.cfg.block_pair = bp ? bp : 256;
  P.cfg.block_couple = 64;
  if (o.fluid_tiles != 0 && o.fluid_tiles != -1) {
    err = "fluid_tiles must be 0 or -1";
    return false;
  }
  // neighbour tiles: one group per block of the pair launches (3D)
  P.tile_gp = (P.dim == 3 && o.fluid_tiles == 0) ? P.cfg.block_pair / P.cfg.lpp_force : 0;
  if (o.solid_blocks != 0 && o.solid_blocks != -1) {
    err = "solid_blocks must be 0 or -1";
    return false;
  }
  if (P.dim == 3 && P.ns > 0 && o.solid_blocks == 0) plan_lattice(sc, n, P);
  if (o.serial_passes != 0 && o.serial_passes != 1) {
    err = "serial_passes must be 0 or 1";
    return false;
  }
  P.cfg.fork = o.serial_passes ? 0 : 1;
  P.cfg.solid_lds_n = P.cfg.solid_ppt ? max_solid_scene : 0;  // confirmed against the device in sph_init
  // split form of the block-resident solid kernel: ceil(n_free / target)
  // workgroups per scene (one for a scene with one shared step), the target
  // doubled until the launch holds at most 256 of them (one per CU, so that
  // all of a scene's workgroups are resident together)
  if (o.solid_parts < 0) {
    err = "solid_parts must be >= 0";
    return false;
  }
  P.parts_map.clear();
  P.cfg.solid_parts = 0;
  if (P.cfg.solid_ppt > 0 && o.solid_parts > 0) {
    constexpr int kMaxPartsBlocks = 256;
    for (long long target = o.solid_parts;; target *= 2) {
      std::vector<int4> m;
      bool split = false;
      for (int s = 0; s < n; ++s) {
        const long long nfree = sc[s].n_solid - sc[s].n_clamp;
        const int k = (sc[s].single_step || nfree <= target) ? 1 : (int)((nfree + target - 1) / target);
        split |= k > 1;
        for (int q = 0; q < k; ++q) m.push_back(make_int4(s, q, k, 0));
      }
      if (!split) break;
      if ((int)m.size() <= kMaxPartsBlocks) {
        P.parts_map = m;
        P.cfg.solid_parts = (int)target;
        break;
      }
    }
  }
  // pair-list capacities: particles of a lattice inside the support 2 h_F,
  // with room for compression (fluid) and for the finer solid lattice
  // (boundary: walls at dp_F plus solid at dp_S)
  {
    double hr = 0.0, ratio = 1.0;
    for (int s = 0; s < n; ++s) {
      hr = std::max(hr, sc[s].h_ratio);
      if (sc[s].n_solid > 0) ratio = std::max(ratio, sc[s].dp_f / sc[s].dp_s);
    }
    double R = 2.0 * hr;
    double ball = P.dim == 2 ? M_PI * R * R : 4.0 / 3.0 * M_PI * R * R * R;
    auto up16 = [](double x) { return ((int)std::ceil(x) + 15) / 16 * 16; };
    int cf = o.max_fluid_nbr, cbn = o.max_boundary_nbr;
    if (cf < 0 || cbn < 0 || cf > 4096 || cbn > 4096) {
      err = "max_fluid_nbr and max_boundary_nbr must lie in [0, 4096]";
      return false;
    }
    P.capf = cf ? up16(cf) : up16(2.0 * ball + 8.0);
    P.capb = cbn ? up16(cbn) : up16(ball * (1.0 + std::pow(ratio, P.dim)) + 16.0);
    P.lw = P.cfg.lpp_force;
    // neighbour indices share 27 bits of an entry with the relative cell id
    if ((long long)P.nf + P.nb >= (1LL << 27)) {
      err = "more than 2^27 fluid plus boundary particles";
      return false;
    }
  }
  return true;
}

// Assign arena offsets; with base == nullptr only the size is computed.
size_t carve(char *base, const Plan &P, Dev &D) {
  size_t off = 0;
  auto take = [&](auto *&ptr, size_t count) {
    using T = std::remove_reference_t<decltype(*ptr)>;
    off = (off + kAlign - 1) / kAlign * kAlign;
    ptr = reinterpret_cast<T *>(base + off);
    off += std::max<size_t>(count, 1) * sizeof(T);
  };
  size_t nf = P.nf, nw = P.nw, ns = P.ns, nb = P.nb, nc = P.ncell, S = P.n_scenes;
  take(D.par, S);
  take(D.st, S);
  take(D.f_scene, nf);
  take(D.f_lin, nf);
  take(D.f_id, nf);
  take(D.f_pos, nf);
  take(D.f_off, nf);
  take(D.f_posd, nf);
  take(D.f_va, nf);
  take(D.f_vb, nf);
  take(D.f_vs, nf);
  take(D.f_acc, nf);
  take(D.f_drho, nf);
  take(D.f_p, nf);
  take(D.f_nnb, nf);
  take(D.f_nbl, nf * (size_t)P.capf);
  take(D.f_bnl, nf * (size_t)P.capb);
  take(D.f_rowlen, nf);
  {
    const size_t groups = P.tile_gp ? (nf + P.tile_gp - 1) / P.tile_gp : 0;
    take(D.t_union, groups * kTileCap);
    take(D.t_count, groups);
    take(D.t_rows, groups ? nf * (size_t)P.capf : 0);
  }
  take(D.f_speed, nf);
  take(D.fs_lin, nf);
  take(D.fs_slot, nf);
  take(D.fs_id, nf);
  take(D.f_perm, nf);
  take(D.f_pkey, nf);
  take(D.fs_off, nf);
  take(D.fs_va, nf);
  take(D.fs_drho, nf);
  take(D.fs_m, nf);
  take(D.fc_count, nc);
  take(D.bc_count, nc);
  take(D.rank_to_cell, nc);
  take(D.cell_scene, nc);
  take(D.fc_se, nc);
  take(D.bc_se, nc);
  take(D.cell_part, (nc + kCellTile - 1) / kCellTile + 1);
  take(D.w_lin, nw);
  take(D.w_scene, nw);
  take(D.w_off, nw);
  take(D.w_nrm, nw);
  take(D.b_pos, nb);
  take(D.b_vbar, nb);
  take(D.b_nrm, nb);
  take(D.b_posd, nb);
  take(D.b_perm, nb);
  take(D.b_solid, nb);
  take(D.b_src, nb);
  take(D.bs_lin, nb);
  take(D.bs_slot, nb);
  take(D.bs_scene, nb);
  take(D.bs_off, nb);
  take(D.s_scene, ns);
  take(D.s_lin0, ns);
  take(D.s_bslot, ns);
  take(D.s_blin, ns);
  take(D.s_cnt, ns);
  take(D.s_off0, 3 * ns);
  double **dvec[] = {&D.s_u, &D.s_v, &D.s_du, &D.s_dv};
  for (double **p : dvec) take(*p, 3 * ns);
  double **dten[] = {&D.s_H, &D.s_dF, &D.s_B};
  for (double **p : dten) take(*p, 9 * ns);
  take(D.s_PBg, 3 * ns);
  take(D.s_PBf, 9 * std::max(ns, P.lat_grid.size()));
  take(D.s_vf, std::max(ns, P.lat_grid.size()));
  take(D.s_nbc, P.dim == 3 ? (size_t)P.maxn * ns : 1);
  take(D.s_gcls, kNbrClasses);
  take(D.nbc_ok, 1);
  take(D.lat_grid, P.lat_grid.size());
  take(D.lat_of, P.lat_grid.empty() ? 1 : ns);
  take(D.lat_jit, P.lat_grid.empty() ? 1 : 3 * P.lat_grid.size());
  take(D.lat_scene, P.lat_scene.size());
  take(D.lat_blocks, P.lat_blocks.size());
  take(D.lat_cls, P.lat_blocks.empty() ? 1 : kNbrClasses);
  float **vec[] = {&D.s_a, &D.s_fF, &D.s_vbar, &D.s_abar, &D.s_n0, &D.s_n, &D.s_fFp,
                   &D.sur_vbar, &D.sur_abar};
  for (float **p : vec) take(*p, 3 * ns);
  take(D.sur_aux, (size_t)6 * ns);
  take(D.s_parts, std::max<size_t>(1, P.parts_map.size()));
  take(D.parts_sync, 4 * (size_t)P.n_scenes);
  take(D.s_xpb, P.parts_map.empty() ? 1 : (size_t)P.dim * P.dim * ns);
  take(D.s_xv, P.parts_map.empty() ? 1 : (size_t)P.dim * ns);
  take(D.sur_stats, 2 * kSurFeat + 2 * kSurOut);
  take(D.s_r0d, 3 * ns);
  take(D.s_gsum, 3 * ns);
  take(D.s_nbr, (size_t)(P.maxn + kSolidBatch) * ns);
  take(D.s_cpl_cnt, ns);
  take(D.s_cpl, (size_t)P.capf * ns);
  take(D.stage, 9 * (size_t)std::max(P.max_count, 64) + 64);
  take(D.red, 16 * 1024);
  take(D.rebuild_count, 1);
  return off + kAlign;
}

#define HIPCHK(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess) {                                                               \
      std::snprintf(ctx->err, sizeof ctx->err, "%s: %s", #call, hipGetErrorString(e_));   \
      return SPH_E_HIP;                                                                   \
    }                                                                                     \
  } while (0)

int check_launch(sph_ctx *ctx, const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    std::snprintf(ctx->err, sizeof ctx->err, "%s: %s", what, hipGetErrorString(e));
    return SPH_E_HIP;
  }
  return SPH_OK;
}

int field_width(int dim, int field) {
  switch (field) {
  case SPH_F_X: case SPH_F_V: case SPH_F_A: case SPH_S_U: case SPH_S_V: case SPH_S_A: case SPH_S_FF:
  case SPH_S_VBAR: case SPH_S_ABAR: case SPH_S_N: case SPH_S_N0: case SPH_S_X0:
    return dim;
  case SPH_F_RHO: case SPH_F_DRHO: case SPH_F_P:
    return 1;
  case SPH_F_NNB:
    return 2;
  case SPH_S_F: case SPH_S_DF: case SPH_S_B:
    return dim * dim;
  }
  return 0;
}

// Call-order check of the step sequence (Algorithm 1): `need` is the phase the
// call requires.
int check_phase(sph_ctx *ctx, const char *call, int need) {
  if (ctx->phase == need) return SPH_OK;
  static const char *where[] = {"at a step boundary (after sph_init or solid_substeps)", "after neighbor_build",
                                "after fluid_step", "after couple"};
  std::snprintf(ctx->err, sizeof ctx->err, "%s called out of sequence: it runs %s, the context is %s", call,
                where[need], where[ctx->phase]);
  return SPH_E_ORDER;
}

int read_states(sph_ctx *ctx, std::vector<SceneState> &st) {
  st.resize(ctx->n_scenes);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipMemcpy(st.data(), ctx->D.st, sizeof(SceneState) * ctx->n_scenes, hipMemcpyDeviceToHost));
  return SPH_OK;
}

// kappa solid sub-steps.  Small 2D solids: one
// register-resident launch per step with kappa decided on the device.  Other
// solids: streamed passes over all solid particles; kappa sizes the host's
// pass loop: inside sph_advance it was copied to pinned memory at the end of
// the step before (the host waits on that copy only), otherwise it is read
// back here (this synchronises the stream).
// Register-resident sub-steps, preceded by the surrogate pass when a network
// is set (the solid launch then takes the learned steps and judges).
// step_end: the solid launch also does the step-end reduction's work;
// alone: nothing runs beside the launch, so its split form may be used
// (not with a surrogate, whose judge reduces over one workgroup per scene)
void enqueue_solid_reg(sph_ctx *ctx, bool step_end, bool alone = true) {
  const bool sur = ctx->net && ctx->D.sur_thr > 0.0f;
  if (sur) launch_sur_net(ctx->D, ctx->net->D, ctx->stream);
  launch_solid(ctx->D, ctx->cfg, ctx->stream, step_end, alone && !sur);
}

// step_end as above; it applies to the register-resident form only (the
// streamed passes leave the step end to its own launch).  maxima: the
// streamed averaging pass also reduces the solid maxima that
// launch_solid_dt_next then takes.
int enqueue_solid(sph_ctx *ctx, bool step_end, bool maxima = false) {
  if (ctx->cfg.solid_ppt > 0) {
    enqueue_solid_reg(ctx, step_end);
  } else if (ctx->D.ns > 0) {
    int kmax = 0;
    bool adopt = false;
    if (ctx->kappa_ready) {
      // kappa as the end of the step before computed it from the same state
      // (the averaging pass flags a scene whose kappa exceeds the passes):
      // k_solid_first adopts it and starts the step's increments
      ctx->kappa_ready = 0;
      adopt = true;
      if (hipEventSynchronize(ctx->ev_kappa) != hipSuccess) {
        std::snprintf(ctx->err, sizeof ctx->err, "solid_substeps: kappa read-back failed");
        return SPH_E_HIP;
      }
      for (int s = 0; s < ctx->n_scenes; ++s) kmax = std::max(kmax, ctx->st_host[s].kappa_next);
    } else {
      launch_solid_dt(ctx->D, ctx->stream);
      std::vector<SceneState> st(ctx->n_scenes);
      if (hipMemcpyAsync(st.data(), ctx->D.st, sizeof(SceneState) * ctx->n_scenes, hipMemcpyDeviceToHost,
                         ctx->stream) != hipSuccess ||
          hipStreamSynchronize(ctx->stream) != hipSuccess) {
        std::snprintf(ctx->err, sizeof ctx->err, "solid_substeps: kappa read-back failed");
        return SPH_E_HIP;
      }
      for (const SceneState &x : st) kmax = std::max(kmax, x.kappa);
    }
    launch_solid_first(ctx->D, adopt, ctx->stream);
    for (int sub = 0; sub < kmax; ++sub) launch_solid_pass(ctx->D, sub, ctx->stream);
    launch_solid_average(ctx->D, kmax, maxima, ctx->stream);
  } else {
    launch_solid_dt(ctx->D, ctx->stream);
  }
  return SPH_OK;
}

// One acoustic step.  With a second stream the continuity pass (which no
// later pass of the step reads until the step-end kernel) runs concurrently
// with the coupling and solid passes.
int enqueue_step(sph_ctx *ctx, bool fork) {
  launch_rebuild(ctx->D, ctx->cfg, ctx->stream, false);
  launch_fluid_force(ctx->D, ctx->cfg, ctx->stream);
  if (fork && ctx->cfg.fork && ctx->side && ctx->cfg.solid_ppt > 0) {
    if (hipEventRecord(ctx->ev_fork, ctx->stream) != hipSuccess ||
        hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0) != hipSuccess)
      return SPH_E_HIP;
    launch_fluid_continuity(ctx->D, ctx->cfg, ctx->side, false);
    launch_couple(ctx->D, ctx->cfg, ctx->stream);
    enqueue_solid_reg(ctx, false, false);
    if (hipEventRecord(ctx->ev_join, ctx->side) != hipSuccess ||
        hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0) != hipSuccess)
      return SPH_E_HIP;
    launch_step_end(ctx->D, ctx->stream, false);
    return check_launch(ctx, "acoustic step");
  }
  if (!launch_fluid_continuity(ctx->D, ctx->cfg, ctx->stream, true)) launch_couple(ctx->D, ctx->cfg, ctx->stream);
  const bool next_kappa = ctx->cfg.solid_ppt == 0 && ctx->D.ns > 0 && ctx->st_host;
  int rc = enqueue_solid(ctx, true, next_kappa);
  if (rc != SPH_OK) return rc;
  // the next step's kappa depends only on the state this close leaves
  launch_step_end(ctx->D, ctx->stream, ctx->cfg.solid_ppt > 0, next_kappa);
  if (next_kappa) {
    if (hipMemcpyAsync(ctx->st_host, ctx->D.st, sizeof(SceneState) * ctx->n_scenes, hipMemcpyDeviceToHost,
                       ctx->stream) != hipSuccess ||
        hipEventRecord(ctx->ev_kappa, ctx->stream) != hipSuccess)
      return SPH_E_HIP;
    ctx->kappa_ready = 1;
  }
  return check_launch(ctx, "acoustic step");
}

}  // namespace

extern "C" {

size_t sph_arena_bytes(const sph_scene *scenes, int n_scenes, const sph_options *opt) {
  Plan P;
  std::string err;
  if (!make_plan(scenes, n_scenes, opt, P, err)) return 0;
  Dev D;
  std::memset(&D, 0, sizeof D);
  return carve(nullptr, P, D);
}

int sph_init(const sph_scene *scenes, int n_scenes, const sph_options *opt, void *dev_arena, size_t arena_bytes,
             void *stream, sph_ctx **out) {
  if (!out) return SPH_E_ARG;
  *out = nullptr;
  Plan P;
  std::string perr;
  if (!make_plan(scenes, n_scenes, opt, P, perr)) return SPH_E_ARG;
  sph_ctx *ctx = new sph_ctx();
  std::memset(&ctx->D, 0, sizeof ctx->D);
  ctx->stream = (hipStream_t)stream;
  ctx->n_scenes = n_scenes;
  ctx->dim = P.dim;
  ctx->par = P.par;
  ctx->cfg = P.cfg;
  ctx->graph = nullptr;
  ctx->graph_exec = nullptr;
  ctx->net = nullptr;
  ctx->side = nullptr;
  ctx->ev_fork = ctx->ev_join = nullptr;
  ctx->st_host = nullptr;
  ctx->ev_kappa = nullptr;
  ctx->kappa_ready = 0;
  if (hipHostMalloc((void **)&ctx->st_host, sizeof(SceneState) * n_scenes, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_kappa, hipEventDisableTiming) != hipSuccess) {
    if (ctx->st_host) (void)hipHostFree(ctx->st_host);
    ctx->st_host = nullptr;
    ctx->ev_kappa = nullptr;
    (void)hipGetLastError();
  }
  if (ctx->stream) {
    // default priority, like every stream here
    if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess) {
      ctx->side = nullptr;
      (void)hipGetLastError();
    }
  }
  {
    // the register-resident solid kernel holds v and P B of the largest
    // scene in LDS; when they do not fit, the streamed passes are used
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      lds_max = 0;
    size_t need_lds = (size_t)ctx->cfg.solid_lds_n * solid_lds_bytes_per_particle(P.dim);
    // the kernel's own shared arrays take under 1 KiB
    if (ctx->cfg.solid_lds_n <= 0 || need_lds + 1024 > (size_t)lds_max ||
        allow_solid_lds(P.dim, ctx->cfg.solid_ppt, need_lds) != hipSuccess) {
      ctx->cfg.solid_lds_n = 0;
      ctx->cfg.solid_ppt = 0;
      (void)hipGetLastError();
    }

  }
  ctx->graph_failed = 0;
  ctx->err[0] = 0;
  ctx->phase = 0;
  ctx->fallback_seen = 0;
  // the static scratch of sph_reduce_noalloc: its device address, taken at
  // set-up on the context's device (null when unavailable: that entry point
  // then reports the failure)
  ctx->red_scratch = nullptr;
  if (reduce_scratch(&ctx->red_scratch) != hipSuccess) {
    ctx->red_scratch = nullptr;
    (void)hipGetLastError();
  }
  size_t need = carve(nullptr, P, ctx->D);
  if (!dev_arena || arena_bytes < need) {
    std::snprintf(ctx->err, sizeof ctx->err, "arena too small: %zu < %zu", arena_bytes, need);
    delete ctx;
    return SPH_E_ARG;
  }
  char *base = (char *)(((uintptr_t)dev_arena + kAlign - 1) / kAlign * kAlign);
  carve(base, P, ctx->D);
  Dev &D = ctx->D;
  D.n_scenes = n_scenes;
  D.dim = P.dim;
  D.nf = P.nf;
  D.nw = P.nw;
  D.ns = P.ns;
  D.nb = P.nb;
  D.ncell = P.ncell;
  D.maxn = P.maxn;
  D.nbr_rows = P.maxn + kSolidBatch;
  {
    size_t tb = (size_t)D.nbr_rows * P.ns * sizeof(float4);
    D.nbr_bytes = tb < (size_t)INT_MAX ? (int)tb : 0;
  }
  D.capf = P.capf;
  // the snapshot pass saves the force pass one gather per pair; a tile forms
  // the snapshot once per neighbour in its staging instead
  D.fluid_prep = (P.nf >= 100000 && P.tile_gp == 0) ? 1 : 0;
  D.any_single = 0;
  for (int s = 0; s < n_scenes; ++s) D.any_single |= P.par[s].single_step;
  D.capb = P.capb;
  D.lw = P.lw;
  D.tile_gp = P.tile_gp;
  ctx->stage_doubles = 9 * (size_t)std::max(P.max_count, 64) + 64;
  hipStream_t st = ctx->stream;
  int rc = SPH_OK;
  auto fail = [&](int code) {
    sph_destroy(ctx);
    return code;
  };
#define HIPCHK_INIT(call)                                                               \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      std::fprintf(stderr, "mrsph: %s: %s\n", #call, hipGetErrorString(e_));            \
      return fail(SPH_E_HIP);                                                           \
    }                                                                                   \
  } while (0)
  HIPCHK_INIT(hipMemcpyAsync(D.par, P.par.data(), sizeof(ScenePar) * n_scenes, hipMemcpyHostToDevice, st));
  std::vector<SceneState> s0(n_scenes);
  std::memset(s0.data(), 0, sizeof(SceneState) * n_scenes);
  for (auto &x : s0) x.need_rebuild = 1;
  HIPCHK_INIT(hipMemcpyAsync(D.st, s0.data(), sizeof(SceneState) * n_scenes, hipMemcpyHostToDevice, st));
  // every scene starts with its flag set
  HIPCHK_INIT(hipMemcpy(D.rebuild_count, &n_scenes, sizeof(int), hipMemcpyHostToDevice));
  if (P.ns) HIPCHK_INIT(hipMemsetAsync(D.s_cpl_cnt, 0, sizeof(int) * P.ns, st));
  // no tile yet: rows hold neighbour indices until a group's first rebuild
  if (P.tile_gp)
    HIPCHK_INIT(hipMemsetAsync(D.t_count, 0xff, sizeof(int) * ((P.nf + P.tile_gp - 1) / P.tile_gp), st));
  if (P.ncell) {
    HIPCHK_INIT(hipMemcpyAsync(D.rank_to_cell, P.rank_to_cell.data(), sizeof(int) * P.ncell, hipMemcpyHostToDevice, st));
    HIPCHK_INIT(hipMemcpyAsync(D.cell_scene, P.cell_scene.data(), sizeof(int) * P.ncell, hipMemcpyHostToDevice, st));
    HIPCHK_INIT(hipMemsetAsync(D.fc_count, 0, sizeof(int) * P.ncell, st));
    HIPCHK_INIT(hipMemsetAsync(D.bc_count, 0, sizeof(int) * P.ncell, st));
    HIPCHK_INIT(hipMemsetAsync(D.fc_se, 0, sizeof(int2) * P.ncell, st));
    HIPCHK_INIT(hipMemsetAsync(D.bc_se, 0, sizeof(int2) * P.ncell, st));
  }
  if (P.nb)
    HIPCHK_INIT(hipMemcpyAsync(D.bs_scene, P.bs_scene.data(), sizeof(int) * P.nb, hipMemcpyHostToDevice, st));
  D.n_parts_blocks = (int)P.parts_map.size();
  if (!P.parts_map.empty())
    HIPCHK_INIT(hipMemcpyAsync(D.s_parts, P.parts_map.data(), sizeof(int4) * P.parts_map.size(),
                               hipMemcpyHostToDevice, st));
  HIPCHK_INIT(hipMemsetAsync(D.parts_sync, 0, sizeof(unsigned) * 4 * n_scenes, st));
  for (int s = 0; s < n_scenes; ++s) {
    const sph_scene &S = scenes[s];
    int d = P.dim;
    size_t n1 = (size_t)d * std::max(S.n_fluid, std::max(S.n_wall, S.n_solid));
    double *x_d = D.stage, *v_d = D.stage + n1;
    if (S.n_fluid) {
      HIPCHK_INIT(hipMemcpyAsync(x_d, S.x_fluid, sizeof(double) * d * S.n_fluid, hipMemcpyHostToDevice, st));
      if (S.v_fluid)
        HIPCHK_INIT(hipMemcpyAsync(v_d, S.v_fluid, sizeof(double) * d * S.n_fluid, hipMemcpyHostToDevice, st));
      double gabs = 0.0;
      for (int k = 0; k < d; ++k) gabs += S.g[k] * S.g[k];
      launch_init_scene(D, s, x_d, v_d, S.v_fluid ? 1 : 0, std::sqrt(gabs), S.hydro_H, std::pow(S.dp_f, d),
                        S.n_fluid, st);
    }
    if (S.n_wall) {
      HIPCHK_INIT(hipMemcpyAsync(x_d, S.x_wall, sizeof(double) * d * S.n_wall, hipMemcpyHostToDevice, st));
      HIPCHK_INIT(hipMemcpyAsync(v_d, S.nrm_wall, sizeof(double) * d * S.n_wall, hipMemcpyHostToDevice, st));
      launch_init_walls(D, s, x_d, v_d, S.n_wall, st);
    }
    if (S.n_solid) {
      HIPCHK_INIT(hipMemcpyAsync(x_d, S.x_solid, sizeof(double) * d * S.n_solid, hipMemcpyHostToDevice, st));
      if (S.v_solid)
        HIPCHK_INIT(hipMemcpyAsync(v_d, S.v_solid, sizeof(double) * d * S.n_solid, hipMemcpyHostToDevice, st));
      launch_init_solid(D, s, x_d, v_d, S.v_solid ? 1 : 0, S.n_solid, st);
      launch_solid_reference(D, s, S.n_solid, st);
    }
    // the staging buffer is reused by the next scene: wait for this one
    HIPCHK_INIT(hipStreamSynchronize(st));
    if ((rc = check_launch(ctx, "scene set-up")) != SPH_OK) return fail(rc);
  }
  launch_solid_B(D, st);
  launch_parts_range(D, st);
  launch_refresh_vmax(D, st);
  if ((rc = check_launch(ctx, "reference configuration")) != SPH_OK) return fail(rc);
  HIPCHK_INIT(hipStreamSynchronize(st));
  // reference pair counts per scene
  if (P.ns) {
    std::vector<int> cnt(P.ns);
    HIPCHK_INIT(hipMemcpy(cnt.data(), D.s_cnt, sizeof(int) * P.ns, hipMemcpyDeviceToHost));
    std::vector<SceneState> stv(n_scenes);
    HIPCHK_INIT(hipMemcpy(stv.data(), D.st, sizeof(SceneState) * n_scenes, hipMemcpyDeviceToHost));
    for (int s = 0; s < n_scenes; ++s) {
      unsigned long long tot = 0;
      for (int a = 0; a < P.par[s].s_count; ++a) tot += cnt[P.par[s].s_begin + a];
      stv[s].n_ss = tot;
      if (stv[s].err & ERR_CAPACITY) {
        std::snprintf(ctx->err, sizeof ctx->err, "solid neighbour table overflow in scene %d (max_solid_nbr %d)", s,
                      P.maxn);
        return fail(SPH_E_CAPACITY);
      }
    }
    HIPCHK_INIT(hipMemcpy(D.st, stv.data(), sizeof(SceneState) * n_scenes, hipMemcpyHostToDevice));
  }
  // compact reference table (3D): where every scene's solid is a lattice of
  // one spacing, smoothing length and volume, and every pair matches its
  // offset class
  D.nbr_compact = 0;
  if (P.dim == 3 && P.ns > 0 && (size_t)P.ns < ((size_t)1 << 25)) {
    int s0 = -1;
    bool same = true;
    for (int s = 0; s < n_scenes; ++s) {
      const ScenePar &q = P.par[s];
      if (q.s_count == 0) continue;
      if (s0 < 0) s0 = s;
      else same = same && q.dps == P.par[s0].dps && q.hs == P.par[s0].hs && q.Vs == P.par[s0].Vs;
    }
    if (same && s0 >= 0) {
      int flag = 1;
      HIPCHK_INIT(hipMemcpy(D.nbc_ok, &flag, sizeof(int), hipMemcpyHostToDevice));
      launch_solid_classes(D, s0, st);
      for (int s = 0; s < n_scenes; ++s) launch_solid_compact(D, s, P.par[s].s_count, st);
      HIPCHK_INIT(hipStreamSynchronize(st));
      HIPCHK_INIT(hipMemcpy(&flag, D.nbc_ok, sizeof(int), hipMemcpyDeviceToHost));
      if (flag) {
        launch_solid_gsum_classes(D, st);
        HIPCHK_INIT(hipStreamSynchronize(st));
        D.nbr_compact = 1;
      }
      if ((rc = check_launch(ctx, "compact reference table")) != SPH_OK) return fail(rc);
    }
  }
  // lattice blocks: on where the compact table is and every free particle's
  // reference neighbours are exactly the lattice points at the offsets of
  // nonzero class gradient (those the table holds are among them, so equal
  // counts suffice)
  D.lat_ncls = D.lat_nblocks = D.lat_ncells = D.lat_jitter = 0;
  // a solid near a lattice without the compact table: the passes form each
  // pair's gradient from its lattice vector and the two particles' offsets
  // (every scene with solid of one spacing, smoothing length and volume)
  int s_ref = -1;
  bool same = true;
  for (int s = 0; s < n_scenes; ++s) {
    const ScenePar &q = P.par[s];
    if (q.s_count == 0) continue;
    if (s_ref < 0) s_ref = s;
    else same = same && q.dps == P.par[s_ref].dps && q.hs == P.par[s_ref].hs && q.Vs == P.par[s_ref].Vs;
  }
  const bool jitter = !D.nbr_compact && same && s_ref >= 0;
  if (P.dim == 3 && !P.lat_blocks.empty() && (D.nbr_compact || jitter)) {
    std::vector<float4> g(kNbrClasses);
    std::vector<int> cnt(P.ns);
    HIPCHK_INIT(hipMemcpy(g.data(), D.s_gcls, sizeof(float4) * kNbrClasses, hipMemcpyDeviceToHost));
    HIPCHK_INIT(hipMemcpy(cnt.data(), D.s_cnt, sizeof(int) * P.ns, hipMemcpyDeviceToHost));
    std::vector<float4> cls;
    std::vector<std::array<int, 3>> off;  // along the lattice axes
    const double dps = jitter ? P.par[s_ref].dps : 0.0, hs = jitter ? P.par[s_ref].hs : 0.0;
    // offsets that a pair can reach within 2 h_S with the largest offsets found
    const double reach = 2.0 * hs + 2.0 * std::sqrt(3.0) * P.lat_jit_max * dps;
    for (int c = 0; c < 125; ++c) {
      const int o[3] = {c / 25 - 2, (c / 5) % 5 - 2, c % 5 - 2};
      const double ol = std::sqrt((double)(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]));
      if (jitter ? (ol == 0.0 || ol * dps >= reach) : (g[c].x == 0.0f && g[c].y == 0.0f && g[c].z == 0.0f))
        continue;
      const int q[3] = {o[P.lat_axis[0]], o[P.lat_axis[1]], o[P.lat_axis[2]]};
      const int shift = q[1] * kLatRow + q[0] * kLatH2 + q[2];
      float sf;
      std::memcpy(&sf, &shift, sizeof sf);
      if (jitter)
        cls.push_back(make_float4((float)(-o[0] * dps), (float)(-o[1] * dps), (float)(-o[2] * dps), sf));
      else
        cls.push_back(make_float4(g[c].x, g[c].y, g[c].z, sf));
      off.push_back({q[0], q[1], q[2]});
    }
    // every free particle's table row holds exactly the existing lattice
    // neighbours at those offsets (the compact table's are among them; with
    // offsets, those within 2 h_S, none within 1e-4 of it)
    bool ok = !cls.empty();
    for (int s = 0; s < n_scenes && ok; ++s) {
      const ScenePar &p = P.par[s];
      const int4 L = P.lat_scene[s];
      const double *xs = scenes[s].x_solid;
      for (int i = 0; i < p.s_count - p.s_nclamp && ok; ++i) {
        const int a = p.s_begin + i;
        const int *c = &P.lat_cell[3 * (size_t)a];
        const int c0 = c[P.lat_axis[0]], c1 = c[P.lat_axis[1]], c2 = c[P.lat_axis[2]];
        int hits = 0;
        for (const auto &q : off) {
          const int x0 = c0 + q[0], x1 = c1 + q[1], x2 = c2 + q[2];
          if (x0 < 0 || x0 >= L.y || x1 < 0 || x1 >= L.z || x2 < 0 || x2 >= L.w) continue;
          const int b = P.lat_grid[L.x + ((size_t)x0 * L.z + x1) * L.w + x2];
          if (b < 0) continue;
          if (!jitter) {
            ++hits;
            continue;
          }
          double r2 = 0.0;
          for (int k = 0; k < 3; ++k) {
            const double d = xs[3 * (size_t)i + k] - xs[3 * (size_t)(b - p.s_begin) + k];
            r2 += d * d;
          }
          const double cut = 4.0 * hs * hs;
          ok = ok && std::fabs(r2 - cut) > 1e-4 * cut;
          hits += r2 < cut;
        }
        ok = ok && hits == cnt[a];
      }
    }
    if (ok) {
      // each particle's cell; the FP32 records move to cell order (the first
      // solid pass of every step writes every particle's)
      std::vector<int> of(P.ns);
      for (int s = 0; s < n_scenes; ++s) {
        const ScenePar &p = P.par[s];
        const int4 L = P.lat_scene[s];
        for (int i = 0; i < p.s_count; ++i) {
          const int a = p.s_begin + i;
          const int *c = &P.lat_cell[3 * (size_t)a];
          of[a] = L.x + ((c[P.lat_axis[0]] * L.z) + c[P.lat_axis[1]]) * L.w + c[P.lat_axis[2]];
        }
      }
      const size_t nrec = std::max((size_t)P.ns, P.lat_grid.size());
      HIPCHK_INIT(hipMemcpy(D.lat_of, of.data(), sizeof(int) * P.ns, hipMemcpyHostToDevice));
      HIPCHK_INIT(hipMemset(D.s_PBf, 0, sizeof(float) * 9 * nrec));
      HIPCHK_INIT(hipMemset(D.s_vf, 0, sizeof(float4) * nrec));
      D.lat_ncells = (int)P.lat_grid.size();
      HIPCHK_INIT(hipMemcpy(D.lat_grid, P.lat_grid.data(), sizeof(int) * P.lat_grid.size(), hipMemcpyHostToDevice));
      HIPCHK_INIT(
          hipMemcpy(D.lat_scene, P.lat_scene.data(), sizeof(int4) * P.lat_scene.size(), hipMemcpyHostToDevice));
      HIPCHK_INIT(
          hipMemcpy(D.lat_blocks, P.lat_blocks.data(), sizeof(int4) * P.lat_blocks.size(), hipMemcpyHostToDevice));
      HIPCHK_INIT(hipMemcpy(D.lat_cls, cls.data(), sizeof(float4) * cls.size(), hipMemcpyHostToDevice));
      D.lat_ncls = (int)cls.size();
      D.lat_nblocks = (int)P.lat_blocks.size();
      if (jitter) {
        // each particle's offset from its lattice point, in cell order
        std::vector<float> jc((size_t)3 * P.lat_grid.size(), 0.0f);
        for (int a = 0; a < P.ns; ++a)
          for (int k = 0; k < 3; ++k) jc[(size_t)k * P.lat_grid.size() + of[a]] = P.lat_jit[3 * (size_t)a + k];
        HIPCHK_INIT(hipMemcpy(D.lat_jit, jc.data(), sizeof(float) * jc.size(), hipMemcpyHostToDevice));
        D.lat_jitter = 1;
      }
    }
  }
#undef HIPCHK_INIT
  ctx->prebin = 1;  // every scene starts with a rebuild
  *out = ctx;
  return SPH_OK;
}

int neighbor_build(sph_ctx *ctx) {
  if (!ctx) return SPH_E_ORDER;
  // at a step boundary, or again after itself (a no-op then: nothing is due)
  int rc = ctx->phase == 1 ? SPH_OK : check_phase(ctx, "neighbor_build", 0);
  if (rc != SPH_OK) return rc;
  launch_rebuild(ctx->D, ctx->cfg, ctx->stream, true);
  rc = check_launch(ctx, "neighbor_build");
  if (rc == SPH_OK) ctx->phase = 1;
  ctx->features_taken = 0;
  return rc;
}

int fluid_step(sph_ctx *ctx) {
  if (!ctx) return SPH_E_ORDER;
  int rc = check_phase(ctx, "fluid_step", 1);
  if (rc != SPH_OK) return rc;
  launch_fluid_force(ctx->D, ctx->cfg, ctx->stream);
  launch_fluid_continuity(ctx->D, ctx->cfg, ctx->stream, false);
  rc = check_launch(ctx, "fluid_step");
  if (rc == SPH_OK) ctx->phase = 2;
  return rc;
}

int couple(sph_ctx *ctx) {
  if (!ctx) return SPH_E_ORDER;
  int rc = check_phase(ctx, "couple", 2);
  if (rc != SPH_OK) return rc;
  launch_couple(ctx->D, ctx->cfg, ctx->stream);
  rc = check_launch(ctx, "couple");
  if (rc == SPH_OK) ctx->phase = 3;
  return rc;
}

int solid_substeps(sph_ctx *ctx) {
  if (!ctx) return SPH_E_ORDER;
  int rc = check_phase(ctx, "solid_substeps", 3);
  if (rc != SPH_OK) return rc;
  rc = enqueue_solid(ctx, true);
  if (rc != SPH_OK) return rc;
  launch_step_end(ctx->D, ctx->stream, ctx->cfg.solid_ppt > 0);
  rc = check_launch(ctx, "solid_substeps");
  if (rc == SPH_OK) ctx->phase = 0;
  return rc;
}

int sph_advance(sph_ctx *ctx, int n_steps) {
  if (!ctx) return SPH_E_ORDER;
  if (n_steps < 0) return SPH_E_ARG;
  if (check_phase(ctx, "sph_advance", 0) != SPH_OK) return SPH_E_ORDER;
  if (n_steps > 0) ctx->features_taken = 0;
  // the streamed solid path reads kappa back to the host: no graph then
  if (!ctx->graph_exec && !ctx->graph_failed && ctx->stream && ctx->cfg.solid_ppt > 0) {
    // capture one acoustic step; every decision inside it is taken on the device
    hipError_t e = hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      enqueue_step(ctx, true);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(ctx->stream, &g);
      if (e == hipSuccess && g) {
        hipGraphExec_t ge = nullptr;
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (e == hipSuccess) {
          ctx->graph = g;
          ctx->graph_exec = ge;
        } else {
          (void)hipGraphDestroy(g);
        }
      }
    }
    if (!ctx->graph_exec) {
      ctx->graph_failed = 1;
      (void)hipGetLastError();
    }
  }
  // rebuilds set from the host are binned (and scanned) here; the steps do
  // that at their end for the rebuilds they decide themselves
  if (ctx->prebin && n_steps > 0) {
    launch_prebin(ctx->D, ctx->stream);
    ctx->prebin = 0;
  }
  for (int k = 0; k < n_steps; ++k) {
    if (ctx->graph_exec) {
      HIPCHK(hipGraphLaunch(ctx->graph_exec, ctx->stream));
    } else {
      int rc = enqueue_step(ctx, false);
      if (rc != SPH_OK) return rc;
    }
  }
  return SPH_OK;
}

int sph_read(sph_ctx *ctx, int field, int scene, double *host) {
  if (!ctx) return SPH_E_ORDER;
  if (scene < 0 || scene >= ctx->n_scenes || !host) return SPH_E_ARG;
  int w = field_width(ctx->dim, field);
  if (!w) return SPH_E_ARG;
  const ScenePar &p = ctx->par[scene];
  int n = field < 10 ? p.f_count : p.s_count;
  if (n == 0) return SPH_OK;
  launch_read(ctx->D, scene, field, n, ctx->D.stage, ctx->stream);
  int rc = check_launch(ctx, "sph_read");
  if (rc != SPH_OK) return rc;
  HIPCHK(hipMemcpyAsync(host, ctx->D.stage, sizeof(double) * w * (size_t)n, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return SPH_OK;
}

int sph_write(sph_ctx *ctx, int field, int scene, const double *host) {
  if (!ctx) return SPH_E_ORDER;
  if (check_phase(ctx, "sph_write", 0) != SPH_OK) return SPH_E_ORDER;
  ctx->kappa_ready = 0;  // the state may change: the next step reads kappa at its solid phase
  if (scene < 0 || scene >= ctx->n_scenes || !host) return SPH_E_ARG;
  static const int writable[] = {SPH_F_X, SPH_F_V, SPH_F_RHO, SPH_F_DRHO, SPH_S_U, SPH_S_V,
                                 SPH_S_A, SPH_S_F, SPH_S_DF, SPH_S_VBAR, SPH_S_ABAR};
  bool ok = false;
  for (int f : writable) ok |= (f == field);
  if (!ok) return SPH_E_ARG;
  int w = field_width(ctx->dim, field);
  const ScenePar &p = ctx->par[scene];
  int n = field < 10 ? p.f_count : p.s_count;
  if (n == 0) return SPH_OK;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->D.stage, host, sizeof(double) * w * (size_t)n, hipMemcpyHostToDevice, ctx->stream));
  launch_write(ctx->D, scene, field, n, ctx->D.stage, ctx->stream);
  // the step-end binning copied the fluid state: a scene binned before this
  // write is binned again when its rebuild starts
  if (field != SPH_F_RHO && field != SPH_F_DRHO) launch_set_rebuild(ctx->D, scene, ctx->stream);
  else launch_unbin(ctx->D, scene, ctx->stream);
  ctx->prebin = 1;
  if (field == SPH_F_V || (ctx->D.any_single && (field == SPH_S_V || field == SPH_S_A)))
    launch_refresh_vmax(ctx->D, ctx->stream);
  int rc = check_launch(ctx, "sph_write");
  if (rc != SPH_OK) return rc;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return SPH_OK;
}

int sph_scalars(sph_ctx *ctx, int scene, double *out) {
  if (!ctx) return SPH_E_ORDER;
  if (scene < 0 || scene >= ctx->n_scenes || !out) return SPH_E_ARG;
  std::vector<SceneState> st;
  int rc = read_states(ctx, st);
  if (rc != SPH_OK) return rc;
  const SceneState &S = st[scene];
  float vm;
  std::memcpy(&vm, &S.vmax_prev, sizeof vm);
  double v[8] = {S.t, S.dt_ac, S.dt_ad, S.dt_s, S.adv_accum, (double)S.kappa, (double)S.need_rebuild, (double)vm};
  std::memcpy(out, v, sizeof v);
  return SPH_OK;
}

int sph_set_scalars(sph_ctx *ctx, int scene, const double *in) {
  if (!ctx) return SPH_E_ORDER;
  if (check_phase(ctx, "sph_set_scalars", 0) != SPH_OK) return SPH_E_ORDER;
  ctx->kappa_ready = 0;  // the state may change: the next step reads kappa at its solid phase
  if (scene < 0 || scene >= ctx->n_scenes || !in) return SPH_E_ARG;
  std::vector<SceneState> st;
  int rc = read_states(ctx, st);
  if (rc != SPH_OK) return rc;
  SceneState &S = st[scene];
  S.t = in[0];
  S.dt_ad = in[2];
  S.adv_accum = in[4];
  const int was = S.need_rebuild;
  S.need_rebuild = in[6] != 0.0;
  if (S.binned && !S.need_rebuild) {  // a withdrawn rebuild gives back its binning
    launch_unbin(ctx->D, scene, ctx->stream);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    S.binned = 0;
  }
  if (S.need_rebuild && !was) ctx->prebin = 1;
  HIPCHK(hipMemcpy(ctx->D.st + scene, &S, sizeof(SceneState), hipMemcpyHostToDevice));
  if (S.need_rebuild != was) {  // keep the count of set flags (the stream is idle here)
    int cnt = 0;
    HIPCHK(hipMemcpy(&cnt, ctx->D.rebuild_count, sizeof(int), hipMemcpyDeviceToHost));
    cnt += S.need_rebuild - was;
    HIPCHK(hipMemcpy(ctx->D.rebuild_count, &cnt, sizeof(int), hipMemcpyHostToDevice));
  }
  return SPH_OK;
}

int sph_counters(sph_ctx *ctx, int scene, unsigned long long *out) {
  if (!ctx) return SPH_E_ORDER;
  if (scene < -1 || scene >= ctx->n_scenes || !out) return SPH_E_ARG;
  std::vector<SceneState> st;
  int rc = read_states(ctx, st);
  if (rc != SPH_OK) return rc;
  unsigned long long o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int s = 0; s < ctx->n_scenes; ++s) {
    if (scene >= 0 && s != scene) continue;
    const SceneState &S = st[s];
    unsigned long long v[8] = {S.n_ff, S.n_fw, S.n_fs, S.n_ss, S.steps, S.rebuilds, S.substeps, S.interactions};
    for (int k = 0; k < 8; ++k) o[k] += v[k];
  }
  std::memcpy(out, o, sizeof o);
  return SPH_OK;
}

int sph_set_surrogate(sph_ctx *ctx, mlp_ctx *net, const float *stats, float threshold, int every) {
  if (!ctx) return SPH_E_ORDER;
  if (check_phase(ctx, "sph_set_surrogate", 0) != SPH_OK) return SPH_E_ORDER;
  ctx->kappa_ready = 0;  // the state may change: the next step reads kappa at its solid phase
  if (net == nullptr || !(threshold > 0.0f)) {
    ctx->net = nullptr;
    ctx->D.sur_thr = 0.0f;
  } else {
    if (!stats || ctx->dim != 2 || ctx->cfg.solid_ppt <= 0 || net->D.in_dim != kSurFeat ||
        net->D.out_dim != kSurOut || net->D.max_rows < ctx->D.ns || ctx->D.ns == 0 || every < 1 ||
        every > (1 << 20))
      return SPH_E_ARG;
    HIPCHK(allow_sur_net_lds());
    HIPCHK(hipMemcpyAsync(ctx->D.sur_stats, stats, sizeof(float) * (2 * kSurFeat + 2 * kSurOut),
                          hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    ctx->net = net;
    ctx->D.sur_thr = threshold;
    ctx->D.sur_every = every;
    // the first step with the network is a judge step
    std::vector<SceneState> st;
    int rc = read_states(ctx, st);
    if (rc != SPH_OK) return rc;
    for (SceneState &x : st) {
      x.sur = 0;
      x.sur_window = 0;
      x.sur_countdown = 0;
      x.sur_last_r = std::nan("");
    }
    HIPCHK(hipMemcpy(ctx->D.st, st.data(), sizeof(SceneState) * ctx->n_scenes, hipMemcpyHostToDevice));
  }
  // the captured step no longer matches: capture again at the next sph_advance
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  ctx->graph_exec = nullptr;
  ctx->graph = nullptr;
  ctx->graph_failed = 0;
  return SPH_OK;
}

int sph_solid_features(sph_ctx *ctx, const float *stats_dev, float *x_dev) {
  if (!ctx) return SPH_E_ORDER;
  if (check_phase(ctx, "sph_solid_features", 3) != SPH_OK) return SPH_E_ORDER;
  if (!x_dev || ctx->dim != 2) return SPH_E_ARG;
  launch_sur_features(ctx->D, stats_dev, x_dev, ctx->stream);
  int rc = check_launch(ctx, "sph_solid_features");
  if (rc == SPH_OK) ctx->features_taken = 1;
  return rc;
}

int sph_solid_targets(sph_ctx *ctx, float *t_dev) {
  if (!ctx) return SPH_E_ORDER;
  if (check_phase(ctx, "sph_solid_targets", 0) != SPH_OK) return SPH_E_ORDER;
  if (!ctx->features_taken) {
    std::snprintf(ctx->err, sizeof ctx->err,
                  "sph_solid_targets: no sph_solid_features in this step (call it between couple and solid_substeps)");
    return SPH_E_ORDER;
  }
  if (!t_dev || ctx->dim != 2) return SPH_E_ARG;
  launch_sur_targets(ctx->D, t_dev, ctx->stream);
  ctx->features_taken = 0;
  return check_launch(ctx, "sph_solid_targets");
}

int sph_surrogate_counters(sph_ctx *ctx, int scene, unsigned long long *out) {
  if (!ctx) return SPH_E_ORDER;
  if (scene < -1 || scene >= ctx->n_scenes || !out) return SPH_E_ARG;
  std::vector<SceneState> st;
  int rc = read_states(ctx, st);
  if (rc != SPH_OK) return rc;
  out[0] = out[1] = out[2] = out[3] = 0;
  for (int s = 0; s < ctx->n_scenes; ++s) {
    if (scene >= 0 && s != scene) continue;
    out[0] += st[s].sur_ok;
    out[1] += st[s].sur_fallback;
    out[2] += st[s].sur_judge_ok;
    out[3] += st[s].sur_judge_fail;
  }
  return SPH_OK;
}

int sph_surrogate_residual(sph_ctx *ctx, int scene, double *out) {
  if (!ctx) return SPH_E_ORDER;
  if (scene < 0 || scene >= ctx->n_scenes || !out) return SPH_E_ARG;
  std::vector<SceneState> st;
  int rc = read_states(ctx, st);
  if (rc != SPH_OK) return rc;
  *out = st[scene].sur_last_r;
  return SPH_OK;
}

int sph_launch_config(sph_ctx *ctx, int *out) {
  if (!ctx) return SPH_E_ORDER;
  if (!out) return SPH_E_ARG;
  const LaunchCfg &c = ctx->cfg;
  int v[10] = {c.lpp_force, c.lpp_couple, c.block_pair, c.solid_ppt, c.block_solid, ctx->D.capf, ctx->D.capb,
               ctx->graph_exec ? 1 : 0, c.solid_parts, ctx->D.n_parts_blocks};
  std::memcpy(out, v, sizeof v);
  return SPH_OK;
}

int sph_fluid_tiles(sph_ctx *ctx, long long *out) {
  if (!ctx) return SPH_E_ORDER;
  if (!out) return SPH_E_ARG;
  const Dev &D = ctx->D;
  const int groups = D.tile_gp ? (D.nf + D.tile_gp - 1) / D.tile_gp : 0;
  long long v[5] = {D.tile_gp, groups, 0, 0, 0};
  if (groups) {
    std::vector<int> cnt(groups);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipMemcpy(cnt.data(), D.t_count, sizeof(int) * groups, hipMemcpyDeviceToHost));
    for (int c : cnt)
      if (c >= 0) {
        v[2] += 1;
        v[3] += c;
        v[4] = std::max<long long>(v[4], c);
      }
  }
  std::memcpy(out, v, sizeof v);
  return SPH_OK;
}

int sph_solid_table(sph_ctx *ctx, int *out) {
  if (!ctx) return SPH_E_ORDER;
  if (!out) return SPH_E_ARG;
  const int compact = ctx->D.nbr_compact;
  int v[5] = {compact, ctx->D.maxn, compact ? (int)sizeof(unsigned) : (int)sizeof(float4), ctx->D.lat_nblocks,
              ctx->D.lat_ncls};
  std::memcpy(out, v, sizeof v);
  return SPH_OK;
}

int sph_reduce(sph_ctx *ctx, int scene, double *out) {
  if (!ctx) return SPH_E_ORDER;
  if (scene < 0 || scene >= ctx->n_scenes || !out) return SPH_E_ARG;
  const ScenePar &p = ctx->par[scene];
  int n = std::max(p.f_count, p.s_count);
  int nb = std::max(1, std::min(1024, (n + 255) / 256));
  double *dst = ctx->D.stage;
  launch_reduce(ctx->D, scene, nb, ctx->D.red, dst, ctx->stream);
  int rc = check_launch(ctx, "sph_reduce");
  if (rc != SPH_OK) return rc;
  double buf[16];
  HIPCHK(hipMemcpyAsync(buf, dst, sizeof buf, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::memcpy(out, buf, 15 * sizeof(double));
  return SPH_OK;
}

int sph_reduce_noalloc(sph_ctx *ctx, int scene, int blocks, double *out_dev) {
  if (!ctx) return SPH_E_ORDER;
  if (scene < 0 || scene >= ctx->n_scenes || !out_dev) return SPH_E_ARG;
  if (blocks < 0 || blocks > kReduceScratchBlocks) {
    std::snprintf(ctx->err, sizeof ctx->err,
                  "sph_reduce_noalloc: %d blocks asked, the static scratch holds the partials of at most %d", blocks,
                  kReduceScratchBlocks);
    return SPH_E_ARG;
  }
  if (!ctx->red_scratch) {
    std::snprintf(ctx->err, sizeof ctx->err, "sph_reduce_noalloc: the static scratch has no device address");
    return SPH_E_HIP;
  }
  const ScenePar &p = ctx->par[scene];
  int n = std::max(p.f_count, p.s_count);
  int nb = blocks > 0 ? blocks : std::max(1, std::min(kReduceScratchBlocks, (n + 255) / 256));
  launch_reduce(ctx->D, scene, nb, ctx->red_scratch, out_dev, ctx->stream);
  return check_launch(ctx, "sph_reduce_noalloc");
}

int sph_pairs(sph_ctx *ctx, int which, int scene, int *start, int *idx) {
  if (!ctx) return SPH_E_ORDER;
  if (scene < 0 || scene >= ctx->n_scenes || !start || which < 0 || which > 3) return SPH_E_ARG;
  const ScenePar &p = ctx->par[scene];
  const Dev &D = ctx->D;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  // sorted fluid index (within the scene) -> original index
  std::vector<int> fid(p.f_count);
  if (p.f_count && which != 3)
    HIPCHK(hipMemcpy(fid.data(), D.f_id + p.f_begin, sizeof(int) * p.f_count, hipMemcpyDeviceToHost));
  std::vector<std::vector<int>> rows;
  if (which <= 1) {
    const int n = p.f_count, lw = D.lw, cap = which == 0 ? D.capf : D.capb;
    const unsigned *list = which == 0 ? D.f_nbl : D.f_bnl;
    rows.resize(n);
    std::vector<int2> len(n);
    std::vector<unsigned> ent((size_t)n * cap);
    std::vector<int> bsrc(which == 1 ? p.b_count : 0);
    if (n) {
      HIPCHK(hipMemcpy(len.data(), D.f_rowlen + p.f_begin, sizeof(int2) * n, hipMemcpyDeviceToHost));
      // the scene's entries of chunk c (lw entries per particle) are contiguous
      for (int c = 0; c < cap / lw; ++c)
        HIPCHK(hipMemcpy(ent.data() + (size_t)c * n * lw, list + ((size_t)c * D.nf + p.f_begin) * lw,
                         sizeof(unsigned) * (size_t)n * lw, hipMemcpyDeviceToHost));
    }
    if (!bsrc.empty())
      HIPCHK(hipMemcpy(bsrc.data(), D.b_src + p.b_begin, sizeof(int) * p.b_count, hipMemcpyDeviceToHost));
    for (int k = 0; k < n; ++k) {
      int L = std::min(which == 0 ? len[k].x : len[k].y, cap);
      std::vector<int> &r = rows[fid[k]];
      for (int e = 0; e < L; ++e) {
        int j = (int)(ent[((size_t)(e / lw) * n + k) * lw + e % lw] & ((1u << 27) - 1u));
        r.push_back(which == 0 ? fid[j - p.f_begin] : bsrc[j - p.b_begin]);
      }
    }
  } else {
    const int n = which == 2 ? p.s_count - p.s_nclamp : p.s_count;
    rows.resize(n);
    if (n) {
      std::vector<int> cnt(n);
      HIPCHK(hipMemcpy(cnt.data(), which == 2 ? D.s_cpl_cnt + p.s_begin : D.s_cnt + p.s_begin, sizeof(int) * n,
                       hipMemcpyDeviceToHost));
      int cap = which == 2 ? D.capf : D.maxn, used = 0;
      for (int a = 0; a < n; ++a) used = std::max(used, std::min(cnt[a], cap));
      for (int q = 0; q < used; ++q) {
        std::vector<int> col(n);
        if (which == 2) {
          HIPCHK(hipMemcpy(col.data(), D.s_cpl + (size_t)q * D.ns + p.s_begin, sizeof(int) * n,
                           hipMemcpyDeviceToHost));
        } else {
          std::vector<float4> g(n);
          HIPCHK(hipMemcpy(g.data(), D.s_nbr + (size_t)q * D.ns + p.s_begin, sizeof(float4) * n,
                           hipMemcpyDeviceToHost));
          for (int a = 0; a < n; ++a) std::memcpy(&col[a], &g[a].w, sizeof(int));
        }
        for (int a = 0; a < n; ++a)
          if (q < std::min(cnt[a], cap))
            rows[a].push_back(which == 2 ? fid[(col[a] & ((1 << 27) - 1)) - p.f_begin] : col[a] - p.s_begin);
      }
    }
  }
  int total = 0;
  start[0] = 0;
  for (size_t a = 0; a < rows.size(); ++a) {
    std::sort(rows[a].begin(), rows[a].end());
    if (idx) std::memcpy(idx + total, rows[a].data(), sizeof(int) * rows[a].size());
    total += (int)rows[a].size();
    start[a + 1] = total;
  }
  return total;
}

int sph_sync(sph_ctx *ctx) {
  if (!ctx) return SPH_E_ORDER;
  std::vector<SceneState> st;
  int rc = read_states(ctx, st);
  if (rc != SPH_OK) return rc;
  for (int s = 0; s < ctx->n_scenes; ++s) {
    int e = st[s].err;
    if (e) {
      std::snprintf(ctx->err, sizeof ctx->err, "scene %d: %s%s%s%s%s%s", s,
                    (e & ERR_NAN_FLUID) ? "non-finite fluid state " : "",
                    (e & ERR_NAN_SOLID) ? "non-finite solid state " : "", (e & ERR_JACOBIAN) ? "det F <= 0 " : "",
                    (e & ERR_CAPACITY) ? "neighbour table overflow " : "",
                    (e & ERR_KAPPA) ? "fewer solid sub-step passes than kappa " : "",
                    (e & ERR_PARTS) ? "the solid's workgroups were not resident together" : "");
      // a state that blew up also crowds cells: instability takes precedence
      if (e & (ERR_NAN_FLUID | ERR_NAN_SOLID | ERR_JACOBIAN)) return SPH_E_UNSTABLE;
      if (e & ERR_CAPACITY) return SPH_E_CAPACITY;
      return (e & ERR_PARTS) ? SPH_E_HIP : SPH_E_ORDER;
    }
  }
  // info: a judge step rejected the network since the last sync
  unsigned long long fb = 0;
  for (int s = 0; s < ctx->n_scenes; ++s) fb += st[s].sur_judge_fail;
  if (fb > ctx->fallback_seen) {
    ctx->fallback_seen = fb;
    return SPH_FALLBACK;
  }
  return SPH_OK;
}

int sph_time_kernel(sph_ctx *ctx, int kernel, int reps, double *avg_ms) {
  if (!ctx) return SPH_E_ORDER;
  if (check_phase(ctx, "sph_time_kernel", 0) != SPH_OK) return SPH_E_ORDER;
  ctx->kappa_ready = 0;  // the state may change: the next step reads kappa at its solid phase
  if (reps <= 0 || !avg_ms || kernel < SPH_K_FLUID_FORCE || kernel > SPH_K_REBUILD) return SPH_E_ARG;
  hipStream_t st = ctx->stream;
  auto enqueue_one = [&]() -> int {
    switch (kernel) {
    case SPH_K_FLUID_FORCE: launch_fluid_force(ctx->D, ctx->cfg, st); break;
    case SPH_K_CONTINUITY: launch_fluid_continuity(ctx->D, ctx->cfg, st, false); break;
    case SPH_K_COUPLE: launch_couple(ctx->D, ctx->cfg, st); break;
    case SPH_K_SOLID: return enqueue_solid(ctx, false);
    case SPH_K_REBUILD:
      for (int s = 0; s < ctx->n_scenes; ++s) launch_set_rebuild(ctx->D, s, st);
      launch_rebuild(ctx->D, ctx->cfg, st, true);
      break;
    }
    return SPH_OK;
  };
  // The repetitions are captured into a graph and replayed twice, the first
  // replay untimed, so that the timed launches follow each other on the
  // device instead of at the host's launch rate.  The streamed solid form
  // reads kappa back once per repetition and is launched directly.
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  if (st && !(kernel == SPH_K_SOLID && ctx->cfg.solid_ppt == 0)) {
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      for (int r = 0; r < reps; ++r) (void)enqueue_one();
      if (hipStreamEndCapture(st, &g) == hipSuccess && g &&
          hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess)
        ge = nullptr;
    }
    if (!ge) (void)hipGetLastError();
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = SPH_OK;
  float ms = 0.0f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = SPH_E_HIP;
  } else if (ge) {
    if (hipGraphLaunch(ge, st) != hipSuccess || hipEventRecord(e0, st) != hipSuccess ||
        hipGraphLaunch(ge, st) != hipSuccess || hipEventRecord(e1, st) != hipSuccess)
      rc = SPH_E_HIP;
  } else if (hipEventRecord(e0, st) != hipSuccess) {
    rc = SPH_E_HIP;
  } else {
    for (int r = 0; r < reps && rc == SPH_OK; ++r) rc = enqueue_one();
    if (rc == SPH_OK && hipEventRecord(e1, st) != hipSuccess) rc = SPH_E_HIP;
  }
  if (rc == SPH_OK) rc = check_launch(ctx, "sph_time_kernel");
  if (rc == SPH_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = SPH_E_HIP;
  if (rc == SPH_E_HIP && !ctx->err[0]) std::snprintf(ctx->err, sizeof ctx->err, "sph_time_kernel: HIP call failed");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (ge) (void)hipGraphExecDestroy(ge);
  if (g) (void)hipGraphDestroy(g);
  // the forced rebuilds consumed their binning: the next steps bin again
  if (kernel == SPH_K_REBUILD) ctx->prebin = 1;
  *avg_ms = (double)ms / reps;
  return rc;
}

const char *sph_last_error(const sph_ctx *ctx) { return ctx ? ctx->err : "no context"; }

int sph_autotune(const sph_scene *scenes, int n_scenes, const sph_options *opt, void *dev_arena,
                 size_t arena_bytes, void *stream, int warmup, int steps, sph_options *best,
                 double *ms_per_step) {
  if (!scenes || !opt || !best || !dev_arena || n_scenes <= 0 || warmup < 0 || steps <= 0) return SPH_E_ARG;
  size_t need = sph_arena_bytes(scenes, n_scenes, opt);
  if (need == 0 || arena_bytes < need) return SPH_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return SPH_E_HIP;
  }
  const int lpps[] = {1, 2, 4, 8, 16}, blocks[] = {64, 128, 256};
  // (the split form of the block-resident solid kernel is not a candidate:
  // it measured slower on every workload, its exchanges writing back and
  // invalidating the L2 of each XCD; the caller's solid_parts is kept)
  std::vector<sph_options> cands;
  for (int serial = 0; serial < 2; ++serial)
    for (int lpp : lpps)
      for (int bp : blocks) {
        sph_options o = *opt;
        o.lanes_per_particle = lpp;
        o.block_pair = bp;
        o.serial_passes = serial;
        cands.push_back(o);
      }
  double best_ms = -1.0;
  sph_options pick = *opt;
  int rc = SPH_OK;
  for (size_t ci = 0; ci < cands.size() && rc == SPH_OK; ++ci) {
    const sph_options o = cands[ci];
    // two timed repetitions, the faster one counts (short runs are noisy);
    // each starts from a fresh context, so a trial never runs more than
    // warmup + steps steps of the scenes
    float ms = 0.0f;
    for (int rep = 0; rep < 2 && rc == SPH_OK; ++rep) {
      sph_ctx *ctx = nullptr;
      float m = 0.0f;
      rc = sph_init(scenes, n_scenes, &o, dev_arena, arena_bytes, stream, &ctx);
      if (rc == SPH_OK) rc = sph_advance(ctx, warmup);
      if (rc == SPH_OK && (hipStreamSynchronize(st) != hipSuccess || hipEventRecord(e0, st) != hipSuccess))
        rc = SPH_E_HIP;
      if (rc == SPH_OK) rc = sph_advance(ctx, steps);
      if (rc == SPH_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&m, e0, e1) != hipSuccess))
        rc = SPH_E_HIP;
      if (rc == SPH_OK) rc = sph_sync(ctx);
      if (ctx) sph_destroy(ctx);
      if (rc == SPH_OK) ms = rep == 0 ? m : std::min(ms, m);
    }
    if (rc != SPH_OK) break;
    const double per = (double)ms / steps;
    if (best_ms < 0.0 || per < best_ms) {
      best_ms = per;
      pick = o;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != SPH_OK) return rc;
  *best = pick;
  if (ms_per_step) *ms_per_step = best_ms;
  return SPH_OK;
}

void sph_destroy(sph_ctx *ctx) {
  if (!ctx) return;
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  if (ctx->ev_kappa) {
    (void)hipEventSynchronize(ctx->ev_kappa);  // any copy into st_host has landed
    (void)hipEventDestroy(ctx->ev_kappa);
  }
  if (ctx->st_host) (void)hipHostFree(ctx->st_host);
  delete ctx;
}

}  // extern "C"
