// Device-side data layout of the multi-resolution SPH FSI library.
//
// Every array lives in the caller's arena.  Fluid particles of all scenes are
// concatenated (scene s owns [f_begin, f_begin + f_count)) and, after each
// rebuild, sorted by cell of the scene's grid in Morton order.  Positions are
// stored as the integer cell of the last rebuild plus an offset from that
// cell's origin: FP64 for the state that integrates and for the
// number-density sum, an FP32 copy for the pair loops.  The fluid density is
// stored as eps = rho / rho0 - 1 and the deformation gradient as H = F - I.
// These keep FP32 sums accurate where the absolute values would cancel (pair
// distances, pressure from density, stress from strain).
#pragma once
#include <hip/hip_runtime.h>

namespace mrsph {

struct ScenePar {
  // particle ranges in the concatenated arrays
  int f_begin, f_count;  // fluid
  int w_begin, w_count;  // walls
  int s_begin, s_count, s_nclamp;  // solid (clamp block last)
  int b_begin, b_count;  // boundary sources: walls then free solid
  int cell_begin, ncell_total;
  int ncell[3];
  int periodic[3];
  float cs[3];         // cell size per axis (>= 2 h_F)
  double lo[3], csd[3];  // FP64 copies for conversions
  double len[3];       // box length per axis
  // fluid
  float hf, inv_hf, r2max_f, alpha_f;  // smoothing length, 1/h, (2h)^2, kernel normalisation
  float rho0, c, eta, gamma;
  float p_coef;       // rho0 c^2 / gamma
  float gam_inv_rho0c2;  // gamma / (rho0 c^2)
  float g[3];
  float Vf;           // dp_f^d (wall volume, reference volume in the number density)
  float psi0;         // number density of the unbounded lattice
  double psi0d, dpf, dps;  // FP64 copies for the number-density sum
  // solid
  float hs, inv_hs, r2max_s, alpha_s;
  float rho0s, mu, lam, c_s;
  float Vs;           // dp_s^d
  // time stepping
  float cfl_ac, cfl_ad, cfl_s, u_ref;
  double dt_visc;     // viscous bound of the advection step (0: none)
  // inflow buffer
  float in_U0, in_ts, in_H, in_len;
  int riemann, reinit;
  int material;     // 0 Neo-Hookean, 1 linear elastic (Kirchhoff)
  int single_step;  // 1: the solid step is the one step of fluid and solid (kappa = 1)
};

struct SceneState {
  double t, dt_ac, dt_ad, dt_s, adv_accum;
  int kappa, need_rebuild, err;
  int kappa_next;      // streamed solid: kappa of the next step, computed at this step's end for the host
  int kappa_next_err;  // the error bits that evaluation would latch (latched when the step adopts it)
  int binned;  // pending rebuild prepared at the end of the last step: 1 particles binned, 2 cells scanned too
  unsigned int vmax_prev, vmax_next;  // max fluid speed (float bits): step start / being reduced
  unsigned int smax_v, smax_a;        // max solid speed and acceleration (float bits) being reduced
  unsigned int send_v, send_a;        // single step: the same at the step end, for the next step's size
  unsigned long long n_ff, n_fw, n_fs, n_ss;  // pairs within support at the last rebuild
  unsigned long long steps, rebuilds, substeps, interactions;
  unsigned long long acc_ff, acc_fw, acc_fs;  // pair counts being reduced after a rebuild
  int base_f, base_b;  // cell-scan prefix at the scene's first cell (rebuild)
  // learned sub-step: mode of this step (0 surrogate off, 1 learned step, 2
  // judge step, 3 plain step), then the schedule the judge steps set: learned
  // steps left in the open window, plain steps left before the next judge
  int sur, sur_window, sur_countdown, pad3;
  unsigned long long sur_ok, sur_fallback;          // steps taken by the network / by the plain sub-steps
  unsigned long long sur_judge_ok, sur_judge_fail;  // judge steps passed / failed
  double sur_last_r;                                // residual R of the last judge step
  double dt_s_next;  // streamed solid: the solid step that goes with kappa_next
};

// mode of a scene's acoustic step while a learned sub-step network is set
enum SurMode { kSurOff = 0, kSurLearned = 1, kSurJudge = 2, kSurPlain = 3 };

// ERR_KAPPA: the streamed solid passes were launched fewer times than the
// scene's kappa (an inconsistency of the host's sub-step count);
// ERR_PARTS: a workgroup of a scene split over several waited at their
// exchange longer than the spin limit (they were not all resident)
enum ErrBits {
  ERR_NAN_FLUID = 1,
  ERR_NAN_SOLID = 2,
  ERR_JACOBIAN = 4,
  ERR_CAPACITY = 8,
  ERR_KAPPA = 16,
  ERR_PARTS = 32
};

// Device pointers, passed by value to every kernel.
struct Dev {
  int n_scenes, dim;
  ScenePar *par;
  SceneState *st;
  // fluid, sorted
  int nf;
  int *f_scene, *f_lin, *f_id;
  float4 *f_pos;   // frozen offset at the last rebuild (xyz), mass (w)
  double4 *f_off;  // current offset from the same cell origin (FP64: positions integrate here)
  double4 *f_posd; // frozen offset in FP64 (read by the number-density sum)
  float4 *f_va;    // (v, eps) at the step start
  float4 *f_vb;    // (v^{n+1}, eps^{n+1/2}) written by the force kernel
  float4 *f_vs;    // mid-point snapshot (v^n, eps^{n+1/2}): force pass and coupling on the solid
  float4 *f_acc;   // acceleration of the last step
  float *f_drho;   // d eps / dt kept for the next half step
  float *f_p;      // mid-step pressure
  int4 *f_nnb;     // fluid, wall and solid neighbours within 2 h_F at the last rebuild
  // Pair lists of the advection step (geometry is frozen between rebuilds):
  // entry = neighbour index | (relative cell id 0..26) << 27; rows are dense.
  // Entry e of particle i sits at ((e / lw) * nf + i) * lw + e % lw, so the
  // lw lanes sharing a particle read lw consecutive entries.
  int capf, capb, lw;
  int fluid_prep;  // 1: k_fluid_prep forms the mid-point snapshot before the force pass
  int any_single;  // 1: some scene takes one shared step (step-end solid maxima needed)
  int sort_blocks; // leading blocks of the force launch that order the coupling lists
  int couple_blocks; // leading blocks of the continuity launch that run the coupling on the solid
  int solid_step_end;    // 1: the block-resident solid launch also ends the step (hand-over, binning, reductions)
  int end_fluid_blocks;  // its blocks beside the scenes' that reduce the fluid's step end
  // the block-resident solid kernel split over several workgroups per scene:
  // per workgroup (scene, part, parts of the scene, 0); null: one per scene
  const int4 *solid_map;
  int solid_map_n;       // workgroups of the split form (the scenes' blocks of its launch)
  int4 *s_parts;         // the split form's map (set at sph_init)
  int n_parts_blocks;    // its workgroups
  unsigned *parts_sync;  // per scene: max |v| and |a| bits, barrier count, workgroups done
  double *s_xpb, *s_xv;  // exchange of P B (D^2 per particle) and v (D) between a scene's workgroups
  unsigned *f_nbl;  // fluid neighbours (capf entries per particle)
  unsigned *f_bnl;  // boundary neighbours: walls and free solid (capb per particle)
  int2 *f_rowlen;  // used length of each particle's two rows
  // Neighbour tiles of the fluid pair loops: group g is the tile_gp fluid
  // particles g tile_gp ... of one block of the force and continuity
  // launches; t_union holds the group's distinct fluid neighbours (sorted
  // indices, kTileCap per group), t_count[g] of them, and t_rows the group's
  // fluid rows as 16-bit entries (position in t_union, relative cell id) in
  // f_nbl's layout; t_count[g] = -1: no tile, the passes walk f_nbl.
  // tile_gp = 0: no tiles.
  int tile_gp;
  unsigned *t_union;
  int *t_count;
  unsigned short *t_rows;
  float *f_speed;  // |v| after the last continuity pass (reduced per scene by the solid kernel)
  // fluid rebuild scratch (indexed by the old sorted index)
  int *fs_lin, *fs_slot, *fs_id, *f_perm, *f_pkey;
  double4 *fs_off;
  float4 *fs_va;
  float *fs_drho, *fs_m;
  // cells
  int ncell;
  int *fc_count, *bc_count, *cell_scene;
  int *rank_to_cell;  // cell of each Morton rank (the scene's cell_begin + its linear index)
  int2 *cell_part;  // per-tile sums and then exclusive prefixes of the cell scan
  int2 *fc_se, *bc_se;  // [start, end) of each cell, indexed by scene-local linear index + cell_begin
  // walls (static)
  int nw;
  int *w_lin, *w_scene;
  double4 *w_off;
  float4 *w_nrm;
  // boundary particles seen by the fluid (walls + free solid), sorted by cell
  int nb;
  float4 *b_pos;   // frozen offset (xyz), volume (w)
  float4 *b_vbar;  // averaged velocity (xyz), max(0, (abar - g).n) (w)
  float4 *b_nrm;   // normal (xyz), +V_ref for walls / -V_ref for solid (w)
  double4 *b_posd; // frozen offset in FP64
  int *b_perm, *bs_lin, *bs_slot, *bs_scene;
  int *b_solid;  // per boundary slot: its solid particle, or -1 for a wall
  int *b_src;    // per boundary slot: its source index within the scene (walls first, then free solid)
  double4 *bs_off;
  // solid (per scene in original order), SoA with component stride ns
  int ns, maxn;
  int *s_scene, *s_lin0, *s_bslot, *s_blin, *s_cnt;
  double *s_off0;  // reference offset from the reference cell, FP64
  double *s_u, *s_v, *s_du, *s_dv;  // integration state in FP64 (displacement, velocity, step increments)
  double *s_H, *s_dF, *s_B;        // H = F - I, dF/dt, B in FP64 (d*d components)
  double *s_PBg;                   // P_a B_a sum_b g_ab in FP64, [k * ns + a]: the own term of the momentum
                                   // sum, formed where P B is (the stress pass), read by the momentum pass
  float *s_PBf;                    // the same rounded to FP32: what the streamed momentum pass gathers
  // compact reference table of lattice reference configurations (3D): per
  // pair the neighbour's index << 7 | its offset class, [q * ns + a]; the
  // classes' gradients in s_gcls (one table for the context)
  unsigned *s_nbc;
  float4 *s_gcls;
  int *nbc_ok;                     // set-up: stays 1 while every pair matches its class
  int nbr_compact;                 // 1: the streamed solid passes walk s_nbc
  // lattice blocks of the streamed solid passes (3D): every scene's solid on
  // one lattice whose reference neighbours are exactly its points within 2 h_S.
  // Lattice axes are ordered slowest to fastest in storage; lat_grid maps a
  // scene's bounding box of cells, [(c0 * L1 + c1) * L2 + c2] from offset
  // lat_scene[s].x with (L0, L1, L2) in .y .z .w, to the particle there or -1;
  // lat_blocks[i] = (scene, first cell per axis) of a block of kLatB0 x kLatB1
  // x kLatB2 cells holding a free particle; lat_cls[j] = (the class gradient
  // in xyz, the offset's position shift in a block's LDS halo as int bits in
  // w) for the lat_ncls classes of nonzero gradient: one uniform 16-byte load
  // per class.  lat_nblocks = 0: the passes walk the pair table.
  // On lattice blocks s_PBf and s_vf are indexed by grid cell (lat_ncells of
  // them; empty cells hold zeros, a particle's velocity record has w = 1) and
  // lat_of[a] is particle a's cell.
  int *lat_grid, *lat_of;
  int4 *lat_scene, *lat_blocks;
  float4 *lat_cls;
  int lat_ncls, lat_nblocks, lat_ncells;
  // lat_jitter = 1: the solid is near a lattice but not on it (no compact
  // table); lat_cls[j] then holds the class's lattice vector -o dp_S (xyz)
  // and its shift, lat_jit[k * lat_ncells + cell] each particle's offset from
  // its lattice point (zero in empty cells), and the passes form each pair's
  // gradient from the two.
  int lat_jitter;
  float *lat_jit;
  float4 *s_vf;                    // v rounded to FP32, one 16-byte record per particle: what the streamed
                                   // rate pass gathers (free particles: written by the momentum pass of the
                                   // same sub-step; clamped ones: by the first pass of the step)
  float *s_a, *s_fF, *s_vbar, *s_abar, *s_n0, *s_n;
  float *s_fFp;                    // pressure part of the coupling force
  int *s_cpl_cnt;                  // fluid neighbours of each free solid particle (set at rebuilds)
  unsigned *s_cpl;                 // [e * ns + a]: fluid index | (cell offset id << kNbrBits), ascending
  // sub-step surrogate (2D)
  float *sur_stats;                // feature mean[24], 1/std[24], output mean[4], std[4]
  float *sur_vbar, *sur_abar;      // predicted averages (SoA, 3 x ns)
  float *sur_aux;                  // ns x 6 of the last training features: s, dt, v, a (targets' references)
  float sur_thr;                   // residual threshold of a judge step (0: surrogate off)
  int sur_every;                   // judge interval: a passed judge opens sur_every - 1 learned steps
  double *s_r0d;                   // reference positions, FP64 (3 per particle)
  double *s_gsum;                  // sum over the reference neighbours of the stored V_b grad_a W_ab, FP64 (SoA)
  float4 *s_nbr;                   // [k * ns + a] = (V_b grad_a W_ab, b as int bits in w; in 2D z holds b - scene start)
  int nbr_rows;                    // rows of s_nbr: maxn plus the null rows that pad every particle's list
  int nbr_bytes;                   // bytes of s_nbr (0 when it would not fit a 31-bit buffer range)
  // number of scenes whose need_rebuild flag is set (every writer of a flag
  // adjusts it); the rebuild kernels exit after this one load when it is 0
  int *rebuild_count;
  // staging and reductions
  double *stage;
  double *red;
};

}  // namespace mrsph
