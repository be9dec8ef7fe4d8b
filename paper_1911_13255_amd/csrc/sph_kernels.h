// Host-side launchers of the HIP kernels (sph_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "mlp_internal.h"
#include "sph_types.h"

namespace mrsph {

// cells per block of the multi-block cell scan
constexpr int kCellTile = 4096;
// offset classes of the compact reference table (3D): offsets of -2..2
// lattice spacings per axis, 125 of them
constexpr int kNbrClasses = 128;
// particles per thread in the grid-wide step-end reductions
constexpr int kReduceItems = 8;
// reference-table rows each lane loads ahead in the block-resident solid
// kernel; the table carries this many null rows beyond the capacity
#ifndef MRSPH_SOLID_BATCH
#define MRSPH_SOLID_BATCH 2
#endif
constexpr int kSolidBatch = MRSPH_SOLID_BATCH;
// doubles per P B record in LDS of the block-resident solid kernel: the four
// 2D components padded to 48 bytes, a stride at which eight consecutive
// records start on distinct LDS banks
constexpr int solid_pb_record(int dim) { return dim == 2 ? 6 : dim * dim; }
// surrogate: features and outputs per solid particle (2D)
constexpr int kSurFeat = 24;
constexpr int kSurOut = 4;

// neighbour tiles of the fluid pair loops: distinct fluid neighbours held
// per group of one block's particles (records staged in LDS, 32 B each)
constexpr int kTileCap = 768;
// a tile row entry: position in the tile (low bits) and relative cell id
constexpr int kTileIdxBits = 10;
static_assert(kTileCap <= (1 << kTileIdxBits), "tile positions fit their bits");

// lattice blocks of the streamed solid passes (3D): cells per block along
// the lattice axes (slowest to fastest in storage), and the halo of offset
// classes (up to 2 spacings per axis) that a block stages in LDS
constexpr int kLatB0 = 4, kLatB1 = 4, kLatB2 = 16;
constexpr int kLatR = 2;
constexpr int kLatH0 = kLatB0 + 2 * kLatR, kLatH1 = kLatB1 + 2 * kLatR, kLatH2 = kLatB2 + 2 * kLatR;
constexpr int kLatHalo = kLatH0 * kLatH1 * kLatH2;
constexpr int kLatThreads = kLatB0 * kLatB1 * kLatB2;
// LDS layout of a halo component: axis 2 contiguous, then axis 0, then axis 1
// at a stride of kLatRow words (16 or 48 modulo 64), so that the four 16-lane
// rows of a wave (one axis-0 plane, four axis-1 rows) read distinct banks
constexpr int lat_row(int w) { return (w % 64 == 16 || w % 64 == 48) ? w : lat_row(w + 1); }
constexpr int kLatRow = lat_row(kLatH0 * kLatH2);
constexpr int kLatLds = kLatH1 * kLatRow;
static_assert(kLatB2 == 16 && kLatB1 == 4 && kLatThreads % 64 == 0, "a wave is one axis-0 plane of 4 x 16 cells");
// the hardware deals consecutive workgroups to its 8 XCDs in turn; lattice
// blocks are launched so that each XCD runs a contiguous run of the block
// list, whose neighbours share halo cells in that XCD's L2
constexpr int kXcds = 8;

struct LaunchCfg {
  int block_pair;    // threads per block of the fluid pair kernels
  int block_couple;  // threads per block of the coupling kernel
  int block_solid;   // threads per scene of the solid sub-step kernel
  int lpp_force, lpp_cont, lpp_couple, lpp_reinit;  // lanes per particle (1, 2, 4, 8, 16)
  int solid_lds_n;   // solid particles per scene held in LDS by the register-resident kernel
  int solid_ppt;     // > 0: register-resident solid kernel (2D) with this many particles per thread;
                     // 0: streamed multi-block solid passes with kappa read back to the host
  int fork;          // 1: the continuity pass runs on a second stream beside coupling and solid
  int solid_parts;   // > 0: serial steps split scenes of the block-resident solid kernel over workgroups
};

void launch_init_scene(const Dev &D, int s, const double *x_f, const double *v_f, int has_vf, double gabs,
                       double hydroH, double dpd, int nf, hipStream_t st);
void launch_init_walls(const Dev &D, int s, const double *x, const double *n, int nw, hipStream_t st);
void launch_init_solid(const Dev &D, int s, const double *x, const double *v, int has_v, int ns,
                       hipStream_t st);
void launch_solid_reference(const Dev &D, int s, int ns_scene, hipStream_t st);
void launch_solid_B(const Dev &D, hipStream_t st);
// the neighbour span of each split solid workgroup (after the reference table)
void launch_parts_range(const Dev &D, hipStream_t st);
// compact reference table: class gradients from scene s, then every scene's
// pairs checked against their class (D.nbc_ok cleared on a mismatch)
void launch_solid_classes(const Dev &D, int s, hipStream_t st);
void launch_solid_compact(const Dev &D, int s, int ns_scene, hipStream_t st);
// gradient sums of the compact table's entries (once it is in use)
void launch_solid_gsum_classes(const Dev &D, hipStream_t st);
void launch_refresh_vmax(const Dev &D, hipStream_t st);
// with_bin: bin (and scan) the scenes whose rebuild was set from the host;
// graph steps leave that to a launch_prebin ahead of the replays (the
// method's own rebuilds are binned by the step-end reduction and, where the
// cells form one tile, scanned by the step close)
void launch_rebuild(const Dev &D, const LaunchCfg &cfg, hipStream_t st, bool with_bin);
void launch_bin(const Dev &D, hipStream_t st);
void launch_prebin(const Dev &D, hipStream_t st);
void launch_unbin(const Dev &D, int s, hipStream_t st);
void launch_fluid_force(const Dev &D, const LaunchCfg &cfg, hipStream_t st);
// with_couple: the coupling on the solid runs in leading blocks of the same
// launch where the shapes allow; returns true when it did
bool launch_fluid_continuity(const Dev &D, const LaunchCfg &cfg, hipStream_t st, bool with_couple);
void launch_couple(const Dev &D, const LaunchCfg &cfg, hipStream_t st);
// step_end: the launch also does the step-end reduction's work (serial steps);
// parts: scenes split over the workgroups of D.s_parts (nothing else may run
// beside the launch: its workgroups wait for each other)
void launch_solid(const Dev &D, const LaunchCfg &cfg, hipStream_t st, bool step_end, bool parts = false);
// reduced: the solid launch already did the step-end reduction's work;
// next_kappa: the close also evaluates the streamed solid's next kappa from
// the maxima of launch_solid_average (maxima on)
void launch_step_end(const Dev &D, hipStream_t st, bool reduced, bool next_kappa = false);
void launch_sur_features(const Dev &D, const float *stats, float *x, hipStream_t st);
void launch_sur_targets(const Dev &D, float *t, hipStream_t st);
// the surrogate pass of a step, before the solid launch: each scene's mode,
// and for learned and judge scenes the features, the network and the
// predicted averages (the solid launch then takes the learned step or judges)
void launch_sur_net(const Dev &D, const MlpDev &M, hipStream_t st);
// allow the surrogate pass its dynamic LDS (once per process and device)
hipError_t allow_sur_net_lds();
void launch_solid_dt(const Dev &D, hipStream_t st);
// adopt: the step starting now takes kappa and dt_S from the evaluation at
// the end of the step before (launch_step_end with next_kappa; the solid
// state has not changed since)
void launch_solid_first(const Dev &D, bool adopt, hipStream_t st);
void launch_solid_pass(const Dev &D, int sub, hipStream_t st);
// launched: sub-step passes launched this step (scenes with a larger kappa are flagged)
// maxima: also reduce the free solid's max |v| and |a| for the next kappa
void launch_solid_average(const Dev &D, int launched, bool maxima, hipStream_t st);
void launch_read(const Dev &D, int s, int field, int n, double *out, hipStream_t st);
void launch_write(const Dev &D, int s, int field, int n, const double *in, hipStream_t st);
// the FP64 reductions of scene s over nblocks blocks: block partials in
// `part` (nblocks x 16 doubles), the 16 totals in `out` (device memory)
void launch_reduce(const Dev &D, int s, int nblocks, double *part, double *out, hipStream_t st);
// blocks whose partials the static reduction scratch holds
constexpr int kReduceScratchBlocks = 1024;
// device address of the static reduction scratch on the current device
// (taken once per device; later calls return the kept address)
hipError_t reduce_scratch(double **ptr);
void launch_set_rebuild(const Dev &D, int s, hipStream_t st);
int solid_lds_bytes_per_particle(int dim);
hipError_t allow_solid_lds(int dim, int ppt, size_t bytes);

}  // namespace mrsph
