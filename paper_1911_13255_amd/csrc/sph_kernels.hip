// HIP kernels of the multi-resolution SPH FSI method for gfx950.
//
// Neighbour sums are gathers: every particle sums over the 3^d cells of edge
// >= 2 h_F around the cell it was binned in at the last rebuild, so no pair
// force is scattered and no floating-point atomic is used.  Pair geometry
// comes from the positions frozen at the last rebuild (the kernel values and
// gradients of the paper's advection step), held as FP32 offsets from the
// cell origin.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "mlp_device.h"
#include "sph_kernels.h"
#include "sph_physics.h"

namespace mrsph {

// ------------------------------------------------------------------ helpers

// Blocks are handed to the 8 XCDs round-robin; remap so that each XCD works
// on one contiguous range of (Morton-sorted) particles and its own L2 holds
// their neighbours.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  int full = (nb / 8) * 8;
  if (b >= full) return b;
  int per = full / 8;
  return (b % 8) * per + b / 8;
}

__device__ __forceinline__ int xcd_block() { return xcd_block(blockIdx.x, gridDim.x); }

__device__ __forceinline__ int particle_index() { return xcd_block() * blockDim.x + threadIdx.x; }

// Component k of particle a's P B (component-major: the lanes of a wave
// gather consecutive neighbours' component k from a few cache lines).
__device__ __forceinline__ size_t pb_at(const Dev &D, int a, int k) { return (size_t)k * D.ns + a; }
// FP32 record slots of the streamed solid passes (s_PBf component k, s_vf):
// particle a's own, or on lattice blocks its cell's
__device__ __forceinline__ int rec_of(const Dev &D, int a) { return D.lat_nblocks ? D.lat_of[a] : a; }
__device__ __forceinline__ size_t pbf_at(const Dev &D, int r, int k) {
  return (size_t)k * (D.lat_nblocks ? D.lat_ncells : D.ns) + r;
}

// smallest power of two >= n (block-wide tree reductions over any block size)
__device__ __forceinline__ int pow2_ceil(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

__device__ __forceinline__ int wrapi(int n, int N) { return n < 0 ? n + N : (n >= N ? n - N : n); }

__device__ __forceinline__ void decode_cell(const ScenePar &P, int lin, int *c) {
  c[0] = lin % P.ncell[0];
  int r = lin / P.ncell[0];
  c[1] = r % P.ncell[1];
  c[2] = r / P.ncell[1];
}

__device__ __forceinline__ int encode_cell(const ScenePar &P, const int *c) {
  return c[0] + P.ncell[0] * (c[1] + P.ncell[1] * c[2]);
}

// Visit the 3^d neighbouring cells of cell `lin`; fn(neighbour linear index,
// geometric offset of its origin from this cell's origin) and the relative
// cell id (dx+1) + 3 (dy+1) + 9 (dz+1), which cell_shift turns back into sh.
template <int DIM, typename Fn>
__device__ __forceinline__ void visit_cells(const ScenePar &P, int lin, Fn &&fn) {
  int c[3];
  decode_cell(P, lin, c);
  const int zlo = DIM == 3 ? -1 : 0, zhi = DIM == 3 ? 1 : 0;
  for (int dz = zlo; dz <= zhi; ++dz) {
    int n2 = c[2] + dz;
    if (DIM == 3) {
      if (P.periodic[2]) n2 = wrapi(n2, P.ncell[2]);
      else if (n2 < 0 || n2 >= P.ncell[2]) continue;
    }
    for (int dy = -1; dy <= 1; ++dy) {
      int n1 = c[1] + dy;
      if (P.periodic[1]) n1 = wrapi(n1, P.ncell[1]);
      else if (n1 < 0 || n1 >= P.ncell[1]) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        int n0 = c[0] + dx;
        if (P.periodic[0]) n0 = wrapi(n0, P.ncell[0]);
        else if (n0 < 0 || n0 >= P.ncell[0]) continue;
        float sh[3] = {(float)dx * P.cs[0], (float)dy * P.cs[1], (float)dz * P.cs[2]};
        fn(n0 + P.ncell[0] * (n1 + P.ncell[1] * n2), sh, (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1));
      }
    }
  }
}

template <int DIM>
__device__ __forceinline__ void cell_shift(const ScenePar &P, int cid, float *sh) {
  int dx = cid % 3 - 1, dy = (cid / 3) % 3 - 1, dz = cid / 9 - 1;
  sh[0] = (float)dx * P.cs[0];
  sh[1] = (float)dy * P.cs[1];
  sh[2] = DIM == 3 ? (float)dz * P.cs[2] : 0.0f;
}

// four dwords as returned by a 128-bit buffer load (components by index in
// unrolled loops; floats are reinterpreted per element with __int_as_float)
typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i3v __attribute__((ext_vector_type(3)));
// word 3 of a buffer resource on this architecture family: 32-bit data
// format, raw byte addressing (stride 0), so loads past the range read zero
constexpr int kBufferWord3 = 0x00020000;

// Pair-list entries: neighbour index in the low 27 bits, relative cell id
// (< 27) in the top 5.
constexpr int kNbrBits = 27;
constexpr unsigned kNbrMask = (1u << kNbrBits) - 1u;

// Re-express (cell c, offset off) so that the offset lies in [0, cs) where the
// grid allows: periodic axes wrap, other axes clamp to the edge cell and keep
// the remainder in the offset (the 3^d search stays complete either way).
// Returns false (and leaves a zero offset) for a non-finite position.
template <int DIM>
__device__ __forceinline__ bool renormalise(const ScenePar &P, int *c, double *off) {
  bool ok = true;
  for (int k = 0; k < DIM; ++k) {
    if (!isfinite(off[k])) {
      off[k] = 0.0;
      ok = false;
    }
    // bounded so that the integer cell arithmetic cannot overflow
    double q = fmin(fmax(floor(off[k] / P.csd[k]), -1.0e7), 1.0e7);
    c[k] += (int)q;
    off[k] -= q * P.csd[k];
    if (P.periodic[k]) {
      c[k] %= P.ncell[k];
      if (c[k] < 0) c[k] += P.ncell[k];
    } else if (c[k] < 0) {
      off[k] += (double)c[k] * P.csd[k];
      c[k] = 0;
    } else if (c[k] >= P.ncell[k]) {
      off[k] += (double)(c[k] - (P.ncell[k] - 1)) * P.csd[k];
      c[k] = P.ncell[k] - 1;
    }
  }
  return ok;
}

// FP64 absolute position -> (cell, FP64 offset)
template <int DIM>
__device__ __forceinline__ void locate(const ScenePar &P, const double *x, int *c, double *off) {
  c[0] = c[1] = c[2] = 0;
  off[0] = off[1] = off[2] = 0.0;
  for (int k = 0; k < DIM; ++k) {
    double s = x[k] - P.lo[k];
    if (P.periodic[k]) s -= P.len[k] * floor(s / P.len[k]);
    double q = floor(s / P.csd[k]);
    if (q < 0) q = 0;
    if (q > P.ncell[k] - 1) q = P.ncell[k] - 1;
    c[k] = (int)q;
    off[k] = s - q * P.csd[k];
  }
}

template <int DIM>
__device__ __forceinline__ double absolute(const ScenePar &P, int lin, double off, int k) {
  int c[3];
  decode_cell(P, lin, c);
  double x = P.lo[k] + c[k] * P.csd[k] + (double)off;
  if (P.periodic[k]) x = P.lo[k] + (x - P.lo[k]) - P.len[k] * floor((x - P.lo[k]) / P.len[k]);
  return x;
}

__device__ __forceinline__ float get4(float4 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }
__device__ __forceinline__ double get4(double4 v, int k) { return k == 0 ? v.x : (k == 1 ? v.y : v.z); }

// Reduction over the whole block (blockDim a multiple of 64); the result is
// returned to every thread.  sh holds one value per wavefront.
template <typename T, typename Op>
__device__ __forceinline__ T block_reduce(T v, Op op, T *sh) {
  for (int m = 32; m > 0; m >>= 1) v = op(v, __shfl_xor(v, m));
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  T r = sh[0];
  for (int k = 1; k < nw; ++k) r = op(r, sh[k]);
  return r;
}

// True in every thread when all threads of the block pass the same key.
__device__ __forceinline__ bool block_uniform(int key, int *sh) {
  __syncthreads();
  if (threadIdx.x == 0) *sh = key;
  __syncthreads();
  return __syncthreads_and(key == *sh) != 0;
}

// atomic max of a non-negative float through its bit pattern
__device__ __forceinline__ void atomic_max_pos(unsigned int *addr, float v) {
  atomicMax(addr, __float_as_uint(v));
}

// ------------------------------------------------------------------ init

// Initial fluid state: cell-relative position, hydrostatic density
// p = rho0 |g| (H - y_last) through the inverse Tait equation, mass rho dp^d.
template <int DIM>
__global__ void k_init_fluid(Dev D, int s, const double *x, const double *v, int has_v, double gabs,
                             double hydroH, double dpd) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const ScenePar &P = D.par[s];
  if (i >= P.f_count) return;
  int gi = P.f_begin + i;
  int c[3];
  double off[3];
  locate<DIM>(P, x + (size_t)DIM * i, c, off);
  double pr = gabs > 0.0 ? (double)P.rho0 * gabs * (hydroH - x[(size_t)DIM * i + DIM - 1]) : 0.0;
  // FP64 inverse equation of state for the initial state
  double s1 = 1.0 + (double)P.gamma * pr / ((double)P.rho0 * (double)P.c * (double)P.c);
  double eps = s1 > 0.0 ? pow(s1, 1.0 / (double)P.gamma) - 1.0 : -1.0;
  double m = (double)P.rho0 * (1.0 + eps) * dpd;
  D.f_scene[gi] = s;
  D.f_lin[gi] = encode_cell(P, c);
  D.f_id[gi] = i;
  D.f_pos[gi] = make_float4((float)off[0], (float)off[1], (float)off[2], (float)m);
  D.f_off[gi] = make_double4(off[0], off[1], off[2], 0.0);
  D.f_posd[gi] = D.f_off[gi];
  float vv[3] = {0.0f, 0.0f, 0.0f};
  if (has_v)
    for (int k = 0; k < DIM; ++k) vv[k] = (float)v[(size_t)DIM * i + k];
  D.f_va[gi] = make_float4(vv[0], vv[1], vv[2], (float)eps);
  D.f_speed[gi] = sqrtf(vv[0] * vv[0] + vv[1] * vv[1] + vv[2] * vv[2]);
  D.f_nnb[gi] = make_int4(0, 0, 0, 0);
  D.f_rowlen[gi] = make_int2(0, 0);
  D.f_vb[gi] = D.f_va[gi];
  D.f_acc[gi] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  D.f_drho[gi] = 0.0f;
  D.f_p[gi] = 0.0f;
}

template <int DIM>
__global__ void k_init_walls(Dev D, int s, const double *x, const double *n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const ScenePar &P = D.par[s];
  if (i >= P.w_count) return;
  int gi = P.w_begin + i;
  int c[3];
  double off[3];
  locate<DIM>(P, x + (size_t)DIM * i, c, off);
  D.w_lin[gi] = encode_cell(P, c);
  D.w_scene[gi] = s;
  D.w_off[gi] = make_double4(off[0], off[1], off[2], 0.0);
  float nn[3] = {0.0f, 0.0f, 0.0f};
  for (int k = 0; k < DIM; ++k) nn[k] = (float)n[(size_t)DIM * i + k];
  D.w_nrm[gi] = make_float4(nn[0], nn[1], nn[2], 0.0f);
}

template <int DIM>
__global__ void k_init_solid(Dev D, int s, const double *x, const double *v, int has_v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const ScenePar &P = D.par[s];
  if (i >= P.s_count) return;
  int a = P.s_begin + i;
  int NS = D.ns;
  int c[3];
  double off[3];
  locate<DIM>(P, x + (size_t)DIM * i, c, off);
  D.s_scene[a] = s;
  D.s_lin0[a] = encode_cell(P, c);
  bool clamp = i >= P.s_count - P.s_nclamp;
  for (int k = 0; k < 3; ++k) D.s_r0d[3 * (size_t)a + k] = k < DIM ? x[(size_t)DIM * i + k] : 0.0;
  for (int k = 0; k < DIM; ++k) {
    D.s_off0[k * NS + a] = off[k];
    D.s_u[k * NS + a] = 0.0;
    D.s_v[k * NS + a] = (has_v && !clamp) ? v[(size_t)DIM * i + k] : 0.0;
    D.s_a[k * NS + a] = 0.0f;
    D.s_fF[k * NS + a] = 0.0f;
    D.s_fFp[k * NS + a] = 0.0f;
    D.s_vbar[k * NS + a] = 0.0f;
    D.s_abar[k * NS + a] = 0.0f;
    D.s_du[k * NS + a] = 0.0;
    D.s_dv[k * NS + a] = 0.0;
  }
  for (int k = 0; k < DIM * DIM; ++k) {
    D.s_H[k * NS + a] = 0.0;
    D.s_dF[k * NS + a] = 0.0;
  }
  for (int k = 0; k < 3; ++k) D.s_PBg[k * NS + a] = 0.0;
  for (int k = 0; k < 9; ++k) D.s_PBf[pb_at(D, a, k)] = 0.0f;
  D.s_bslot[a] = -1;
  D.s_blin[a] = 0;
}

// Reference-table gradient of one pair: V_b grad_a W(r) for r = X_a - X_b
// with r2 = |r|^2 inside the support, rounded to FP32 per component.
template <int DIM>
__device__ __forceinline__ void ref_gradient(const ScenePar &P, const double *r, double r2, float *g) {
  double h = P.hs;
  double alpha = DIM == 2 ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
  double rr = sqrt(r2);
  double qq = rr / h, t = 1.0 - 0.5 * qq;
  double dW = -5.0 * alpha * qq * t * t * t / h;
  double Vb = P.Vs;
  for (int k = 0; k < DIM; ++k) g[k] = (float)(Vb * r[k] / rr * dW);
}

// Reference neighbour table of the solid (Section 2.2, corrected
// configuration), by exhaustive search over the scene's solid in FP64 with
// ascending neighbour index: b != a with |r0_a - r0_b| < 2 h_S, stored as
// (V_b grad_a W(r0_ab, h_S), b).  Tiles of reference positions go through LDS.
template <int DIM>
__global__ void __launch_bounds__(256) k_solid_neighbours(Dev D, int s) {
  __shared__ double tile[256 * 3];
  const ScenePar &P = D.par[s];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int a = P.s_begin + i;
  bool active = i < P.s_count;
  double xa[3] = {0.0, 0.0, 0.0};
  if (active)
    for (int k = 0; k < 3; ++k) xa[k] = D.s_r0d[3 * (size_t)a + k];
  double h = P.hs, r2max = 4.0 * h * h;
  int cnt = 0;
  int NS = D.ns;
  double gsum[3] = {0.0, 0.0, 0.0};
  for (int t0 = 0; t0 < P.s_count; t0 += 256) {
    __syncthreads();
    int tb = t0 + threadIdx.x;
    if (tb < P.s_count)
      for (int k = 0; k < 3; ++k) tile[3 * threadIdx.x + k] = D.s_r0d[3 * (size_t)(P.s_begin + tb) + k];
    __syncthreads();
    int tn = min(256, P.s_count - t0);
    if (!active) continue;
    for (int q = 0; q < tn; ++q) {
      int ib = t0 + q;
      if (ib == i) continue;
      double r[3];
      double r2 = 0.0;
      for (int k = 0; k < DIM; ++k) {
        r[k] = xa[k] - tile[3 * q + k];
        r2 += r[k] * r[k];
      }
      if (r2 >= r2max) continue;
      if (cnt < D.maxn) {
        float g[3] = {0.0f, 0.0f, 0.0f};
        ref_gradient<DIM>(P, r, r2, g);
        for (int k = 0; k < DIM; ++k) gsum[k] += (double)g[k];  // of the stored values, in slot order
        // (in 2D z holds the neighbour's index within the scene)
        D.s_nbr[(size_t)cnt * NS + a] =
            make_float4(g[0], g[1], DIM == 2 ? __int_as_float(ib) : g[2], __int_as_float(P.s_begin + ib));
      }
      cnt++;
    }
  }
  if (active) {
    D.s_cnt[a] = cnt < D.maxn ? cnt : D.maxn;
    if (cnt > D.maxn) atomicOr(&D.st[s].err, (int)ERR_CAPACITY);
    // null entries (zero gradient, the particle itself) fill the rest of the
    // list, so kernels may walk any row count up to nbr_rows
    for (int q = min(cnt, D.maxn); q < D.nbr_rows; ++q)
      D.s_nbr[(size_t)q * NS + a] = make_float4(0.0f, 0.0f, DIM == 2 ? __int_as_float(i) : 0.0f, __int_as_float(a));
    for (int k = 0; k < 3; ++k) D.s_gsum[k * NS + a] = gsum[k];
  }
}

// Compact reference table (3D).  Where the reference configuration is a
// lattice of spacing dp_S, the offset X_b - X_a of a pair is o dp_S for an
// integer o with |o_k| <= 2 inside the support 2 h_S < 3 dp_S, and the pair's
// gradient depends on o alone: a table entry shrinks to the neighbour's index
// and o's class c = 25 (o_x + 2) + 5 (o_y + 2) + (o_z + 2), 4 bytes instead of
// 16, and the class gradients sit in LDS of the passes that walk the table.

// the class gradient of class c (zero for the centre and offsets outside the support)
__global__ void k_solid_classes(Dev D, int s) {
  const int c = threadIdx.x;
  if (c >= kNbrClasses) return;
  const ScenePar &P = D.par[s];
  const int o[3] = {c / 25 - 2, (c / 5) % 5 - 2, c % 5 - 2};
  double r[3], r2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    r[k] = -(double)o[k] * P.dps;
    r2 += r[k] * r[k];
  }
  float g[3] = {0.0f, 0.0f, 0.0f};
  const double h = P.hs;
  if (c < 125 && r2 > 0.0 && r2 < 4.0 * h * h) ref_gradient<3>(P, r, r2, g);
  D.s_gcls[c] = make_float4(g[0], g[1], g[2], 0.0f);
}

// every pair of scene s: its lattice offset, the class entry, and a check that
// the stored gradient equals the class gradient to FP32 rounding
__global__ void __launch_bounds__(256) k_solid_compact(Dev D, int s) {
  const ScenePar &P = D.par[s];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.s_count) return;
  const int a = P.s_begin + i, NS = D.ns;
  double xa[3];
  for (int k = 0; k < 3; ++k) xa[k] = D.s_r0d[3 * (size_t)a + k];
  const int cnt = D.s_cnt[a];
  bool ok = true;
  for (int q = 0; q < cnt && ok; ++q) {
    const float4 g = D.s_nbr[(size_t)q * NS + a];
    const int b = __float_as_int(g.w);
    int o[3];
    for (int k = 0; k < 3; ++k) {
      const double d = (D.s_r0d[3 * (size_t)b + k] - xa[k]) / P.dps;
      o[k] = (int)rint(d);
      ok &= fabs(d - (double)o[k]) <= 1e-6 && abs(o[k]) <= 2;
    }
    if (!ok) break;
    const int c = 25 * (o[0] + 2) + 5 * (o[1] + 2) + (o[2] + 2);
    const float4 e = D.s_gcls[c];
    const float tol = 1e-6f * (fabsf(e.x) + fabsf(e.y) + fabsf(e.z));
    ok &= tol > 0.0f && fabsf(g.x - e.x) <= tol && fabsf(g.y - e.y) <= tol && fabsf(g.z - e.z) <= tol;
    D.s_nbc[(size_t)q * NS + a] = ((unsigned)b << 7) | (unsigned)c;
  }
  if (!ok) atomicAnd(D.nbc_ok, 0);
}

// gradient sums of the compact entries, in slot order (the own term of the
// momentum sum then uses the same gradients as the neighbour terms)
__global__ void __launch_bounds__(256) k_solid_gsum_classes(Dev D) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= D.ns) return;
  const int NS = D.ns, cnt = D.s_cnt[a];
  double gs[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < cnt; ++q) {
    const float4 e = D.s_gcls[D.s_nbc[(size_t)q * NS + a] & 127u];
    gs[0] += (double)e.x;
    gs[1] += (double)e.y;
    gs[2] += (double)e.z;
  }
  for (int k = 0; k < 3; ++k) D.s_gsum[k * NS + a] = gs[k];
}

// Correction matrix B_a = (sum_b V_b (r0_b - r0_a) (x) grad_a W_ab)^-1 in FP64
// (Section 2.2; the volume V_b makes B dimensionless) and the reference
// surface normal n0 = normalise(-sum_b V_b grad_a W_ab), zero where the sum
// times h_S is below 0.01 (the mid-plane of a thin plate).
template <int DIM>
__global__ void k_solid_B(Dev D) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= D.ns) return;
  const ScenePar &P = D.par[D.s_scene[a]];
  int NS = D.ns;
  double h = P.hs;
  double alpha = DIM == 2 ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
  double A[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, ns[3] = {0, 0, 0};
  double xa[3];
  for (int k = 0; k < 3; ++k) xa[k] = D.s_r0d[3 * (size_t)a + k];
  int cnt = D.s_cnt[a];
  for (int q = 0; q < cnt; ++q) {
    int b = __float_as_int(D.s_nbr[(size_t)q * NS + a].w);
    double r[3], r2 = 0.0;
    for (int k = 0; k < DIM; ++k) {
      r[k] = xa[k] - D.s_r0d[3 * (size_t)b + k];
      r2 += r[k] * r[k];
    }
    double rr = sqrt(r2);
    double qq = rr / h, t = 1.0 - 0.5 * qq;
    double dW = -5.0 * alpha * qq * t * t * t / h;
    double Vb = P.Vs;
    for (int i = 0; i < DIM; ++i) {
      double gi = r[i] / rr * dW;
      ns[i] -= Vb * gi;
      for (int j = 0; j < DIM; ++j) A[i * DIM + j] += Vb * (-r[i]) * (r[j] / rr * dW);
    }
  }
  double Bm[9];
  if (cnt == 0) {
    for (int k = 0; k < DIM * DIM; ++k) Bm[k] = (k % (DIM + 1) == 0) ? 1.0 : 0.0;
  } else if (DIM == 2) {
    double det = A[0] * A[3] - A[1] * A[2];
    Bm[0] = A[3] / det;
    Bm[1] = -A[1] / det;
    Bm[2] = -A[2] / det;
    Bm[3] = A[0] / det;
  } else {
    double det = A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                 A[2] * (A[3] * A[7] - A[4] * A[6]);
    Bm[0] = (A[4] * A[8] - A[5] * A[7]) / det;
    Bm[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    Bm[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    Bm[3] = (A[5] * A[6] - A[3] * A[8]) / det;
    Bm[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    Bm[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    Bm[6] = (A[3] * A[7] - A[4] * A[6]) / det;
    Bm[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    Bm[8] = (A[0] * A[4] - A[1] * A[3]) / det;
  }
  for (int k = 0; k < DIM * DIM; ++k) D.s_B[k * NS + a] = Bm[k];
  double nn = 0.0;
  for (int k = 0; k < DIM; ++k) nn += ns[k] * ns[k];
  nn = sqrt(nn);
  for (int k = 0; k < DIM; ++k) {
    float v = (nn * h >= 0.01) ? (float)(ns[k] / nn) : 0.0f;
    D.s_n0[k * NS + a] = v;
    D.s_n[k * NS + a] = v;
  }
}

// Solid time step (Section 3.2): dt_S = cfl_s min(h_S / (c_S + |v|max),
// sqrt(h_S / |a|max)), the acceleration bound dropped while |a|max = 0.
__device__ __forceinline__ double solid_dt(const ScenePar &P, float vmax, float amax) {
  double dts = (double)P.cfl_s * (double)P.hs / ((double)P.c_s + (double)vmax);
  if (amax > 0.0f) dts = fmin(dts, (double)P.cfl_s * sqrt((double)P.hs / (double)amax));
  return dts;
}

// Max fluid speed of each scene and the acoustic time step that follows
// (Section 3.2, acoustic criterion); one block per scene.  A scene
// that takes one shared step also takes the solid step of its free solid.
__global__ void k_refresh_vmax(Dev D) {
  __shared__ float red[256];
  int s = blockIdx.x;
  const ScenePar &P = D.par[s];
  float m = 0.0f;
  for (int i = threadIdx.x; i < P.f_count; i += blockDim.x) {
    float4 v = D.f_va[P.f_begin + i];
    m = fmaxf(m, sqrtf(v.x * v.x + v.y * v.y + v.z * v.z));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const float vmax = red[0];
  double dt = (double)P.cfl_ac * (double)P.hf / ((double)P.c + (double)vmax);
  if (P.single_step && P.s_count > P.s_nclamp) {
    // one shared step: the solid step of the current free-solid state
    __syncthreads();
    float sv = 0.0f, sa = 0.0f;
    const int NS = D.ns;
    for (int l = threadIdx.x; l < P.s_count - P.s_nclamp; l += blockDim.x) {
      const int a = P.s_begin + l;
      float v2 = 0.0f, a2 = 0.0f;
      for (int k = 0; k < D.dim; ++k) {
        float v = (float)D.s_v[k * NS + a], q = D.s_a[k * NS + a];
        v2 += v * v;
        a2 += q * q;
      }
      sv = fmaxf(sv, sqrtf(v2));
      sa = fmaxf(sa, sqrtf(a2));
    }
    auto fmx = [](float x, float y) { return fmaxf(x, y); };
    __shared__ float shv[16], sha[16];
    sv = block_reduce(sv, fmx, shv);
    sa = block_reduce(sa, fmx, sha);
    dt = fmin(dt, solid_dt(P, sv, sa));
  }
  if (threadIdx.x == 0) {
    SceneState &S = D.st[s];
    S.vmax_prev = __float_as_uint(vmax);
    S.vmax_next = 0u;
    S.send_v = S.send_a = 0u;
    S.dt_ac = dt;
  }
}

// ------------------------------------------------------------------ rebuild
//
// A rebuild runs for the scenes whose need_rebuild flag is set (set at the end
// of the acoustic step that closes an advection step, or by a state write);
// the kernels below test the flag and exit at once otherwise, and the
// step-close kernel at the end of the step clears it.  Stages of a rebuild the
// method decides run ahead, in kernels that run anyway: the binning in the
// step-end reduction and, where the cells form one tile, the cell scan in the
// step close; the coupling lists are put in order by the force launch.

// The advection step ends with the acoustic step that is closing: the same
// test, on the same values, as close_scene's.
__device__ __forceinline__ bool rebuilds_next(const SceneState &S) { return S.adv_accum + S.dt_ac >= S.dt_ad; }

// binning blocks of the step-end kernel (a grid-stride loop over the entries),
// and the scene count up to which its blocks check the scenes' clocks first
constexpr int kBinBlocksMax = 1024;
constexpr int kBinSceneCheck = 8;

// Bin entry t (fluid, then walls and free solid) of a rebuilding scene: new
// cell and offset from the current position, slot within the cell, and a
// copy of the fluid state by old index.  at_step_end: binned by the step-end
// kernel for the rebuild that the closing step is about to set; otherwise at
// the start of a step for a rebuild set from the host (scenes not binned yet).
// which entries a bin_entry call takes
enum { kBinFluid = 1, kBinWalls = 2, kBinSolid = 4, kBinAll = 7 };

template <int DIM>
__device__ void bin_entry(const Dev &D, int t, bool at_step_end, int which = kBinAll) {
  auto due = [&](int s) {
    const SceneState &S = D.st[s];
    return at_step_end ? rebuilds_next(S) : (S.need_rebuild && !S.binned);
  };
  if (t < D.nf) {
    if (!(which & kBinFluid)) return;
    int i = t;
    int s = D.f_scene[i];
    if (!due(s)) return;
    const ScenePar &P = D.par[s];
    int c[3];
    decode_cell(P, D.f_lin[i], c);
    double4 o = D.f_off[i];
    double off[3] = {o.x, o.y, o.z};
    if (!renormalise<DIM>(P, c, off)) atomicOr(&D.st[s].err, (int)ERR_NAN_FLUID);
    int lin = encode_cell(P, c);
    D.fs_lin[i] = lin;
    D.fs_off[i] = make_double4(off[0], off[1], off[2], 0.0);
    D.fs_slot[i] = atomicAdd(&D.fc_count[P.cell_begin + lin], 1);
    D.fs_va[i] = D.f_va[i];
    D.fs_drho[i] = D.f_drho[i];
    D.fs_id[i] = D.f_id[i];
    D.fs_m[i] = D.f_pos[i].w;
    return;
  }
  int q = t - D.nf;
  if (q >= D.nb) return;
  int s = D.bs_scene[q];
  if (!due(s)) return;
  const ScenePar &P = D.par[s];
  int local = q - P.b_begin;
  if (!(which & (local < P.w_count ? kBinWalls : kBinSolid))) return;
  int c[3];
  double off[3] = {0.0, 0.0, 0.0};
  int NS = D.ns;
  if (local < P.w_count) {
    int w = P.w_begin + local;
    decode_cell(P, D.w_lin[w], c);
    double4 o = D.w_off[w];
    off[0] = o.x;
    off[1] = o.y;
    off[2] = o.z;
  } else {
    int a = P.s_begin + (local - P.w_count);
    decode_cell(P, D.s_lin0[a], c);
    for (int k = 0; k < DIM; ++k) off[k] = D.s_off0[k * NS + a] + D.s_u[k * NS + a];
    if (!renormalise<DIM>(P, c, off)) atomicOr(&D.st[s].err, (int)ERR_NAN_SOLID);
  }
  int lin = encode_cell(P, c);
  D.bs_lin[q] = lin;
  D.bs_off[q] = make_double4(off[0], off[1], off[2], 0.0);
  D.bs_slot[q] = atomicAdd(&D.bc_count[P.cell_begin + lin], 1);
}

// Binning at the start of a step, for rebuilds set from the host (state
// writes, initialisation, a forced rebuild); the rebuilds the method itself
// decides are binned by the step-end kernel of the step before.
template <int DIM>
__global__ void __launch_bounds__(256) k_bin(Dev D) {
  if (*D.rebuild_count == 0) return;  // no scene rebuilds this step
  bin_entry<DIM>(D, blockIdx.x * blockDim.x + threadIdx.x, false);
}

// Cell scan of the rebuilding scenes: every cell's [start, end) in the sorted
// fluid and boundary arrays, cells in Morton order within each scene.  The
// cells of all scenes form one rank space (scene s owns [cell_begin,
// cell_begin + ncell_total)); it is cut into tiles of kCellTile cells: tile
// sums, an exclusive scan of the tile sums, then a scan inside each tile.
// Scenes that do not rebuild hold zero counts, so a rebuilding scene's
// entries start at its f_begin / b_begin plus the prefix from its first cell.

// a rebuilding scene whose cells are not scanned yet (binned == 2: scanned
// by the close of the step that set the rebuild)
__device__ __forceinline__ bool scan_due(const SceneState &S) { return S.need_rebuild && S.binned != 2; }

// true when a tile holds cells of a scene due for its scan
__device__ __forceinline__ bool tile_rebuilds(const Dev &D, int g0, int g1) {
  int s0 = D.cell_scene[g0], s1 = D.cell_scene[g1 - 1];
  for (int s = s0; s <= s1; ++s)
    if (scan_due(D.st[s])) return true;
  return false;
}

__global__ void __launch_bounds__(1024) k_cell_sum(Dev D) {
  __shared__ int shf[16], shb[16];
  if (*D.rebuild_count == 0) return;  // no scene rebuilds this step
  const int g0 = blockIdx.x * kCellTile, g1 = min(D.ncell, g0 + kCellTile);
  if (!tile_rebuilds(D, g0, g1)) {
    if (threadIdx.x == 0) D.cell_part[blockIdx.x] = make_int2(0, 0);
    return;
  }
  int lf = 0, lb = 0;
  for (int g = g0 + threadIdx.x; g < g1; g += blockDim.x) {
    int c = D.rank_to_cell[g];
    lf += D.fc_count[c];
    lb += D.bc_count[c];
  }
  auto add = [](int a, int b) { return a + b; };
  lf = block_reduce(lf, add, shf);
  lb = block_reduce(lb, add, shb);
  if (threadIdx.x == 0) D.cell_part[blockIdx.x] = make_int2(lf, lb);
}

// The scan prefix at the first cell of each scene due for its scan.
__device__ __forceinline__ void scan_bases(const Dev &D) {
  int bf = 0, bb = 0;
  for (int s = 0; s < D.n_scenes; ++s) {
    SceneState &S = D.st[s];
    const ScenePar &P = D.par[s];
    S.base_f = bf;
    S.base_b = bb;
    if (!scan_due(S)) continue;
    bf += P.f_count;
    bb += P.b_count;
  }
}

// Per-scene bookkeeping when the rebuild runs (advection time step, Section
// 3.2: dt_ad = cfl_ad min(h / max(|v|max, U_ref), h^2 rho0 / eta)).
__device__ __forceinline__ void rebuild_bookkeeping(const Dev &D) {
  for (int s = 0; s < D.n_scenes; ++s) {
    SceneState &S = D.st[s];
    const ScenePar &P = D.par[s];
    if (!S.need_rebuild) continue;
    double vm = fmax((double)__uint_as_float(S.vmax_prev), (double)P.u_ref);
    double dt = (double)P.cfl_ad * (double)P.hf / vm;
    if (P.dt_visc > 0.0) dt = fmin(dt, P.dt_visc);
    S.dt_ad = dt;
    S.adv_accum = 0.0;
    S.rebuilds += 1;
  }
}

// The scenes whose cells were just scanned (after the last use of scan_due).
__device__ __forceinline__ void mark_scanned(const Dev &D) {
  for (int s = 0; s < D.n_scenes; ++s)
    if (scan_due(D.st[s])) D.st[s].binned = 2;
}

__global__ void __launch_bounds__(1024) k_cell_prefix(Dev D, int ntiles) {
  __shared__ int sf[1024], sb[1024];
  __shared__ int carry[2];
  if (*D.rebuild_count == 0) return;  // no scene rebuilds this step
  const int t = threadIdx.x, T = blockDim.x;
  if (t == 0) {
    scan_bases(D);
    carry[0] = carry[1] = 0;
  }
  __syncthreads();
  for (int c0 = 0; c0 < ntiles; c0 += T) {
    int k = c0 + t;
    int2 v = k < ntiles ? D.cell_part[k] : make_int2(0, 0);
    sf[t] = v.x;
    sb[t] = v.y;
    __syncthreads();
    for (int w = 1; w < T; w <<= 1) {
      int af = t >= w ? sf[t - w] : 0, ab = t >= w ? sb[t - w] : 0;
      __syncthreads();
      sf[t] += af;
      sb[t] += ab;
      __syncthreads();
    }
    if (k < ntiles) D.cell_part[k] = make_int2(carry[0] + sf[t] - v.x, carry[1] + sb[t] - v.y);
    __syncthreads();
    if (t == T - 1) {
      carry[0] += sf[t];
      carry[1] += sb[t];
    }
    __syncthreads();
  }
}

// Each tile: scan of its cells (kCellTile / blockDim consecutive cells per
// thread), [start, end) of every cell of a rebuilding scene; counts reset.
// LDS of one tile of the cell scan: the cells of the tile, then per cell its
// fluid and boundary counts, turned into exclusive prefixes in place.
struct TileLds {
  int cell[kCellTile], pf[kCellTile], pb[kCellTile];
  int wf[16], wb[16];
};

// Scan of one tile (at most kCellTile cells, 1024 threads): counts staged in
// LDS by coalesced loads, per-thread sums of kCellTile / 1024 consecutive
// cells, a block scan by wavefront shuffles, then [start, end) and the count
// reset written cell by cell in coalesced order.
__device__ __forceinline__ void apply_tile(const Dev &D, int g0, int g1, int2 base, TileLds &L) {
  const int t = threadIdx.x, T = blockDim.x, lane = t & 63, w = t >> 6;
  const int ng = g1 - g0, per = kCellTile / T;
  for (int g = t; g < ng; g += T) {
    const int c = D.rank_to_cell[g0 + g];
    L.cell[g] = c;
    L.pf[g] = D.fc_count[c];
    L.pb[g] = D.bc_count[c];
  }
  __syncthreads();
  const int gs = t * per, ge = min(ng, gs + per);
  int lf = 0, lb = 0;
  for (int g = gs; g < ge; ++g) {
    lf += L.pf[g];
    lb += L.pb[g];
  }
  // inclusive block scan of (lf, lb)
  int xf = lf, xb = lb;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int yf = __shfl_up(xf, o), yb = __shfl_up(xb, o);
    if (lane >= o) {
      xf += yf;
      xb += yb;
    }
  }
  if (lane == 63) {
    L.wf[w] = xf;
    L.wb[w] = xb;
  }
  __syncthreads();
  if (t == 0) {
    int af = 0, ab = 0;
    for (int k = 0; k < (T + 63) / 64; ++k) {
      const int vf = L.wf[k], vb = L.wb[k];
      L.wf[k] = af;
      L.wb[k] = ab;
      af += vf;
      ab += vb;
    }
  }
  __syncthreads();
  int pf = base.x + L.wf[w] + xf - lf, pb = base.y + L.wb[w] + xb - lb;
  for (int g = gs; g < ge; ++g) {
    const int cf = L.pf[g], cb = L.pb[g];
    L.pf[g] = pf;
    L.pb[g] = pb;
    pf += cf;
    pb += cb;
  }
  __syncthreads();
  for (int g = t; g < ng; g += T) {
    const int s = D.cell_scene[g0 + g];
    const SceneState &S = D.st[s];
    if (!scan_due(S)) continue;
    const ScenePar &P = D.par[s];
    const int c = L.cell[g];
    const int f0 = P.f_begin + L.pf[g] - S.base_f, b0 = P.b_begin + L.pb[g] - S.base_b;
    D.fc_se[c] = make_int2(f0, f0 + D.fc_count[c]);
    D.bc_se[c] = make_int2(b0, b0 + D.bc_count[c]);
    D.fc_count[c] = 0;
    D.bc_count[c] = 0;
  }
}

__global__ void __launch_bounds__(1024) k_cell_apply(Dev D) {
  __shared__ TileLds L;
  if (*D.rebuild_count == 0) return;  // no scene rebuilds this step
  const int g0 = blockIdx.x * kCellTile, g1 = min(D.ncell, g0 + kCellTile);
  if (!tile_rebuilds(D, g0, g1)) return;
  apply_tile(D, g0, g1, D.cell_part[blockIdx.x], L);
}

// All cells in one tile: scene bases, scan and [start, end) in one block.
__device__ void scan_one_tile(const Dev &D, TileLds &L) {
  if (!tile_rebuilds(D, 0, D.ncell)) return;  // the same answer in every thread
  if (threadIdx.x == 0) scan_bases(D);
  __syncthreads();
  apply_tile(D, 0, D.ncell, make_int2(0, 0), L);
  __syncthreads();
  if (threadIdx.x == 0) mark_scanned(D);
}

__global__ void __launch_bounds__(1024) k_cell_one(Dev D) {
  __shared__ TileLds L;
  if (*D.rebuild_count == 0) return;  // no scene rebuilds this step
  scan_one_tile(D, L);
}

// Counting-sort scatter into cell slots in arrival order, with the sort key
// (original index; boundary: source index) beside each entry.
__global__ void __launch_bounds__(256) k_scatter(Dev D) {
  if (*D.rebuild_count == 0) return;  // no scene rebuilds this step
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) rebuild_bookkeeping(D);  // read by no kernel before the step close
  if (t < D.nf) {
    int s = D.f_scene[t];
    if (!D.st[s].need_rebuild) return;
    int slot = D.fc_se[D.par[s].cell_begin + D.fs_lin[t]].x + D.fs_slot[t];
    D.f_perm[slot] = t;
    D.f_pkey[slot] = D.fs_id[t];
    return;
  }
  int q = t - D.nf;
  if (q >= D.nb) return;
  int s = D.bs_scene[q];
  if (!D.st[s].need_rebuild) return;
  D.b_perm[D.bc_se[D.par[s].cell_begin + D.bs_lin[q]].x + D.bs_slot[q]] = q;
}

// Boundary particle in its cell slot: frozen offset, volume, averaged velocity
// with the hydrostatic factor max(0, (abar - g).n), normal.  For the solid the
// normal is updated from the deformation (n = normalise(F^-T n0)) and the
// current volume is V0 det F.
template <int DIM>
__device__ void gather_boundary(const Dev &D, const ScenePar &P, int k, int q) {
  int local = q - P.b_begin;
  double4 off = D.bs_off[q];
  int NS = D.ns;
  float n[3] = {0.0f, 0.0f, 0.0f}, vb[3] = {0.0f, 0.0f, 0.0f}, ab[3] = {0.0f, 0.0f, 0.0f};
  float V, Vref;
  if (local < P.w_count) {
    D.b_solid[k] = -1;
    float4 wn = D.w_nrm[P.w_begin + local];
    n[0] = wn.x;
    n[1] = wn.y;
    n[2] = wn.z;
    V = P.Vf;
    Vref = P.Vf;
  } else {
    int a = P.s_begin + (local - P.w_count);
    double H[9], Fi[9];
    for (int c = 0; c < DIM * DIM; ++c) H[c] = D.s_H[c * NS + a];
    double J;
    if (DIM == 2) {
      // F^-T = (1/J) [[f11, -f10], [-f01, f00]]; the 1/J drops out of the normalisation
      J = (1.0 + H[0]) * (1.0 + H[3]) - H[1] * H[2];
      Fi[0] = 1.0 + H[3];
      Fi[1] = -H[2];
      Fi[2] = -H[1];
      Fi[3] = 1.0 + H[0];
    } else {
      double F[9];
      for (int c = 0; c < 9; ++c) F[c] = H[c] + ((c % 4 == 0) ? 1.0 : 0.0);
      J = F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) + F[2] * (F[3] * F[7] - F[4] * F[6]);
      // cofactor matrix = J F^-T
      Fi[0] = F[4] * F[8] - F[5] * F[7];
      Fi[1] = F[5] * F[6] - F[3] * F[8];
      Fi[2] = F[3] * F[7] - F[4] * F[6];
      Fi[3] = F[2] * F[7] - F[1] * F[8];
      Fi[4] = F[0] * F[8] - F[2] * F[6];
      Fi[5] = F[1] * F[6] - F[0] * F[7];
      Fi[6] = F[1] * F[5] - F[2] * F[4];
      Fi[7] = F[2] * F[3] - F[0] * F[5];
      Fi[8] = F[0] * F[4] - F[1] * F[3];
    }
    double n0[3] = {0.0, 0.0, 0.0}, nn[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < DIM; ++c) n0[c] = D.s_n0[c * NS + a];
    double l2 = 0.0;
    for (int i = 0; i < DIM; ++i) {
      double v = 0.0;
      for (int j = 0; j < DIM; ++j) v += Fi[i * DIM + j] * n0[j];
      nn[i] = v;
      l2 += v * v;
    }
    double inv = l2 > 0.0 ? 1.0 / sqrt(l2) : 0.0;
    for (int i = 0; i < DIM; ++i) {
      n[i] = (float)(nn[i] * inv);
      D.s_n[i * NS + a] = n[i];
      vb[i] = D.s_vbar[i * NS + a];
      ab[i] = D.s_abar[i * NS + a];
    }
    V = (float)(P.Vs * J);
    Vref = -P.Vs;
    D.s_bslot[a] = k;
    D.s_blin[a] = D.bs_lin[q];
    D.b_solid[k] = a;
    D.s_cpl_cnt[a] = 0;  // the fluid side fills the coupling list in k_reinit
  }
  float sa = 0.0f;
  for (int i = 0; i < DIM; ++i) sa += (ab[i] - P.g[i]) * n[i];
  sa = fmaxf(0.0f, sa);
  D.b_src[k] = local;
  D.b_pos[k] = make_float4((float)off.x, (float)off.y, (float)off.z, V);
  D.b_posd[k] = off;
  D.b_vbar[k] = make_float4(vb[0], vb[1], vb[2], sa);
  D.b_nrm[k] = make_float4(n[0], n[1], n[2], Vref);
}

// One thread per cell slot of a rebuilding scene: the entry's final place in
// its cell is its rank by key among the cell's entries (fluid: original
// index; boundary: source index), so the layout does not depend on atomic
// arrival order; the particle's state moves straight to that place.
template <int DIM>
__global__ void __launch_bounds__(256) k_rank_move(Dev D) {
  if (*D.rebuild_count == 0) return;  // no scene rebuilds this step
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < D.nf) {
    int s = D.f_scene[t];  // scenes own fixed index ranges
    if (!D.st[s].need_rebuild) return;
    const ScenePar &P = D.par[s];
    int o = D.f_perm[t];
    int key = D.f_pkey[t];
    int2 se = D.fc_se[P.cell_begin + D.fs_lin[o]];
    int rank = 0;
    for (int j = se.x; j < se.y; ++j) rank += D.f_pkey[j] < key;
    int k = se.x + rank;
    double4 off = D.fs_off[o];
    D.f_lin[k] = D.fs_lin[o];
    D.f_id[k] = key;
    D.f_pos[k] = make_float4((float)off.x, (float)off.y, (float)off.z, D.fs_m[o]);
    D.f_posd[k] = off;
    D.f_off[k] = off;
    D.f_va[k] = D.fs_va[o];
    D.f_drho[k] = D.fs_drho[o];
    return;
  }
  int kb = t - D.nf;
  if (kb >= D.nb) return;
  int s = D.bs_scene[kb];  // the slot range of a scene equals its source range
  if (!D.st[s].need_rebuild) return;
  const ScenePar &P = D.par[s];
  int q = D.b_perm[kb];
  int2 be = D.bc_se[P.cell_begin + D.bs_lin[q]];
  int rank = 0;
  for (int j = be.x; j < be.y; ++j) rank += D.b_perm[j] < q;
  gather_boundary<DIM>(D, P, be.x + rank, q);
}

// Sum over a group of LPP consecutive lanes (a power of two dividing 64).
template <int LPP, typename T>
__device__ __forceinline__ T group_sum(T v) {
  for (int m = 1; m < LPP; m <<= 1) v += __shfl_xor(v, m, LPP);
  return v;
}

// Pair loops: LPP lanes share one particle; each lane takes every LPP-th
// candidate of each neighbouring cell, and the partial sums are combined
// with cross-lane shuffles.  More lanes per particle keep small scenes'
// waves busy while their loads are in flight.

// Density reinitialisation and pair counts at the start of an advection step
// (Algorithm 1).  psi_i = sum_j V_ref,j W_ij over fluid (self included), walls
// and free solid; mode 1: rho = rho0 max(1, psi/psi0); mode 2: rho =
// max(rho, rho0 psi/psi0).  The pair counts feed the interaction counters.
// The sum is an FP64 island: the pressure that follows is rho0 c^2 times the
// relative excess of psi, so FP32 rounding of W or of positions would appear
// as pressure noise; distances come from the FP64 frozen offsets.
// The same pass writes the pair lists that the force and continuity passes
// walk until the next rebuild (pair geometry is frozen over an advection
// step, Section 3.2).  The LPP lanes of a particle test LPP candidates at a
// time and give their matches consecutive entries (a wavefront ballot ranks
// them), so each row is dense in visiting order whatever LPP is.
template <int DIM, int LPP>
__global__ void __launch_bounds__(256) k_reinit(Dev D) {
  if (*D.rebuild_count == 0) return;  // no scene rebuilds this step
  int g = particle_index();
  int i = g / LPP, q = g % LPP;
  bool active = i < D.nf;
  int s = active ? D.f_scene[i] : 0;
  if (active && !D.st[s].need_rebuild) active = false;
  double psi = 0.0;
  unsigned long long nff = 0, nfw = 0, nfs = 0;
  int lenf = 0, lenb = 0;  // the particle's row lengths so far (equal in its LPP lanes)
  const size_t lstride = (size_t)D.nf * LPP;
  unsigned *lf = D.f_nbl + (size_t)i * LPP, *lb = D.f_bnl + (size_t)i * LPP;
  const int gsh = __lane_id() & ~(LPP - 1);  // first lane of this particle's group
  const unsigned below = (1u << q) - 1u;
  // rank of this lane's match among the group's matches of this round
  auto rank_hits = [&](bool hit, int &len) {
    unsigned grp = (unsigned)(__ballot(hit) >> gsh) & ((1u << LPP) - 1u);
    int e = len + __popc(grp & below);
    len += __popc(grp);
    return e;
  };
  if (active) {
    const ScenePar &P = D.par[s];
    float4 pi = D.f_pos[i];
    double4 qi = D.f_posd[i];
    const double h = P.hf, inv_h = 1.0 / h;
    const double alpha = DIM == 2 ? 7.0 / (4.0 * M_PI * h * h) : 21.0 / (16.0 * M_PI * h * h * h);
    const double Vf = DIM == 2 ? P.dpf * P.dpf : P.dpf * P.dpf * P.dpf;
    const double Vs = DIM == 2 ? P.dps * P.dps : P.dps * P.dps * P.dps;
    auto W64 = [&](double r) {
      double qq = r * inv_h, t = fmax(0.0, 1.0 - 0.5 * qq);
      return alpha * t * t * t * t * (1.0 + 2.0 * qq);
    };
    if (q == 0) psi = Vf * alpha;
    int cb = P.cell_begin;
    // One candidate of each lane of the group (all lanes take part: the
    // matches are ranked by a ballot in candidate order).  sh / shd: the
    // neighbour cell's offset in FP32 and FP64; tag: its cell id in the entry;
    // qload(): the candidate's FP64 offset (taken only for a match where the
    // caller has not loaded it ahead).
    auto fluid_candidate = [&](bool valid, int j, float4 pj, auto qload, const float *sh, const double *shd,
                               unsigned tag) {
      bool hit = false;
      if (valid) {
        // pair membership decided in FP32 exactly as in the force passes
        float rx = (pi.x - pj.x) - sh[0], ry = (pi.y - pj.y) - sh[1];
        float rz = DIM == 3 ? (pi.z - pj.z) - sh[2] : 0.0f;
        float r2 = rx * rx + ry * ry + rz * rz;
        if (r2 < P.r2max_f) {
          if constexpr (DIM == 2) {
            const double4 qj = qload();
            double dx = (qi.x - qj.x) - shd[0], dy = (qi.y - qj.y) - shd[1];
            psi += Vf * W64(sqrt(dx * dx + dy * dy));
          }
          nff++;
          hit = true;
        }
      }
      int e = rank_hits(hit, lenf);
      if (hit && e < D.capf) lf[(size_t)(e / LPP) * lstride + e % LPP] = tag | (unsigned)j;
    };
    // qload(), nwload(): the boundary candidate's FP64 offset and the sign of
    // its reference volume (walls positive), for a match
    auto boundary_candidate = [&](bool valid, int k, float4 pb, auto qload, auto nwload, const float *sh,
                                  const double *shd, unsigned tag, int cid) {
      bool hit = false;
      if (valid) {
        float rx = (pi.x - pb.x) - sh[0], ry = (pi.y - pb.y) - sh[1];
        float rz = DIM == 3 ? (pi.z - pb.z) - sh[2] : 0.0f;
        float r2 = rx * rx + ry * ry + rz * rz;
        if (r2 < P.r2max_f) {
          bool wall = nwload() > 0.0f;
          if constexpr (DIM == 2) {
            const double4 qb = qload();
            double dx = (qi.x - qb.x) - shd[0], dy = (qi.y - qb.y) - shd[1];
            psi += (wall ? Vf : Vs) * W64(sqrt(dx * dx + dy * dy));
          }
          if (wall) {
            nfw++;
          } else {
            nfs++;
            // the transposed entry for the solid particle's coupling list,
            // with the cell offset seen from its side (26 - cid)
            const int a = D.b_solid[k];
            const int e = atomicAdd(&D.s_cpl_cnt[a], 1);
            if (e < D.capf) D.s_cpl[(size_t)e * D.ns + a] = ((unsigned)(26 - cid) << kNbrBits) | (unsigned)i;
          }
          hit = true;
        }
      }
      int e = rank_hits(hit, lenb);
      if (hit && e < D.capb) lb[(size_t)(e / LPP) * lstride + e % LPP] = tag | (unsigned)k;
    };
    if constexpr (DIM == 2) {
      // The 3 x 3 cells' ranges are requested together; their candidates are
      // then taken in one enumeration (cell by cell in visit_cells' order,
      // then by index, so the rows are the same as a cell-by-cell walk), the
      // loads of kRounds rounds issued before any is used.
      constexpr int kRounds = 2;
      int c[3];
      decode_cell(P, D.f_lin[i], c);
      int nlv[9];
      int2 sev[9], bev[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        int n0 = c[0] + k % 3 - 1, n1 = c[1] + k / 3 - 1;
        bool ok = true;
        if (P.periodic[0]) n0 = wrapi(n0, P.ncell[0]);
        else ok &= n0 >= 0 && n0 < P.ncell[0];
        if (P.periodic[1]) n1 = wrapi(n1, P.ncell[1]);
        else ok &= n1 >= 0 && n1 < P.ncell[1];
        nlv[k] = ok ? n0 + P.ncell[0] * n1 : -1;
        const int2 fr = D.fc_se[cb + (ok ? nlv[k] : 0)], br = D.bc_se[cb + (ok ? nlv[k] : 0)];
        sev[k] = ok ? fr : make_int2(0, 0);
        bev[k] = ok ? br : make_int2(0, 0);
      }
      int pf[10], pb[10];  // prefix counts of the candidates over the cells
      pf[0] = pb[0] = 0;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        pf[k + 1] = pf[k] + (sev[k].y - sev[k].x);
        pb[k + 1] = pb[k] + (bev[k].y - bev[k].x);
      }
      // cell k of enumeration position e and the index offset of its range
      // (a select chain over constant indices: the arrays stay in registers)
      auto locate = [](int e, const int *pre, const int2 *rng, int &k, int &off) {
        k = 0;
        off = rng[0].x;
#pragma unroll
        for (int m = 1; m < 9; ++m)
          if (e >= pre[m]) {
            k = m;
            off = rng[m].x - pre[m];
          }
      };
      auto offsets = [&](int k, float *sh, double *shd) {
        const int dx = k % 3 - 1, dy = k / 3 - 1;
        sh[0] = (float)dx * P.cs[0];
        sh[1] = (float)dy * P.cs[1];
        sh[2] = 0.0f;
        shd[0] = (double)dx * P.csd[0];
        shd[1] = (double)dy * P.csd[1];
        shd[2] = 0.0;
      };
      for (int e0 = 0; e0 < pf[9]; e0 += kRounds * LPP) {
        float4 pj[kRounds];
        double4 qj[kRounds];
        int jr[kRounds], kr[kRounds];
        bool vr[kRounds];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
          const int e = e0 + r * LPP + q;
          int off;
          locate(e, pf, sev, kr[r], off);
          jr[r] = off + e;
          vr[r] = e < pf[9] && jr[r] != i;
          if (vr[r]) {
            pj[r] = D.f_pos[jr[r]];
            qj[r] = D.f_posd[jr[r]];
          }
        }
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
          float sh[3];
          double shd[3];
          offsets(kr[r], sh, shd);
          fluid_candidate(vr[r], jr[r], pj[r], [&] { return qj[r]; }, sh, shd, (unsigned)(kr[r] + 9) << kNbrBits);
        }
      }
      for (int e0 = 0; e0 < pb[9]; e0 += kRounds * LPP) {
        float4 pq[kRounds];
        double4 qq[kRounds];
        float nw[kRounds];
        int kb[kRounds], kr[kRounds];
        bool vr[kRounds];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
          const int e = e0 + r * LPP + q;
          int off;
          locate(e, pb, bev, kr[r], off);
          kb[r] = off + e;
          vr[r] = e < pb[9];
          if (vr[r]) {
            pq[r] = D.b_pos[kb[r]];
            qq[r] = D.b_posd[kb[r]];
            nw[r] = D.b_nrm[kb[r]].w;
          }
        }
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
          float sh[3];
          double shd[3];
          offsets(kr[r], sh, shd);
          boundary_candidate(vr[r], kb[r], pq[r], [&] { return qq[r]; }, [&] { return nw[r]; }, sh, shd,
                             (unsigned)(kr[r] + 9) << kNbrBits, kr[r] + 9);
        }
      }
    } else {
      visit_cells<DIM>(P, D.f_lin[i], [&](int nl, const float *sh, int cid) {
        const unsigned tag = (unsigned)cid << kNbrBits;
        // the same cell offset in FP64 (sh is an exact multiple of the FP32 cell size)
        double shd[3];
        for (int k = 0; k < 3; ++k) shd[k] = (double)(sh[k] / P.cs[k]) * P.csd[k];
        // the candidates are tested in FP32 only; the FP64 number density
        // is summed over the finished rows below
        const int2 se = D.fc_se[cb + nl];
        for (int j0 = se.x; j0 < se.y; j0 += LPP) {
          const int j = j0 + q;
          const bool valid = j < se.y && j != i;
          float4 pj;
          if (valid) pj = D.f_pos[j];
          fluid_candidate(valid, j, pj, [&] { return make_double4(0.0, 0.0, 0.0, 0.0); }, sh, shd, tag);
        }
        const int2 be = D.bc_se[cb + nl];
        for (int k0 = be.x; k0 < be.y; k0 += LPP) {
          const int k = k0 + q;
          const bool valid = k < be.y;
          float4 pb;
          float nw = 0.0f;
          if (valid) {
            pb = D.b_pos[k];
            nw = D.b_nrm[k].w;
          }
          boundary_candidate(valid, k, pb, [&] { return make_double4(0.0, 0.0, 0.0, 0.0); }, [&] { return nw; },
                             sh, shd, tag, cid);
        }
      });
      // FP64 number density over the rows just written (every entry a pair,
      // so the lanes stay converged): lane q reads the entries it would walk
      // in the pair passes, written by any lane of its group
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      auto shift64 = [&](unsigned ent, double *shd) {
        const int cid = (int)(ent >> kNbrBits);
        shd[0] = (double)(cid % 3 - 1) * P.csd[0];
        shd[1] = (double)((cid / 3) % 3 - 1) * P.csd[1];
        shd[2] = (double)(cid / 9 - 1) * P.csd[2];
      };
      const int nfl = min(lenf, D.capf), nbl = min(lenb, D.capb);
      for (int e = q; e < nfl; e += LPP) {
        const unsigned ent = lf[(size_t)(e / LPP) * lstride + q];
        double shd[3];
        shift64(ent, shd);
        const double4 qj = D.f_posd[ent & kNbrMask];
        const double dx = (qi.x - qj.x) - shd[0], dy = (qi.y - qj.y) - shd[1], dz = (qi.z - qj.z) - shd[2];
        psi += Vf * W64(sqrt(dx * dx + dy * dy + dz * dz));
      }
      for (int e = q; e < nbl; e += LPP) {
        const unsigned ent = lb[(size_t)(e / LPP) * lstride + q];
        const int k = (int)(ent & kNbrMask);
        double shd[3];
        shift64(ent, shd);
        const double4 qb = D.b_posd[k];
        const double dx = (qi.x - qb.x) - shd[0], dy = (qi.y - qb.y) - shd[1], dz = (qi.z - qb.z) - shd[2];
        psi += (D.b_nrm[k].w > 0.0f ? Vf : Vs) * W64(sqrt(dx * dx + dy * dy + dz * dz));
      }
    }
  }
  psi = group_sum<LPP>(psi);
  nff = group_sum<LPP>(nff);
  nfw = group_sum<LPP>(nfw);
  nfs = group_sum<LPP>(nfs);
  bool lead = active && q == 0;
  if (lead) {
    const ScenePar &P = D.par[s];
    D.f_nnb[i] = make_int4((int)nff, (int)nfw, (int)nfs, 0);
    D.f_rowlen[i] = make_int2(min(lenf, D.capf), min(lenb, D.capb));
    if (lenf > D.capf || lenb > D.capb) atomicOr(&D.st[s].err, (int)ERR_CAPACITY);
    if (P.reinit) {
      float4 va = D.f_va[i];
      double e = psi / P.psi0d - 1.0;
      va.w = P.reinit == 2 ? fmaxf(va.w, (float)e) : (float)fmax(0.0, e);
      D.f_va[i] = va;
    }
  }
}

// Coupling lists of the free solid particles of rebuilding scenes, put in
// ascending entry order (their entries arrive by atomics in any order), so
// the coupling sums do not depend on arrival order.  Run by the leading
// blocks of the fluid force launch (the lists are read by the coupling pass
// that follows it): each wave takes one list at a time, stages it in LDS
// and sends every entry to its rank (entries are distinct: a fluid particle
// appears once per list).  Every thread of a block runs the same number of
// rounds, so the barriers are uniform.
__device__ void sort_coupling_lists(const Dev &D, int nsort) {
  extern __shared__ unsigned cpl_stage[];
  if (*D.rebuild_count == 0) return;  // no scene rebuilds this step (uniform)
  const int waves = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  unsigned *ent = cpl_stage + w * D.capf;
  const int NS = D.ns;
  const int stride = nsort * waves;
  const int rounds = (NS + stride - 1) / stride;
  for (int it = 0; it < rounds; ++it) {
    const int a = it * stride + (int)blockIdx.x * waves + w;
    int n = 0;
    if (a < NS) {
      const int s = D.s_scene[a];
      if (D.st[s].need_rebuild && D.s_bslot[a] >= 0) {
        const int c = D.s_cpl_cnt[a];
        if (c > D.capf && lane == 0) atomicOr(&D.st[s].err, (int)ERR_CAPACITY);
        n = min(c, D.capf);
      }
    }
    unsigned *l = D.s_cpl + (a < NS ? a : 0);
    if (n >= 2)
      for (int e = lane; e < n; e += 64) ent[e] = l[(size_t)e * NS];
    __syncthreads();
    if (n >= 2)
      for (int e = lane; e < n; e += 64) {
        const unsigned v = ent[e];
        int rank = 0;
        for (int f = 0; f < n; ++f) rank += ent[f] < v;
        l[(size_t)rank * NS] = v;
      }
    __syncthreads();
  }
}

// Neighbour tiles of the fluid pair loops.  A block of the force and
// continuity launches takes tile_gp consecutive fluid particles (Morton
// sorted, so a compact group); their fluid neighbours together are a few
// hundred particles (about 530 for 64 particles of the 3D dam break, against
// about 5,000 pairs).  The pair loops stage those neighbours' records in LDS
// once and read them there: a gather of one 16-byte record per lane costs
// the texture data path a cache-line lookup per lane, and that path, not the
// arithmetic, bounds the per-pair form.  After a rebuild this kernel collects
// each group's distinct neighbours in an LDS hash table, sorts them (so the
// staging reads runs of consecutive particles), and writes the group's rows
// again as 16-bit entries: the position in that list and the relative cell
// id (half the bytes for the pair loops to stream).  A group with more than
// kTileCap distinct neighbours, or one that straddles two scenes, has no
// tile (t_count -1).  Groups of scenes that do not rebuild keep their tiles.
// Every thread of a block runs the same barriers.
template <int LPP>
__global__ void __launch_bounds__(256) k_tile_union(Dev D) {
  if (*D.rebuild_count == 0) return;  // no scene rebuilds this step
  constexpr int kHash = 2048;         // > 2 (kTileCap + 256): probing always ends
  __shared__ unsigned key[kHash];     // neighbour index + 1, 0: empty
  __shared__ unsigned short rank[kHash];
  __shared__ unsigned srt[1024];
  __shared__ int n_key, n_put;
  __shared__ volatile int full;
  const int G = D.tile_gp, grp = blockIdx.x;
  const int i0 = grp * G, i1 = min(i0 + G, D.nf);
  const int s0 = D.f_scene[i0], s1 = D.f_scene[i1 - 1];
  if (!D.st[s0].need_rebuild && !D.st[s1].need_rebuild) return;  // rows and list as they were
  if (s0 != s1) {
    if (threadIdx.x == 0) D.t_count[grp] = -1;
    return;
  }
  const int p = threadIdx.x / LPP, q = threadIdx.x % LPP, i = i0 + p;
  const int len = i < i1 ? D.f_rowlen[i].x : 0;
  const int nq = len > q ? (len - 1 - q) / LPP + 1 : 0;  // this lane's entries
  const size_t lstride = (size_t)D.nf * LPP;
  const unsigned *row = D.f_nbl + (size_t)i * LPP + q;
  unsigned short *trow = D.t_rows + (size_t)i * LPP + q;
  auto slot_of = [](unsigned k) { return (k * 2654435761u) >> 21; };  // 11 bits
  // the lane's entries kBatch at a time, all loads issued before any is used
  // (a slot past the lane's last one reads that last slot again)
  constexpr int kBatch = 8;
  auto batch = [&](int k0, unsigned *ent) {
#pragma unroll
    for (int u = 0; u < kBatch; ++u) ent[u] = row[(size_t)min(k0 + u, nq - 1) * lstride];
  };
  for (int k = threadIdx.x; k < kHash; k += blockDim.x) key[k] = 0u;
  if (threadIdx.x == 0) {
    n_key = 0;
    n_put = 0;
    full = 0;
  }
  __syncthreads();
  for (int k0 = 0; k0 < nq; k0 += kBatch) {
    if (full) break;
    unsigned ent[kBatch];
    batch(k0, ent);
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (k0 + u >= nq) break;
      const unsigned k1 = (ent[u] & kNbrMask) + 1u;
      for (unsigned h = slot_of(k1);; h = (h + 1u) & (kHash - 1)) {
        const unsigned old = atomicCAS(&key[h], 0u, k1);
        if (old == 0u) {
          if (atomicAdd(&n_key, 1) >= kTileCap) full = 1;
          break;
        }
        if (old == k1) break;
      }
    }
  }
  __syncthreads();
  if (full) {
    if (threadIdx.x == 0) D.t_count[grp] = -1;
    return;
  }
  const int n = n_key;
  const int np2 = pow2_ceil(max(n, 2));
  for (int k = threadIdx.x; k < kHash; k += blockDim.x)
    if (key[k]) srt[atomicAdd(&n_put, 1)] = key[k] - 1u;
  for (int k = n + threadIdx.x; k < np2; k += blockDim.x) srt[k] = 0xffffffffu;
  __syncthreads();
  // bitonic sort of srt[0, np2) ascending
  for (int size = 2; size <= np2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < np2 / 2; t += blockDim.x) {
        const int lo = 2 * t - (t & (stride - 1)), hi = lo + stride;
        const bool up = (lo & size) == 0;
        const unsigned a = srt[lo], b = srt[hi];
        if ((a > b) == up) {
          srt[lo] = b;
          srt[hi] = a;
        }
      }
      __syncthreads();
    }
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const unsigned k1 = srt[k] + 1u;
    unsigned h = slot_of(k1);
    while (key[h] != k1) h = (h + 1u) & (kHash - 1);
    rank[h] = (unsigned short)k;
    D.t_union[(size_t)grp * kTileCap + k] = srt[k];
  }
  __syncthreads();
  for (int k0 = 0; k0 < nq; k0 += kBatch) {
    unsigned ent[kBatch];
    batch(k0, ent);
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      if (k0 + u >= nq) break;
      const unsigned k1 = (ent[u] & kNbrMask) + 1u;
      unsigned h = slot_of(k1);
      while (key[h] != k1) h = (h + 1u) & (kHash - 1);
      trow[(size_t)(k0 + u) * lstride] = (unsigned short)(rank[h] | ((ent[u] >> kNbrBits) << kTileIdxBits));
    }
  }
  if (threadIdx.x == 0) D.t_count[grp] = n;
}

// ------------------------------------------------------------------ fluid step

// Mid-point snapshot (v^n, eps^{n+1/2}) of every fluid particle for the
// force pass and the coupling on the solid (half step of the density,
// Section 3.3); one record per particle so that the force pass gathers a
// neighbour's state in one read.  Used for large particle counts, where the
// saved gathers outweigh one more launch.  (A third per-particle record of
// pressure and volume, saving their evaluation per pair, was measured
// slower: the pair loops are bound by their gathers as much as by their
// arithmetic.)
__global__ void __launch_bounds__(256) k_fluid_prep(Dev D) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= D.nf) return;
  float dt = (float)D.st[D.f_scene[i]].dt_ac;
  float4 va = D.f_va[i];
  D.f_vs[i] = make_float4(va.x, va.y, va.z, va.w + 0.5f * dt * D.f_drho[i]);
}

// Geometric shifts of the 27 neighbour cells, by relative cell id
// (dx+1) + 3 (dy+1) + 9 (dz+1), staged in LDS for the scene of the block's
// first particle: a pair's shift is one LDS read instead of a base-3 decode.
// Returns whether the calling lane's particle belongs to that scene (other
// lanes, in blocks that straddle scenes, decode the id themselves).  Every
// thread of the block must call it.
template <int DIM>
__device__ __forceinline__ bool stage_shifts(const Dev &D, int s, float4 *tab) {
  __shared__ int s0;
  if (threadIdx.x == 0) s0 = s;
  __syncthreads();
  const int sb = s0;
  if (threadIdx.x < 27) {
    float sh[3];
    cell_shift<DIM>(D.par[sb], (int)threadIdx.x, sh);
    tab[threadIdx.x] = make_float4(sh[0], sh[1], sh[2], 0.0f);
  }
  __syncthreads();
  return s == sb;
}

template <int DIM>
__device__ __forceinline__ float4 pair_shift_cid(const ScenePar &P, bool tab_ok, const float4 *tab, int cid) {
  if (tab_ok) return tab[cid];
  float sh[3];
  cell_shift<DIM>(P, cid, sh);
  return make_float4(sh[0], sh[1], sh[2], 0.0f);
}

template <int DIM>
__device__ __forceinline__ float4 pair_shift(const ScenePar &P, bool tab_ok, const float4 *tab, unsigned ent) {
  return pair_shift_cid<DIM>(P, tab_ok, tab, (int)(ent >> kNbrBits));
}

// Fluid acoustic step, first part (Section 3.3, Eqs. verlet-first-half and
// verlet-first-mediate; Section 3.1 momentum): half step of density (kept as
// eps) and position, Riemann pressure and viscous forces from fluid
// neighbours, coupling forces from walls and solid, gravity, full step of
// velocity.  Reads the mid-point snapshot (v^n, eps^{n+1/2}) of k_fluid_prep;
// writes (v^{n+1}, eps^{n+1/2}), pressure and acceleration.
//
// Per fluid pair (e = r/|r|, du = U_L - U_R = -(v_i - v_j).e):
//   P* = (p_i + p_j)/2 + (rho_i + rho_j)/4 clamp(3 du, 0, c) du,
//   f_i += -2 V_i V_j P* dW e + 2 eta V_i V_j dW / |r| (v_i - v_j).
// An opaque copy of x: the compiler cannot fuse the multiply that produced x
// into a later add or subtract, so a value formed per pair rounds in its sums
// as the same value read from a neighbour tile does.
__device__ __forceinline__ float unfused(float x) {
  asm("" : "+v"(x));
  return x;
}

// A fluid neighbour as the pair loops read it.  Gathered per pair: a = its
// frozen position and mass, b = its velocity and eps.  From a neighbour
// tile: a = position and volume V_j, b = velocity and pressure p_j, s the
// pass's density term (1 + eps_j in the force pass, rho_j in continuity),
// formed once per neighbour by the same expressions the per-pair form
// evaluates.
struct NbrRec {
  float4 a, b;
  float s;
  float4 sh;  // the pair's geometric cell shift, read with the record
};

// Lane q's walk over a pair-list row (entries q, q + LPP, ... below n, at
// lp, lp + lstride, ...): body(entry, rec) for each, where load(entry, rec)
// reads the neighbour's record.  A pair's record is read one pair ahead of
// its arithmetic (measured on the 3D dam break: force pass 634 -> 583 us
// against no look-ahead), and the entries of a round of four pairs are all
// read at the start of the round before, so a round never waits for an
// entry load issued late in the round before it.  Two record sets take the
// pairs in turn, so a record is summed where it was loaded.  Every load is
// unconditional: past the lane's last slot the walk rereads that slot (the
// value then goes unused), so no loaded register is merged with another
// value, which would make the lane wait for its loads in flight.
template <int LPP, typename E, typename Load, typename Body>
__device__ __forceinline__ void walk_pairs(const E *lp, size_t lstride, int q, int n, Load &&load, Body &&body) {
  if (q >= n) return;
  // this lane's slot m, or its last valid slot past the row's end (so every
  // load reads an entry of the row)
  const unsigned last = (unsigned)(n - 1 - q) / LPP, lsb = (unsigned)(lstride * sizeof(E));
  const char *lb = reinterpret_cast<const char *>(lp);
  auto at = [&](unsigned m) {
    return (unsigned)*reinterpret_cast<const E *>(lb + (unsigned long long)min(m, last) * lsb);
  };
  unsigned c0 = *lp, c1 = at(1), c2 = at(2), c3 = at(3);
  NbrRec ra, rb;
  load(c0, ra);
  for (unsigned e = q, m = 4;; e += 4 * LPP, m += 4) {
    const unsigned n0 = at(m), n1 = at(m + 1), n2 = at(m + 2), n3 = at(m + 3);
    // keep those loads here: the scheduler would otherwise sink them to
    // where they are used, a pair before
    __builtin_amdgcn_sched_barrier(0);
    load(c1, rb);
    body(c0, ra);
    if (e + LPP >= n) break;
    load(c2, ra);
    body(c1, rb);
    if (e + 2 * LPP >= n) break;
    load(c3, rb);
    body(c2, ra);
    if (e + 3 * LPP >= n) break;
    load(n0, ra);
    body(c3, rb);
    if (e + 4 * LPP >= n) break;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
}

// One fluid particle's force pass (LPP lanes: lane q takes list entries q,
// q + LPP, ...).  fetch(j, PREP) gives the neighbour's frozen position and
// its snapshot (v^n, eps^{n+1/2}) (formed from the step-start state when
// there is no snapshot pass); every lane of the group must call it.
template <int DIM, int LPP, typename Fetch>
__device__ __forceinline__ void force_particle(const Dev &D, int i, int q, bool active, int s, bool tab_ok,
                                               const float4 *shift_tab, Fetch &&fetch) {
  const int ii = active ? i : 0;
  const ScenePar P = D.par[s];  // by value: the pair loop keeps its fields in registers
  float dt = (float)D.st[s].dt_ac;
  float4 pi = D.f_pos[ii];
  // (v^n, eps^{n+1/2}): from k_fluid_prep for large particle counts, else formed here
  const bool prep = D.fluid_prep != 0;
  float4 va = prep ? D.f_vs[ii] : D.f_va[ii];
  float ehi = prep ? va.w : va.w + 0.5f * dt * D.f_drho[ii];
  float rhoi = P.rho0 * (1.0f + ehi);
  float p_i = eos_p(ehi, P);
  const bool tait7 = __all(P.gamma == 7.0f) != 0;  // before any divergence: uniform
  float mi = pi.w;
  float Vi = mi / rhoi;
  float vi[3] = {va.x, va.y, va.z};
  float fsum[3] = {0.0f, 0.0f, 0.0f};
  // loop invariants of the pair terms
  const float half_pi = 0.5f * p_i;
  const float qrho_i = 0.25f * rhoi;            // (rho_i + rho_j)/4 = qrho_i + qrho0 (1 + eps_j)
  const float qrho0 = 0.25f * P.rho0;
  const float cm = P.riemann ? P.c : 0.0f;     // clamp bound of 3 du (0: simple averages)
  const float kdw = -5.0f * P.alpha_f * P.inv_hf * P.inv_hf;  // dW = kdw r t^3, t = 1 - r/(2h)
  const float kt = -0.5f * P.inv_hf;
  const float m2Vi = -2.0f * Vi, e2Vi = 2.0f * P.eta * Vi;
  if (active) {
    const int2 rl = D.f_rowlen[i];
    const size_t lstride = (size_t)D.nf * LPP;
    // the loop is written once and instantiated for both snapshot sources
    auto fluid_pairs = [&](auto prep_tag) {
      constexpr bool PREP = decltype(prep_tag)::value;
      auto load = [&](unsigned ent, NbrRec &rec) {
        fetch(ent, PREP, dt, rec);
        rec.sh = pair_shift_cid<DIM>(P, std::decay_t<Fetch>::kOneScene || tab_ok, shift_tab,
                                     (int)(ent >> std::decay_t<Fetch>::kIdxBits));
      };
      walk_pairs<LPP>(fetch.rows() + (size_t)i * LPP + q, lstride, q, rl.x, load, [&](unsigned, const NbrRec &rec) {
        const float4 &pj = rec.a, &vj4 = rec.b, &sh = rec.sh;
        float p_j, Vj, s1;  // p_j, V_j, 1 + eps_j
        if constexpr (std::decay_t<Fetch>::kDerived) {
          p_j = vj4.w;
          Vj = pj.w;
          s1 = rec.s;
        } else {
          p_j = unfused(eos_p_pair(vj4.w, P, tait7));
          s1 = 1.0f + vj4.w;
          Vj = unfused(pj.w * fast_rcp(P.rho0 * s1));
        }
        // every fused multiply-add written out and no other contraction, so
        // that the tile and per-pair instantiations of this body round alike
        {
#pragma clang fp contract(off)
        float r[3] = {(pi.x - pj.x) - sh.x, (pi.y - pj.y) - sh.y, DIM == 3 ? (pi.z - pj.z) - sh.z : 0.0f};
        float r2 = fmaf(r[1], r[1], r[0] * r[0]);
        if (DIM == 3) r2 = fmaf(r[2], r[2], r2);
        const float inv_r = __builtin_amdgcn_rsqf(r2);
        const float rr = r2 * inv_r;
        const float t = fmaf(kt, rr, 1.0f);
        const float dW = (kdw * rr) * (t * (t * t));
        const float dv[3] = {vi[0] - vj4.x, vi[1] - vj4.y, DIM == 3 ? vi[2] - vj4.z : 0.0f};
        float w = fmaf(dv[1], r[1], dv[0] * r[0]);
        if (DIM == 3) w = fmaf(dv[2], r[2], w);
        w *= inv_r;  // (v_i - v_j).e = -du
        const float beta = __builtin_amdgcn_fmed3f(-3.0f * w, 0.0f, cm);
        const float qrho = fmaf(qrho0, s1, qrho_i);
        const float Ps = fmaf(-w, qrho * beta, fmaf(0.5f, p_j, half_pi));
        const float VdW = Vj * dW;
        const float cpress = ((m2Vi * VdW) * Ps) * inv_r;  // times r: the unit vector's 1/|r| folded in
        const float cvisc = (e2Vi * VdW) * inv_r;
        for (int k = 0; k < DIM; ++k) fsum[k] += fmaf(cvisc, dv[k], cpress * r[k]);
        }
      });
    };
    if (prep) fluid_pairs(std::true_type{});
    else fluid_pairs(std::false_type{});
    const unsigned *lp = D.f_bnl + (size_t)i * LPP + q;
    for (int e = q; e < rl.y; e += LPP, lp += lstride) {
      unsigned ent = *lp;
      int k = (int)(ent & kNbrMask);
      const float4 sh = pair_shift<DIM>(P, tab_ok, shift_tab, ent);
      float4 pb = D.b_pos[k];
      float r[3] = {(pi.x - pb.x) - sh.x, (pi.y - pb.y) - sh.y, DIM == 3 ? (pi.z - pb.z) - sh.z : 0.0f};
      float f[3];
      coupling_force<DIM>(P, mi, ehi, p_i, vi, r, pb, D.b_vbar[k], D.b_nrm[k], f);
      for (int c = 0; c < DIM; ++c) fsum[c] += f[c];
    }
  }
  for (int k = 0; k < DIM; ++k) fsum[k] = group_sum<LPP>(fsum[k]);
  if (!active || q != 0) return;
  float a[3] = {0.0f, 0.0f, 0.0f}, vn[3] = {vi[0], vi[1], vi[2]};
  for (int k = 0; k < DIM; ++k) {
    a[k] = fsum[k] / mi + P.g[k];
    vn[k] = vi[k] + dt * a[k];
  }
  double4 off = D.f_off[i];
  const double hdt = 0.5 * D.st[s].dt_ac;
  off.x += hdt * vi[0];
  off.y += hdt * vi[1];
  if (DIM == 3) off.z += hdt * vi[2];
  D.f_off[i] = off;
  D.f_vb[i] = make_float4(vn[0], vn[1], vn[2], ehi);
  if (!prep) D.f_vs[i] = make_float4(vi[0], vi[1], vi[2], ehi);
  D.f_p[i] = p_i;
  D.f_acc[i] = make_float4(a[0], a[1], a[2], 0.0f);
}

// neighbour state from global memory (the per-particle form)
struct FetchGlobal {
  static constexpr bool kDerived = false;
  static constexpr bool kOneScene = false;
  static constexpr int kIdxBits = kNbrBits;
  const Dev &D;
  __device__ __forceinline__ const unsigned *rows() const { return D.f_nbl; }
  __device__ __forceinline__ void operator()(unsigned ent, bool prep, float dt, NbrRec &rec) const {
    const int j = (int)(ent & kNbrMask);
    rec.a = D.f_pos[j];
    if (prep) {
      rec.b = D.f_vs[j];
    } else {
      rec.b = D.f_va[j];
      rec.b.w += 0.5f * dt * D.f_drho[j];
    }
  }
};

// A block's neighbour tile in LDS: the records of the group's distinct
// fluid neighbours (entries of its rows index them).
struct NbrTile {
  float4 a[kTileCap], b[kTileCap];
  float s[kTileCap];
};

// Stage a block's tile: rec(j, r) gives neighbour j's record, stored for the
// tile's k-th neighbour tu[k].  Each thread issues the loads of three of its
// neighbours before storing any (a slot past the end reads the last
// neighbour again and is not stored).  Every thread of the block calls it.
template <typename Rec>
__device__ __forceinline__ void stage_tile(int cnt, const unsigned *tu, NbrTile &t, Rec &&rec) {
  constexpr int kUnroll = 3;
  for (int k0 = threadIdx.x; k0 < cnt; k0 += kUnroll * (int)blockDim.x) {
    int j[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) j[u] = (int)tu[min(k0 + u * (int)blockDim.x, cnt - 1)];
    NbrRec r[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) rec(j[u], r[u]);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int k = k0 + u * (int)blockDim.x;
      if (k < cnt) {
        t.a[k] = r[u].a;
        t.b[k] = r[u].b;
        t.s[k] = r[u].s;
      }
    }
  }
  __syncthreads();
}

// neighbour records from the block's tile in LDS (entries index the tile)
struct FetchTile {
  static constexpr bool kDerived = true;
  static constexpr bool kOneScene = true;  // a tile's group lies in one scene: its shift table holds
  static constexpr int kIdxBits = kTileIdxBits;
  const NbrTile &t;
  const unsigned short *trows;
  __device__ __forceinline__ const unsigned short *rows() const { return trows; }
  __device__ __forceinline__ void operator()(unsigned ent, NbrRec &rec) const {
    const unsigned k = ent & ((1u << kTileIdxBits) - 1u);
    rec.a = t.a[k];
    rec.b = t.b[k];
    rec.s = t.s[k];
  }
  __device__ __forceinline__ void operator()(unsigned ent, bool, float, NbrRec &rec) const { (*this)(ent, rec); }
  __device__ __forceinline__ void operator()(unsigned ent, bool, NbrRec &rec) const { (*this)(ent, rec); }
};

// the continuity pass's per-pair gathers: position and mass, (v^{n+1},
// eps^{n+1/2}), and the force pass's pressure where it is not recomputed
struct FetchContinuity {
  static constexpr bool kDerived = false;
  static constexpr bool kOneScene = false;
  static constexpr int kIdxBits = kNbrBits;
  const Dev &D;
  __device__ __forceinline__ const unsigned *rows() const { return D.f_nbl; }
  __device__ __forceinline__ void operator()(unsigned ent, bool tait7, NbrRec &rec) const {
    const int j = (int)(ent & kNbrMask);
    rec.a = D.f_pos[j];
    rec.b = D.f_vb[j];
    if (!tait7) rec.s = D.f_p[j];
  }
};

template <int DIM, int LPP>
__global__ void __launch_bounds__(256, 5) k_fluid_force(Dev D) {
  __shared__ float4 shift_tab[27];
  if ((int)blockIdx.x < D.sort_blocks) {
    sort_coupling_lists(D, D.sort_blocks);
    return;
  }
  // the leading blocks are a multiple of 8: the XCD of a force block is
  // still its index modulo 8
  const int b = xcd_block(blockIdx.x - D.sort_blocks, gridDim.x - D.sort_blocks);
  int g = b * blockDim.x + threadIdx.x;
  int i = g / LPP, q = g % LPP;
  bool active = i < D.nf;
  int s = D.nf > 0 ? D.f_scene[active ? i : 0] : 0;
  const bool tab_ok = stage_shifts<DIM>(D, s, shift_tab);
  if constexpr (DIM == 3) {
    if (D.tile_gp > 0) {  // the same for the whole launch
      const int cnt = D.t_count[b];  // the same for the whole block
      if (cnt >= 0) {
        // the group lies in one scene: its first particle's step
        const int sg = D.f_scene[b * D.tile_gp];
        const float dt = (float)D.st[sg].dt_ac;
        __shared__ NbrTile tile;
        const unsigned *tu = D.t_union + (size_t)b * kTileCap;
        const ScenePar &P = D.par[sg];
        // the snapshot as the per-pair gathers form it, then p_j, V_j and
        // 1 + eps_j by the pair loop's expressions
        auto derive = [&](NbrRec &r) {
          const float eps = r.b.w;
          r.s = 1.0f + eps;
          r.a.w = r.a.w * fast_rcp(P.rho0 * r.s);
          r.b.w = eos_p(eps, P);
        };
        if (D.fluid_prep)
          stage_tile(cnt, tu, tile, [&](int j, NbrRec &r) {
            r.a = D.f_pos[j];
            r.b = D.f_vs[j];
            derive(r);
          });
        else
          stage_tile(cnt, tu, tile, [&](int j, NbrRec &r) {
            r.a = D.f_pos[j];
            r.b = D.f_va[j];
            r.b.w += 0.5f * dt * D.f_drho[j];
            derive(r);
          });
        force_particle<DIM, LPP>(D, i, q, active, s, tab_ok, shift_tab, FetchTile{tile, D.t_rows});
        return;
      }
    }
  }
  force_particle<DIM, LPP>(D, i, q, active, s, tab_ok, shift_tab, FetchGlobal{D});
}

// Force of the fluid on each free solid particle (Section 2.2, F:p and F:v at
// h_F): the exact negatives of the fluid-side pair terms, from the same
// mid-point snapshot (v^n, eps^{n+1/2}, p^{n+1/2}) and the same frozen geometry.
template <int DIM, int LPP>
__device__ __forceinline__ void couple_entry(const Dev &D, int g) {
  int a = g / LPP, q = g % LPP;
  bool active = a < D.ns;
  int aa = active ? a : 0;
  int s = D.ns > 0 ? D.s_scene[aa] : 0;
  const ScenePar &P = D.par[s];
  int NS = D.ns;
  int local = aa - P.s_begin;
  float fa[3] = {0.0f, 0.0f, 0.0f}, fap[3] = {0.0f, 0.0f, 0.0f};
  int k = active ? D.s_bslot[aa] : -1;
  if (active && local < P.s_count - P.s_nclamp && k >= 0) {
    float4 pb = D.b_pos[k], bv = D.b_vbar[k], bn = D.b_nrm[k];
    // the fluid neighbours listed for this particle at the last rebuild
    const int n = min(D.s_cpl_cnt[a], D.capf);
    for (int e = q; e < n; e += LPP) {
      const unsigned ent = D.s_cpl[(size_t)e * NS + a];
      const int i = (int)(ent & kNbrMask);
      float sh[3];
      cell_shift<DIM>(P, (int)(ent >> kNbrBits), sh);
      float4 pi = D.f_pos[i];
      // same rounding as the fluid side's (p_i - p_b) - shift
      float r[3] = {(pi.x - pb.x) + sh[0], (pi.y - pb.y) + sh[1], DIM == 3 ? (pi.z - pb.z) + sh[2] : 0.0f};
      float r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      if (r2 >= P.r2max_f) continue;  // listed pairs passed this same test
      float4 vs = D.f_vs[i];
      float vi[3] = {vs.x, vs.y, vs.z};
      float f[3], fp[3];
      coupling_force<DIM>(P, pi.w, vs.w, D.f_p[i], vi, r, pb, bv, bn, f, fp);
      for (int c = 0; c < DIM; ++c) {
        fa[c] -= f[c];
        fap[c] -= fp[c];
      }
    }
  }
  for (int c = 0; c < DIM; ++c) {
    fa[c] = group_sum<LPP>(fa[c]);
    fap[c] = group_sum<LPP>(fap[c]);
  }
  if (active && q == 0)
    for (int c = 0; c < DIM; ++c) {
      D.s_fF[c * NS + a] = fa[c];
      D.s_fFp[c * NS + a] = fap[c];
    }
}

template <int DIM, int LPP>
__global__ void __launch_bounds__(256) k_couple(Dev D) {
  couple_entry<DIM, LPP>(D, blockIdx.x * blockDim.x + threadIdx.x);
}

// Fluid acoustic step, second part (Section 3.1 continuity with the Riemann
// interface velocity; Section 3.3, Eq. verlet-first-final): density rate with
// v^{n+1} at the mid-point density, plus rho_i sum_a V_a (v_i - vbar_a).grad W
// for walls and solid; second half step of position and density; inflow
// buffer; max speed for the next acoustic step.
// One fluid particle's continuity pass (LPP lanes: lane q takes list
// entries q, q + LPP, ...).  fetch(entry, pj, vj4) gives the neighbour's
// frozen position and its (v^{n+1}, eps^{n+1/2}); every lane of the group
// must call it.
template <int DIM, int LPP, typename Fetch>
__device__ __forceinline__ void continuity_particle(const Dev &D, int i, int q, bool active, int ii, int s,
                                                   bool tab_ok, const float4 *shift_tab, Fetch &&fetch) {
  const ScenePar P = D.par[s];  // by value: the pair loop keeps its fields in registers
  SceneState &S = D.st[s];
  float4 pi = D.f_pos[ii];
  float4 vb = D.f_vb[ii];
  float ehi = vb.w;
  float rhoi = P.rho0 * (1.0f + ehi);
  float p_i = D.f_p[ii];
  const bool tait7 = __all(P.gamma == 7.0f) != 0;  // before any divergence: uniform
  float vi[3] = {vb.x, vb.y, vb.z};
  float drho = 0.0f;
  // Per fluid pair, with v* the Riemann interface velocity:
  //   (v_i - v*).e = (v_i - v_j).e / 2 + (p_i - p_j) / ((rho_i + rho_j) c),
  //   drho_i += 2 rho_i V_j (v_i - v*).e dW.
  const float rc = P.riemann ? P.c : 0.0f;
  const float kdw = -5.0f * P.alpha_f * P.inv_hf * P.inv_hf;
  const float kt = -0.5f * P.inv_hf;
  if (active) {
    const int2 rl = D.f_rowlen[i];
    const size_t lstride = (size_t)D.nf * LPP;
    // The force pass's pressure p_j: for gamma = 7 recomputed from eps (the
    // same expression, so the same bits), otherwise gathered; the loop is
    // instantiated for each, so that neither carries a load taken for only
    // some pairs (it would make every pair wait for all of its lane's loads
    // in flight).  A tile holds p_j, V_j and rho_j already.
    auto fluid_pairs = [&](auto t7_tag) {
      constexpr bool T7 = decltype(t7_tag)::value;
      auto load = [&](unsigned ent, NbrRec &rec) {
        fetch(ent, T7, rec);
        rec.sh = pair_shift_cid<DIM>(P, std::decay_t<Fetch>::kOneScene || tab_ok, shift_tab,
                                     (int)(ent >> std::decay_t<Fetch>::kIdxBits));
      };
      walk_pairs<LPP>(fetch.rows() + (size_t)i * LPP + q, lstride, q, rl.x, load, [&](unsigned, const NbrRec &rec) {
        const float4 &pj = rec.a, &vj4 = rec.b, &sh = rec.sh;
        float p_j, Vj, rhoj;
        if constexpr (std::decay_t<Fetch>::kDerived) {
          p_j = vj4.w;
          Vj = pj.w;
          rhoj = rec.s;
        } else {
          p_j = T7 ? unfused(eos_p_pair(vj4.w, P, true)) : rec.s;
          rhoj = unfused(P.rho0 * (1.0f + vj4.w));
          Vj = unfused(pj.w * fast_rcp(rhoj));
        }
        // every fused multiply-add written out and no other contraction, so
        // that the tile and per-pair instantiations of this body round alike
        {
#pragma clang fp contract(off)
        float r[3] = {(pi.x - pj.x) - sh.x, (pi.y - pj.y) - sh.y, DIM == 3 ? (pi.z - pj.z) - sh.z : 0.0f};
        float r2 = fmaf(r[1], r[1], r[0] * r[0]);
        if (DIM == 3) r2 = fmaf(r[2], r[2], r2);
        const float inv_r = __builtin_amdgcn_rsqf(r2);
        const float rr = r2 * inv_r;
        const float t = fmaf(kt, rr, 1.0f);
        const float dW = (kdw * rr) * (t * (t * t));
        float w = fmaf(vi[1] - vj4.y, r[1], (vi[0] - vj4.x) * r[0]);
        if (DIM == 3) w = fmaf(vi[2] - vj4.z, r[2], w);
        const float wr = 0.5f * (w * inv_r);
        const float dvs = fmaf(p_i - p_j, fast_rcp((rhoi + rhoj) * rc), wr);
        drho = fmaf((2.0f * rhoi) * (Vj * dW), rc > 0.0f ? dvs : wr, drho);
        }
      });
    };
    if (std::decay_t<Fetch>::kDerived || tait7)
      fluid_pairs(std::true_type{});
    else
      fluid_pairs(std::false_type{});
    const unsigned *lp = D.f_bnl + (size_t)i * LPP + q;
    for (int e = q; e < rl.y; e += LPP, lp += lstride) {
      unsigned ent = *lp;
      int k = (int)(ent & kNbrMask);
      const float4 sh = pair_shift<DIM>(P, tab_ok, shift_tab, ent);
      {
        float4 pb = D.b_pos[k];
        float r[3] = {(pi.x - pb.x) - sh.x, (pi.y - pb.y) - sh.y, DIM == 3 ? (pi.z - pb.z) - sh.z : 0.0f};
        float r2 = r[0] * r[0] + r[1] * r[1];
        if (DIM == 3) r2 += r[2] * r[2];
        float4 bv = D.b_vbar[k];
        const float inv_r = __builtin_amdgcn_rsqf(r2);
        const float rr = r2 * inv_r;
        const float t = 1.0f + kt * rr;
        const float dW = (kdw * rr) * (t * t * t);
        float dv = (vi[0] - bv.x) * r[0] + (vi[1] - bv.y) * r[1];
        if (DIM == 3) dv += (vi[2] - bv.z) * r[2];
        drho += rhoi * pb.w * (dv * inv_r) * dW;
      }
    }
  }
  drho = group_sum<LPP>(drho);
  bool lead = active && q == 0;
  float speed = 0.0f;
  if (lead) {
    float dt = (float)S.dt_ac;
    float de = drho / P.rho0;
    float enew = ehi + 0.5f * dt * de;
    double4 off = D.f_off[i];
    const double hdt = 0.5 * S.dt_ac;
    off.x += hdt * vi[0];
    off.y += hdt * vi[1];
    if (DIM == 3) off.z += hdt * vi[2];
    if (P.in_len > 0.0f) {
      // inflow buffer at the start of the first axis (periodic channel)
      int lin = D.f_lin[i];
      double x0 = absolute<DIM>(P, lin, off.x, 0);
      if (x0 - P.lo[0] < (double)P.in_len) {
        double y = absolute<DIM>(P, lin, off.y, 1);
        double t = S.t + S.dt_ac;
        double ub = t <= (double)P.in_ts ? 0.5 * (double)P.in_U0 * (1.0 - cos(0.5 * M_PI * t)) : (double)P.in_U0;
        double H = P.in_H;
        double u = (y > 0.0 && y < H) ? 6.0 * ub * y * (H - y) / (H * H) : 0.0;
        vi[0] = (float)u;
        vi[1] = 0.0f;
        vi[2] = 0.0f;
      }
    }
    D.f_off[i] = off;
    D.f_va[i] = make_float4(vi[0], vi[1], vi[2], enew);
    D.f_drho[i] = de;
    speed = sqrtf(vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]);
    D.f_speed[i] = speed;
    if (!(isfinite(speed) && isfinite(enew))) atomicOr(&S.err, (int)ERR_NAN_FLUID);
  }
}
template <int DIM, int LPP>
__global__ void __launch_bounds__(256) k_fluid_continuity(Dev D) {
  __shared__ float4 shift_tab[27];
  // in a graph step the coupling on the solid, which reads only the force
  // pass's snapshot, runs in the leading blocks (a multiple of 8, so the XCD
  // of a continuity block is still its index modulo 8)
  if ((int)blockIdx.x < D.couple_blocks) {
    couple_entry<DIM, LPP>(D, blockIdx.x * blockDim.x + threadIdx.x);
    return;
  }
  int g = xcd_block(blockIdx.x - D.couple_blocks, gridDim.x - D.couple_blocks) * blockDim.x + threadIdx.x;
  int i = g / LPP, q = g % LPP;
  bool active = i < D.nf;
  int ii = active ? i : 0;
  int s = D.nf > 0 ? D.f_scene[ii] : 0;
  const bool tab_ok = stage_shifts<DIM>(D, s, shift_tab);
  if constexpr (DIM == 3) {
    if (D.tile_gp > 0) {  // the same for the whole launch
      const int b = xcd_block(blockIdx.x - D.couple_blocks, gridDim.x - D.couple_blocks);
      const int cnt = D.t_count[b];  // the same for the whole block
      if (cnt >= 0) {
        __shared__ NbrTile tile;
        // the group lies in one scene
        const ScenePar &P = D.par[D.f_scene[b * D.tile_gp]];
        // p_j, V_j and rho_j by the pair loop's expressions (the force pass
        // stored p_j = eos_p(eps_j))
        stage_tile(cnt, D.t_union + (size_t)b * kTileCap, tile, [&](int j, NbrRec &r) {
          r.a = D.f_pos[j];
          r.b = D.f_vb[j];
          const float eps = r.b.w;
          r.s = P.rho0 * (1.0f + eps);
          r.a.w = r.a.w * fast_rcp(r.s);
          r.b.w = eos_p(eps, P);
        });
        continuity_particle<DIM, LPP>(D, i, q, active, ii, s, tab_ok, shift_tab, FetchTile{tile, D.t_rows});
        return;
      }
    }
  }
  continuity_particle<DIM, LPP>(D, i, q, active, ii, s, tab_ok, shift_tab, FetchContinuity{D});
}

// ------------------------------------------------------------------ solid sub-steps

constexpr int KAPPA_MAX = 4096;

// Close of an acoustic step of scene s (after the step-end reductions):
// time, advection accumulator and rebuild flag, next acoustic time step from
// the reduced max fluid speed (Section 3.2), pair counts after a rebuild and
// the interaction counters.
// vmax: the step's max fluid speed (float bits); counts: the pair counts
// after a rebuild (null: take the accumulators the reduction kernel filled).
__device__ void solid_kappa_next(const Dev &D, int s);

// next_kappa: then also the next step's kappa of the streamed solid
// (solid_kappa_next).
__device__ void close_scene(const Dev &D, int s, unsigned vmax_bits, const unsigned long long *counts,
                            bool next_kappa = false) {
  const ScenePar &P = D.par[s];
  SceneState &S = D.st[s];
  const bool rebuilt = S.need_rebuild != 0;  // the rebuild kernels of this step ran
  if (rebuilt) {
    S.n_ff = counts ? counts[0] : S.acc_ff;
    S.n_fw = counts ? counts[1] : S.acc_fw;
    S.n_fs = counts ? counts[2] : S.acc_fs;
    S.acc_ff = S.acc_fw = S.acc_fs = 0ull;
  }
  const int kap = S.kappa;
  const double dt_ac = S.dt_ac;
  unsigned long long inter = 2ull * (S.n_ff + S.n_fw + S.n_fs) + S.n_fs + 2ull * (unsigned long long)kap * S.n_ss;
  if (rebuilt && P.reinit) inter += S.n_ff + S.n_fw + S.n_fs;
  // surrogate steps: the feature means over the solid pairs (learned and
  // judge steps) and the rate pass of a learned step
  if (S.sur) {
    if (S.sur == kSurLearned) {
      inter += 2ull * S.n_ss;
      S.sur_ok += 1;
    } else {
      if (S.sur == kSurJudge) inter += S.n_ss;
      S.sur_fallback += 1;
    }
    S.sur = 0;
  }
  S.interactions += inter;
  S.substeps += kap;
  S.steps += 1;
  S.t += dt_ac;
  S.adv_accum += dt_ac;
  const int was = S.need_rebuild, now = S.adv_accum >= S.dt_ad ? 1 : 0;
  S.need_rebuild = now;
  S.binned = now;  // the step-end kernel binned exactly these scenes
  if (now != was) atomicAdd(D.rebuild_count, now - was);
  float vmax = __uint_as_float(vmax_bits);
  S.vmax_prev = vmax_bits;
  S.vmax_next = 0u;
  double dt = (double)P.cfl_ac * (double)P.hf / ((double)P.c + (double)vmax);
  // one shared step: the solid step of the state the next step starts from
  if (P.single_step && P.s_count > P.s_nclamp)
    dt = fmin(dt, solid_dt(P, __uint_as_float(S.send_v), __uint_as_float(S.send_a)));
  S.send_v = S.send_a = 0u;
  S.dt_ac = dt;
  if (next_kappa) solid_kappa_next(D, s);
}

__global__ void k_step_close(Dev D, int next_kappa) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= D.n_scenes) return;
  close_scene(D, s, D.st[s].vmax_next, nullptr, next_kappa != 0);
}

// The same close, one thread per scene, then (all cells in one tile) the
// cell scan of the rebuilds it has just set, whose particles the step-end
// reduction binned: the next step starts with the scatter.
__global__ void __launch_bounds__(1024) k_step_close_scan(Dev D, int next_kappa) {
  __shared__ TileLds L;
  const int s = threadIdx.x;
  if (s < D.n_scenes) close_scene(D, s, D.st[s].vmax_next, nullptr, next_kappa != 0);
  __syncthreads();
  scan_one_tile(D, L);
}

// kappa solid sub-steps of the position-based Verlet scheme (Section 3.3,
// Eqs. verlet-*-solid), the fluid force held constant:
//   F += dt/2 dF/dt;  u += dt/2 v;  P B from the Neo-Hookean stress;
//   a = [sum_b V_a V_b (P_a B_a + P_b B_b) grad0_a W_ab + f^F_a] / m_a + g;  v += dt a;
//   dF/dt = sum_b V_b (v_b - v_a) (x) (B_a grad0_a W_ab);  F += dt/2 dF/dt;  u += dt/2 v;
// with dt_S = cfl_s min(h_S / (c_S + |v|max), sqrt(h_S / |a|max)) and kappa =
// floor(dt_ac / dt_S) + 1 equal sub-steps summing to dt_ac.  Afterwards the
// averages vbar = du / dt_ac and abar = dv / dt_ac over the acoustic step
// (Section 3.2) are stored for the step-end kernel.  The solid arithmetic is
// an FP64 island: the acceleration is a second difference of the
// displacement and amplifies rounding noise at the particle scale.
//
// Streamed form for solids of any size: one kernel per phase over all solid
// particles of all scenes (a scene past its own kappa skips the pass).

// Solid time step and kappa of each scene: max |v| and |a| of the free solid
// over all solid particles (one atomic per block and scene), the step
// increments cleared; then k_solid_dt_close, one thread per scene.
// max |v| and |a| of the free solid particles a0 .. a1 - 1 per scene into
// smax_v and smax_a (one atomic per block and scene)
__device__ __forceinline__ void solid_block_maxima(const Dev &D, int dim, int a0, int a1, float *shv, float *sha) {
  const int NS = D.ns;
  const int s0 = D.s_scene[a0], s1 = D.s_scene[a1 - 1];
  auto fmx = [](float x, float y) { return fmaxf(x, y); };
  for (int s = s0; s <= s1; ++s) {
    const ScenePar &P = D.par[s];
    float vm = 0.0f, am = 0.0f;
    for (int a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
      if (D.s_scene[a] != s || a - P.s_begin >= P.s_count - P.s_nclamp) continue;
      float v2 = 0.0f, a2 = 0.0f;
      for (int k = 0; k < dim; ++k) {
        float v = (float)D.s_v[k * NS + a], q = D.s_a[k * NS + a];
        v2 += v * v;
        a2 += q * q;
      }
      vm = fmaxf(vm, sqrtf(v2));
      am = fmaxf(am, sqrtf(a2));
    }
    vm = block_reduce(vm, fmx, shv);
    am = block_reduce(am, fmx, sha);
    if (threadIdx.x == 0) {
      atomic_max_pos(&D.st[s].smax_v, vm);
      atomic_max_pos(&D.st[s].smax_a, am);
    }
  }
}

__global__ void __launch_bounds__(256) k_solid_dt_reduce(Dev D) {
  __shared__ float shv[16], sha[16];
  const int dim = D.dim, NS = D.ns;
  const int span = blockDim.x * kReduceItems;
  const int a0 = blockIdx.x * span, a1 = min(NS, a0 + span);
  for (int a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
    for (int k = 0; k < dim; ++k) {
      D.s_du[k * NS + a] = 0.0;
      D.s_dv[k * NS + a] = 0.0;
    }
  }
  solid_block_maxima(D, dim, a0, a1, shv, sha);
}

// dt_S = cfl_s min(h_S / (c_S + |v|max), sqrt(h_S / |a|max)), kappa =
// floor(dt_ac / dt_S) + 1 (bounded: a collapsed solid step is reported).
__device__ __forceinline__ void solid_kappa(const ScenePar &P, SceneState &S, float vmax, float amax, double dt_ac,
                                            int &kap, double &dts) {
  dts = solid_dt(P, vmax, amax);
  double ratio = dt_ac / dts;
  if (!(ratio >= 0.0) || !(dt_ac > 0.0) || ratio > (double)(KAPPA_MAX - 1)) {
    kap = (ratio >= 0.0 && dt_ac > 0.0) ? KAPPA_MAX : 1;
    atomicOr(&S.err, (int)ERR_NAN_SOLID);
  } else {
    // one shared step: dt_ac <= dt_S was chosen at the step start
    kap = P.single_step ? 1 : (int)floor(ratio) + 1;
  }
}

// The next step's kappa and dt_S of scene s at the end of a step, from the
// solid maxima the step's averaging pass reduced and the next acoustic step;
// the error bits are latched by the step that adopts this evaluation.
__device__ void solid_kappa_next(const Dev &D, int s) {
  SceneState &S = D.st[s];
  int kap;
  double dts;
  const int err = S.err;
  solid_kappa(D.par[s], S, __uint_as_float(S.smax_v), __uint_as_float(S.smax_a), S.dt_ac, kap, dts);
  S.kappa_next_err = S.err & ~err;
  S.err = err;
  S.kappa_next = kap;
  S.dt_s_next = dts;
  S.smax_v = S.smax_a = 0u;
}

// The step starting now adopts that evaluation (nothing changes the solid in
// between); atomic on the error word, which passes running beside may set.
__device__ __forceinline__ void solid_kappa_adopt(SceneState &S) {
  S.kappa = S.kappa_next;
  S.dt_s = S.dt_s_next;
  if (S.kappa_next_err) atomicOr(&S.err, S.kappa_next_err);
}

// kappa and dt_S of the step starting now, from k_solid_dt_reduce's maxima
__global__ void k_solid_dt_close(Dev D) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= D.n_scenes) return;
  SceneState &S = D.st[s];
  int kap;
  double dts;
  solid_kappa(D.par[s], S, __uint_as_float(S.smax_v), __uint_as_float(S.smax_a), S.dt_ac, kap, dts);
  S.dt_s = dts;
  S.kappa = kap;
  S.smax_v = S.smax_a = 0u;
}

// First half of a sub-step for particle a (own state only), and its stress.
// Particle a's stress for the momentum pass: the own term P_a B_a sum_b g_ab
// in FP64 and P_a B_a in FP32 at record slot r (what the neighbours read).
template <int DIM>
__device__ __forceinline__ void solid_stress_store(const Dev &D, int a, int r, const double *PB) {
  const int NS = D.ns;
  double gs[3];
  for (int j = 0; j < DIM; ++j) gs[j] = D.s_gsum[j * NS + a];
  for (int i = 0; i < DIM; ++i) {
    double own = 0.0;
    for (int j = 0; j < DIM; ++j) own += PB[i * DIM + j] * gs[j];
    D.s_PBg[i * NS + a] = own;
  }
  for (int k = 0; k < DIM * DIM; ++k) D.s_PBf[pbf_at(D, r, k)] = (float)PB[k];
}

template <int DIM>
__device__ __forceinline__ void solid_first_half(const Dev &D, const ScenePar &P, SceneState &S, int a, double hd) {
  const int NS = D.ns;
  double H[9], B[9], PB[9];
  for (int k = 0; k < DIM * DIM; ++k) {
    H[k] = D.s_H[k * NS + a] + hd * D.s_dF[k * NS + a];
    D.s_H[k * NS + a] = H[k];
    B[k] = D.s_B[k * NS + a];
  }
  // the step's increments start here: du = the first half's, dv = 0
  for (int k = 0; k < DIM; ++k) {
    double inc = hd * D.s_v[k * NS + a];
    D.s_u[k * NS + a] += inc;
    D.s_du[k * NS + a] = inc;
    D.s_dv[k * NS + a] = 0.0;
  }
  double J;
  solid_PB<DIM, double>(P.material, H, B, (double)P.mu, (double)P.lam, PB, J);
  if (!(J > 0.0)) atomicOr(&S.err, (int)ERR_JACOBIAN);
  solid_stress_store<DIM>(D, a, rec_of(D, a), PB);
}

// First half of sub-step 0 (clamp particles: zero stress).  adopt: the step
// takes the kappa and dt_S that the step before evaluated at its end (its
// leading threads adopt them for every scene; the particles read kappa_next,
// which nothing here writes).
template <int DIM>
__global__ void __launch_bounds__(256) k_solid_first(Dev D, int adopt) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (adopt)
    for (int s = a; s < D.n_scenes; s += gridDim.x * blockDim.x) solid_kappa_adopt(D.st[s]);
  if (a >= D.ns) return;
  int s = D.s_scene[a];
  const ScenePar &P = D.par[s];
  SceneState &S = D.st[s];
  const int kappa = adopt ? S.kappa_next : S.kappa;
  if (a - P.s_begin >= P.s_count - P.s_nclamp) {
    const int r = rec_of(D, a);
    const int NS = D.ns;
    for (int k = 0; k < DIM; ++k) D.s_PBg[k * NS + a] = 0.0;
    for (int k = 0; k < DIM * DIM; ++k) D.s_PBf[pbf_at(D, r, k)] = 0.0f;
    D.s_vf[r] = make_float4((float)D.s_v[a], (float)D.s_v[NS + a], DIM == 3 ? (float)D.s_v[2 * NS + a] : 0.0f, 1.0f);
    return;
  }
  solid_first_half<DIM>(D, P, S, a, 0.5 * S.dt_ac / kappa);
}

// Momentum of free particle a: sum_b (P_a B_a + P_b B_b) g_ab = P_a B_a
// sum_b g_ab + sum_b P_b B_b g_ab, the own term in FP64 (here), the
// neighbours' P B in FP32 (their rounding reaches the acceleration scaled by
// about the ratio of the stress length scale to h).
template <int DIM>
__device__ __forceinline__ void solid_momentum_own(const Dev &D, int a, double *acc) {
  const int NS = D.ns;
  for (int i = 0; i < DIM; ++i) acc[i] = D.s_PBg[i * NS + a];
}

// Own state of free particle a that the momentum update reads besides its
// P B: the fluid force, v and the step's dv.
struct MomOwn {
  float fF[3];
  double v[3], dv[3];
};
template <int DIM>
__device__ __forceinline__ void solid_momentum_load(const Dev &D, int a, MomOwn &o) {
  const int NS = D.ns;
  for (int k = 0; k < DIM; ++k) {
    o.fF[k] = D.s_fF[k * NS + a];
    o.v[k] = D.s_v[k * NS + a];
    o.dv[k] = D.s_dv[k * NS + a];
  }
}

// Acceleration, velocity and velocity record (slot r) of free particle a
// from the own term acc and the FP32 neighbour sum accn.
template <int DIM>
__device__ __forceinline__ void solid_momentum_finish(const Dev &D, const ScenePar &P, const SceneState &S, int a,
                                                      int r, const double *acc, const float *accn, const MomOwn &o) {
  const int NS = D.ns;
  const double del = S.dt_ac / S.kappa;
  const double m_inv = 1.0 / ((double)P.rho0s * (double)P.Vs);
  double vn[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < DIM; ++k) {
    double ak = ((double)P.Vs * (acc[k] + (double)accn[k]) + (double)o.fF[k]) * m_inv + (double)P.g[k];
    D.s_a[k * NS + a] = (float)ak;
    double dv = del * ak;
    vn[k] = o.v[k] + dv;
    D.s_v[k * NS + a] = vn[k];
    D.s_dv[k * NS + a] = o.dv[k] + dv;
  }
  D.s_vf[r] = make_float4((float)vn[0], (float)vn[1], (float)vn[2], 1.0f);
}

// Momentum and velocity of free particle a in the current sub-step, its
// velocity record at slot r; acc holds the own term and walk(accn) adds sum_b
// P_b B_b g_ab over a's reference neighbours in FP32.
template <int DIM, class Walk>
__device__ __forceinline__ void solid_momentum_at(const Dev &D, const ScenePar &P, const SceneState &S, int a, int r,
                                                  const double *acc, Walk walk) {
  float accn[3] = {0.0f, 0.0f, 0.0f};
  walk(accn);
  MomOwn o;
  solid_momentum_load<DIM>(D, a, o);
  solid_momentum_finish<DIM>(D, P, S, a, r, acc, accn, o);
}

// Deformation rate of free particle a with the new velocity and second half
// of sub-step `sub`; then the first half and stress of the next sub-step,
// its FP32 P B at record slot r.  walk(Gn) adds sum_b (v_b - v_a) (x) g_ab
// over a's reference neighbours in FP32: the neighbours' v as one FP32
// record each, the differences v_b - v_a taken between FP32-rounded values
// (so a rigid translation still gives exactly zero).
// kPre: B and H loaded before the walk.
template <int DIM, bool kPre = false, class Walk>
__device__ __forceinline__ void solid_rate_at(const Dev &D, const ScenePar &P, SceneState &S, int a, int r, int sub,
                                              Walk walk) {
  const int NS = D.ns;
  const double hd = 0.5 * S.dt_ac / S.kappa;
  double H[9], B[9];
  auto load = [&]() {
    for (int k = 0; k < DIM * DIM; ++k) {
      B[k] = D.s_B[k * NS + a];
      H[k] = D.s_H[k * NS + a];
    }
  };
  if (kPre) load();
  float Gn[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  walk(Gn);
  double va[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < DIM; ++k) va[k] = D.s_v[k * NS + a];
  double G[9];
  for (int k = 0; k < DIM * DIM; ++k) G[k] = (double)Gn[k];
  // (v_b - v_a) (x) (B grad W) summed = G B^T; then, for a following
  // sub-step, its first half on the values still in registers (the same
  // arithmetic as solid_first_half, without reading back what was just
  // written)
  const bool more = sub + 1 < S.kappa;
  if (!kPre) load();
  for (int i = 0; i < DIM; ++i)
    for (int j = 0; j < DIM; ++j) {
      double sum = 0.0;
      for (int k = 0; k < DIM; ++k) sum += G[i * DIM + k] * B[j * DIM + k];
      D.s_dF[(i * DIM + j) * NS + a] = sum;
      const double h1 = H[i * DIM + j] + hd * sum;
      H[i * DIM + j] = more ? h1 + hd * sum : h1;
      D.s_H[(i * DIM + j) * NS + a] = H[i * DIM + j];
    }
  for (int k = 0; k < DIM; ++k) {
    const double inc = hd * va[k];
    const double u1 = D.s_u[k * NS + a] + inc, du1 = D.s_du[k * NS + a] + inc;
    D.s_u[k * NS + a] = more ? u1 + inc : u1;
    D.s_du[k * NS + a] = more ? du1 + inc : du1;
  }
  if (more) {
    double PB[9], J;
    solid_PB<DIM, double>(P.material, H, B, (double)P.mu, (double)P.lam, PB, J);
    if (!(J > 0.0)) atomicOr(&S.err, (int)ERR_JACOBIAN);
    solid_stress_store<DIM>(D, a, r, PB);
  }
}

// Momentum and velocity of sub-step `sub`, one thread per solid particle
// walking its reference table (the neighbours' P B gathered per pair, the
// gathers bound this pass).
template <int DIM>
__global__ void __launch_bounds__(256) k_solid_momentum(Dev D, int sub) {
  __shared__ float4 gcl[kNbrClasses];
  const bool compact = DIM == 3 && D.nbr_compact;
  if (compact) {
    if (threadIdx.x < kNbrClasses) gcl[threadIdx.x] = D.s_gcls[threadIdx.x];
    __syncthreads();
  }
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= D.ns) return;
  int s = D.s_scene[a];
  const ScenePar &P = D.par[s];
  SceneState &S = D.st[s];
  if (sub >= S.kappa || a - P.s_begin >= P.s_count - P.s_nclamp) return;
  const int NS = D.ns;
  double acc[3];
  solid_momentum_own<DIM>(D, a, acc);
  solid_momentum_at<DIM>(D, P, S, a, a, acc, [&](float *accn) {
    int cnt = D.s_cnt[a];
    auto pair = [&](int b, const float4 &g) {
      float gv[3] = {g.x, g.y, g.z};
      float PBb[9];
      for (int k = 0; k < DIM * DIM; ++k) PBb[k] = D.s_PBf[pb_at(D, b, k)];
      for (int i = 0; i < DIM; ++i)
        for (int j = 0; j < DIM; ++j) accn[i] += PBb[i * DIM + j] * gv[j];
    };
    if (compact) {
#pragma unroll 4
      for (int q = 0; q < cnt; ++q) {
        const unsigned e = D.s_nbc[(size_t)q * NS + a];
        pair((int)(e >> 7), gcl[e & 127u]);
      }
    } else {
#pragma unroll 4
      for (int q = 0; q < cnt; ++q) {
        const float4 g = D.s_nbr[(size_t)q * NS + a];
        pair(__float_as_int(g.w), g);
      }
    }
  });
}

// Deformation rate and second half of sub-step `sub` (then the next one's
// first half), one thread per solid particle walking its reference table.
template <int DIM>
__global__ void __launch_bounds__(256) k_solid_rate(Dev D, int sub) {
  __shared__ float4 gcl[kNbrClasses];
  const bool compact = DIM == 3 && D.nbr_compact;
  if (compact) {
    if (threadIdx.x < kNbrClasses) gcl[threadIdx.x] = D.s_gcls[threadIdx.x];
    __syncthreads();
  }
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= D.ns) return;
  int s = D.s_scene[a];
  const ScenePar &P = D.par[s];
  SceneState &S = D.st[s];
  if (sub >= S.kappa || a - P.s_begin >= P.s_count - P.s_nclamp) return;
  const int NS = D.ns;
  float vaf[3] = {0.0f, 0.0f, 0.0f};
  for (int k = 0; k < DIM; ++k) vaf[k] = (float)D.s_v[k * NS + a];
  solid_rate_at<DIM>(D, P, S, a, a, sub, [&](float *Gn) {
    int cnt = D.s_cnt[a];
    auto pair = [&](int b, const float4 &g) {
      float gv[3] = {g.x, g.y, g.z};
      float4 vb = D.s_vf[b];
      float vbv[3] = {vb.x, vb.y, vb.z};
      for (int i = 0; i < DIM; ++i) {
        float dvi = vbv[i] - vaf[i];
        for (int j = 0; j < DIM; ++j) Gn[i * DIM + j] += dvi * gv[j];
      }
    };
    if (compact) {
#pragma unroll 4
      for (int q = 0; q < cnt; ++q) {
        const unsigned e = D.s_nbc[(size_t)q * NS + a];
        pair((int)(e >> 7), gcl[e & 127u]);
      }
    } else {
#pragma unroll 4
      for (int q = 0; q < cnt; ++q) {
        const float4 g = D.s_nbr[(size_t)q * NS + a];
        pair(__float_as_int(g.w), g);
      }
    }
  });
}

// Lattice blocks (3D): one workgroup per block of kLatB0 x kLatB1 x kLatB2
// lattice cells of one scene, a thread per cell (the fastest storage axis
// fastest across the lanes).  The FP32 records are kept in cell order, so the
// workgroup stages those of the cells within kLatR spacings (zeros for empty
// ones) in LDS with coalesced loads and no index lookups, and each free
// particle sums over the offset classes at fixed shifts from its own halo
// position: every pair becomes three LDS reads at the class's shift, with
// no table entry and no gather.  The set summed over is the reference table's
// (checked at set-up), the order the classes'.

// the block of the list this workgroup takes (-1: none); the grid is
// kXcds * ceil(lat_nblocks / kXcds) workgroups
__device__ __forceinline__ int lat_block(const Dev &D) {
  const int per = (D.lat_nblocks + kXcds - 1) / kXcds;
  const int b = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
  return b < D.lat_nblocks ? b : -1;
}

// Halo cell q of this thread (cells threadIdx.x + q * kLatThreads) of block
// blk: c its grid index (-1 outside the scene's bounding box), l its LDS
// position.
constexpr int kLatPer = kLatHalo / kLatThreads;
static_assert(kLatHalo % kLatThreads == 0, "every thread stages kLatPer halo cells");
__device__ __forceinline__ void lat_halo_cell(const int4 &L, const int4 &blk, int q, int &c, int &l) {
  const int i = threadIdx.x + q * kLatThreads;
  const int h0 = i / (kLatH1 * kLatH2), h12 = i - h0 * (kLatH1 * kLatH2);
  const int h1 = h12 / kLatH2, h2 = h12 - h1 * kLatH2;
  const int c0 = blk.y - kLatR + h0, c1 = blk.z - kLatR + h1, c2 = blk.w - kLatR + h2;
  const bool in = (unsigned)c0 < (unsigned)L.y && (unsigned)c1 < (unsigned)L.z && (unsigned)c2 < (unsigned)L.w;
  c = in ? L.x + (c0 * L.z + c1) * L.w + c2 : -1;
  l = h1 * kLatRow + h0 * kLatH2 + h2;
}

// Stage rec(cell, lds) for every halo cell of block blk.
template <class Rec>
__device__ __forceinline__ void lat_stage(const int4 &L, const int4 &blk, Rec rec) {
#pragma unroll
  for (int q = 0; q < kLatPer; ++q) {
    int c, l;
    lat_halo_cell(L, blk, q, c, l);
    rec(c, l);
  }
}

// This thread's cell of block blk: its grid index (-1 outside the bounding
// box) and its LDS position.
__device__ __forceinline__ int lat_own(const int4 &L, const int4 &blk, int &pos) {
  const int t = threadIdx.x;
  const int t0 = t / (kLatB1 * kLatB2), t12 = t - t0 * (kLatB1 * kLatB2);
  const int t1 = t12 / kLatB2, t2 = t12 - t1 * kLatB2;
  pos = (t1 + kLatR) * kLatRow + (t0 + kLatR) * kLatH2 + (t2 + kLatR);
  const int c0 = blk.y + t0, c1 = blk.z + t1, c2 = blk.w + t2;
  const bool in = (unsigned)c0 < (unsigned)L.y && (unsigned)c1 < (unsigned)L.z && (unsigned)c2 < (unsigned)L.w;
  return in ? L.x + (c0 * L.z + c1) * L.w + c2 : -1;
}

// Jittered lattice (lat_jitter): V_b grad_a W(r) of a pair in FP32 from
// r = X_a - X_b = (the class's lattice vector) + (offset of a) - (offset of
// b), the offsets staged in LDS after the pass's own components (jt), and
// the same kernel as the reference table: g = r Vs (-5 alpha / h^2) t^3 with
// t = max(0, 1 - |r| / (2 h)) (zero beyond the support).
struct LatKernel {
  float kc, inv2h;
};
__device__ __forceinline__ LatKernel lat_kernel(const ScenePar &P) {
  const double h = P.hs, alpha = 21.0 / (16.0 * M_PI * h * h * h);
  return {(float)(-5.0 * alpha * (double)P.Vs / (h * h)), (float)(0.5 / h)};
}
__device__ __forceinline__ void lat_pair_gradient(const LatKernel &K, const float4 &cls, const float *ja,
                                                  const float *jb, float *g) {
  const float r[3] = {cls.x + (ja[0] - jb[0]), cls.y + (ja[kLatLds] - jb[kLatLds]),
                      cls.z + (ja[2 * kLatLds] - jb[2 * kLatLds])};
  const float rr = sqrtf(fmaf(r[0], r[0], fmaf(r[1], r[1], r[2] * r[2])));
  const float t = fmaxf(0.0f, fmaf(-rr, K.inv2h, 1.0f));
  const float f = K.kc * (t * t * t);
  for (int k = 0; k < 3; ++k) g[k] = r[k] * f;
}

// Momentum pass on lattice blocks: the halo's FP32 P B in LDS one row of
// three components at a time (17 KB, so that LDS admits eight workgroups per
// CU; all nine at once held it to three).
//
// kJit: all nine components and the halo's offsets at once (68 KB, two
// workgroups per CU), each pair's gradient formed once for the three rows.
template <bool kJit>
__global__ void __launch_bounds__(kLatThreads) k_solid_momentum_lat(Dev D, int sub) {
  __shared__ float pb[(kJit ? 12 : 3) * kLatLds];
  float *jt = pb + 9 * kLatLds;  // kJit: the halo's offsets
  const int bi = lat_block(D);
  if (bi < 0) return;
  const int4 blk = D.lat_blocks[bi];
  const ScenePar &P = D.par[blk.x];
  SceneState &S = D.st[blk.x];
  if (sub >= S.kappa) return;
  const int4 L = D.lat_scene[blk.x];
  int pos;
  const int cell = lat_own(L, blk, pos);
  const int a = cell >= 0 ? D.lat_grid[cell] : -1;
  const bool act = a >= 0 && a - P.s_begin < P.s_count - P.s_nclamp;
  // the own term's loads in flight with the staging (the rest of the own
  // state loaded there too measured slower)
  double acc[3] = {0.0, 0.0, 0.0};
  if (act) solid_momentum_own<3>(D, a, acc);
  const size_t NC = D.lat_ncells;
  float accr[3] = {0.0f, 0.0f, 0.0f};
  if constexpr (kJit) {
    lat_stage(L, blk, [&](int c, int l) {
#pragma unroll
      for (int k = 0; k < 9; ++k) pb[k * kLatLds + l] = c >= 0 ? D.s_PBf[k * NC + c] : 0.0f;
#pragma unroll
      for (int k = 0; k < 3; ++k) jt[k * kLatLds + l] = c >= 0 ? D.lat_jit[k * NC + c] : 0.0f;
    });
    const LatKernel K = lat_kernel(P);
    __syncthreads();
    if (!act) return;
    const float *r0 = pb + pos;
    const int nc = D.lat_ncls;
#pragma unroll 2
    for (int j = 0; j < nc; ++j) {
      const float4 e = D.lat_cls[j];
      const int sh = __float_as_int(e.w);
      float gv[3];
      lat_pair_gradient(K, e, jt + pos, jt + pos + sh, gv);
      const float *r = r0 + sh;
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) accr[i] += r[(3 * i + k) * kLatLds] * gv[k];
    }
    MomOwn o;
    solid_momentum_load<3>(D, a, o);
    solid_momentum_finish<3>(D, P, S, a, cell, acc, accr, o);
    return;
  }
  // row i + 1's halo loaded into registers while row i is walked
  float stg[kLatPer][3];
  auto fetch = [&](int i) {
#pragma unroll
    for (int q = 0; q < kLatPer; ++q) {
      int c, l;
      lat_halo_cell(L, blk, q, c, l);
#pragma unroll
      for (int k = 0; k < 3; ++k) stg[q][k] = c >= 0 ? D.s_PBf[(3 * i + k) * NC + c] : 0.0f;
    }
  };
  fetch(0);
  for (int i = 0; i < 3; ++i) {
    if (i > 0) __syncthreads();  // row i - 1 walked
#pragma unroll
    for (int q = 0; q < kLatPer; ++q) {
      int c, l;
      lat_halo_cell(L, blk, q, c, l);
#pragma unroll
      for (int k = 0; k < 3; ++k) pb[k * kLatLds + l] = stg[q][k];
    }
    __syncthreads();
    if (i < 2) fetch(i + 1);
    if (act) {
      const float *r0 = pb + pos;
      const int nc = D.lat_ncls;
      float sum = 0.0f;
#pragma unroll 4
      for (int j = 0; j < nc; ++j) {
        const float4 g = D.lat_cls[j];
        const float gv[3] = {g.x, g.y, g.z};
        const float *r = r0 + __float_as_int(g.w);
        for (int k = 0; k < 3; ++k) sum += r[k * kLatLds] * gv[k];
      }
      accr[i] = sum;
    }
  }
  if (!act) return;
  MomOwn o;
  solid_momentum_load<3>(D, a, o);
  solid_momentum_finish<3>(D, P, S, a, cell, acc, accr, o);
}

// Rate pass on lattice blocks: the halo's FP32 v and presence weight (1 for
// a cell with a particle, 0 for an empty one) in LDS (kJit: and the offsets).
template <bool kJit>
__global__ void __launch_bounds__(kLatThreads) k_solid_rate_lat(Dev D, int sub) {
  __shared__ float vh[(kJit ? 7 : 4) * kLatLds];
  float *jt = vh + 4 * kLatLds;
  const int bi = lat_block(D);
  if (bi < 0) return;
  const int4 blk = D.lat_blocks[bi];
  const ScenePar &P = D.par[blk.x];
  SceneState &S = D.st[blk.x];
  if (sub >= S.kappa) return;
  const int4 L = D.lat_scene[blk.x];
  int pos;
  const int cell = lat_own(L, blk, pos);
  const int a = cell >= 0 ? D.lat_grid[cell] : -1;
  lat_stage(L, blk, [&](int c, int l) {
    const float4 v = c >= 0 ? D.s_vf[c] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    vh[l] = v.x;
    vh[kLatLds + l] = v.y;
    vh[2 * kLatLds + l] = v.z;
    vh[3 * kLatLds + l] = v.w;
    if (kJit) {
      const size_t NC = D.lat_ncells;
#pragma unroll
      for (int k = 0; k < 3; ++k) jt[k * kLatLds + l] = c >= 0 ? D.lat_jit[k * NC + c] : 0.0f;
    }
  });
  const LatKernel K = lat_kernel(P);
  __syncthreads();
  if (a < 0 || a - P.s_begin >= P.s_count - P.s_nclamp) return;
  // B and H in flight during the LDS walk
  solid_rate_at<3, true>(D, P, S, a, cell, sub, [&](float *Gn) {
    const float *r0 = vh + pos;
    // v_a rounded to FP32 is the particle's own record
    const float vaf[3] = {r0[0], r0[kLatLds], r0[2 * kLatLds]};
    const int nc = D.lat_ncls;
#pragma unroll 8
    for (int j = 0; j < nc; ++j) {
      const float4 g = D.lat_cls[j];
      float gv[3] = {g.x, g.y, g.z};
      const float *r = r0 + __float_as_int(g.w);
      if (kJit) lat_pair_gradient(K, g, jt + pos, jt + pos + __float_as_int(g.w), gv);
      const float w = r[3 * kLatLds];
      for (int i = 0; i < 3; ++i) {
        // (v_b - v_a) exactly for a particle, zero for an empty cell
        const float dvi = (r[i * kLatLds] - vaf[i]) * w;
        for (int k = 0; k < 3; ++k) Gn[i * 3 + k] += dvi * gv[k];
      }
    }
  });
}

// Time averages over the acoustic step, kReduceItems particles per thread.
// maxima: also the free solid's max |v| and |a| after the step's last
// sub-step (as k_solid_dt_reduce takes them, for the next step's kappa; one
// atomic per block and scene).
template <int DIM>
__global__ void __launch_bounds__(256) k_solid_average(Dev D, int launched, int maxima) {
  __shared__ float shv[16], sha[16];
  const int NS = D.ns;
  const int span = blockDim.x * kReduceItems;
  const int a0 = blockIdx.x * span, a1 = min(NS, a0 + span);
  for (int a = a0 + threadIdx.x; a < a1; a += blockDim.x) {
    const int s = D.s_scene[a];
    const ScenePar &P = D.par[s];
    SceneState &S = D.st[s];
    if (a == P.s_begin && S.kappa > launched) atomicOr(&S.err, (int)ERR_KAPPA);
    if (a - P.s_begin >= P.s_count - P.s_nclamp) continue;
    const double inv_dt = 1.0 / S.dt_ac;
    bool bad = false;
    for (int k = 0; k < DIM; ++k) {
      float vb = (float)(D.s_du[k * NS + a] * inv_dt), ab = (float)(D.s_dv[k * NS + a] * inv_dt);
      D.s_vbar[k * NS + a] = vb;
      D.s_abar[k * NS + a] = ab;
      bad |= !isfinite(vb) || !isfinite(ab);
    }
    if (bad) atomicOr(&S.err, (int)ERR_NAN_SOLID);
  }
  if (maxima) solid_block_maxima(D, DIM, a0, a1, shv, sha);
}

// Hand-over of free solid particle a's step results to its boundary particle
// seen by the fluid: current volume V0 det F, averaged velocity and the
// hydrostatic factor max(0, (abar - g).n).
template <int DIM>
__device__ __forceinline__ void hand_over_values(const Dev &D, const ScenePar &P, int a, double J, const float *vbar,
                                                 const float *abar) {
  const int NS = D.ns;
  const int kslot = D.s_bslot[a];
  if (kslot < 0) return;
  float sa = 0.0f;
  for (int k = 0; k < DIM; ++k) sa += (abar[k] - P.g[k]) * D.s_n[k * NS + a];
  float4 bp = D.b_pos[kslot];
  bp.w = (float)(P.Vs * J);
  D.b_pos[kslot] = bp;
  D.b_vbar[kslot] = make_float4(vbar[0], vbar[1], DIM == 3 ? vbar[2] : 0.0f, fmaxf(0.0f, sa));
}

template <int DIM>
__device__ __forceinline__ double det_F(const double *H) {
  if (DIM == 2) return (1.0 + H[0]) * (1.0 + H[3]) - H[1] * H[2];
  return (1.0 + H[0]) * ((1.0 + H[4]) * (1.0 + H[8]) - H[5] * H[7]) - H[1] * (H[3] * (1.0 + H[8]) - H[5] * H[6]) +
         H[2] * (H[3] * H[7] - (1.0 + H[4]) * H[6]);
}

// The same from the stored state (solid index a, any free particle).
template <int DIM>
__device__ void hand_over(const Dev &D, int a) {
  const int NS = D.ns;
  if (a >= NS) return;
  const ScenePar &P = D.par[D.s_scene[a]];
  if (a - P.s_begin >= P.s_count - P.s_nclamp) return;
  double H[9];
  for (int k = 0; k < DIM * DIM; ++k) H[k] = D.s_H[k * NS + a];
  float vbar[3] = {0.0f, 0.0f, 0.0f}, abar[3] = {0.0f, 0.0f, 0.0f};
  for (int k = 0; k < DIM; ++k) {
    vbar[k] = D.s_vbar[k * NS + a];
    abar[k] = D.s_abar[k * NS + a];
  }
  hand_over_values<DIM>(D, P, a, det_F<DIM>(H), vbar, abar);
}

__device__ void fluid_step_end(const Dev &D, int blk, float *shm, unsigned long long (*shc)[16]);

// Sub-step surrogate schedule (2D).  Per scene and step the mode is:
//   judge step: the plain sub-steps run and stand, and the network's
//     averages are compared with theirs over the N free particles,
//     R = max(|dvbar|_2 / (|vbar|_2 + |g| dt sqrt(N)),
//             |dabar|_2 / (|abar|_2 + |g| sqrt(N)));
//     R <= threshold opens a window of every - 1 learned steps, else every - 1
//     plain steps follow (a non-finite R fails);
//   learned step: the predicted averages advance the solid (u += dt vbar,
//     v += dt abar, F from the corrected gradient of vbar, a = abar) and the
//     sub-steps are skipped;
//   plain step: the plain sub-steps, no network.
// The first step after the network is set is a judge step.  Exact averages
// give R = 0 and pass any threshold.

// mode of scene S's current step from the schedule its last judge set
__device__ __forceinline__ int sur_mode(const SceneState &S) {
  if (S.sur_window > 0) return kSurLearned;
  return S.sur_countdown <= 0 ? kSurJudge : kSurPlain;
}

// The schedule after a step of the given mode (one thread of the scene's
// block; sums over the free particles for a judge step).
__device__ __forceinline__ void sur_schedule(const Dev &D, const ScenePar &P, SceneState &S, int mode, double dv2,
                                             double v2, double da2, double a2) {
  const int every = D.sur_every > 0 ? D.sur_every : 1;
  if (mode == kSurLearned) {
    S.sur_window -= 1;  // the judge step follows the last learned step
  } else if (mode == kSurJudge) {
    const int nfree = P.s_count - P.s_nclamp;
    const double gabs = sqrt((double)P.g[0] * P.g[0] + (double)P.g[1] * P.g[1]);
    const double rn = sqrt((double)(nfree > 0 ? nfree : 1));
    const double rv = sqrt(dv2) / (sqrt(v2) + gabs * S.dt_ac * rn + 1e-300);
    const double ra = sqrt(da2) / (sqrt(a2) + gabs * rn + 1e-300);
    const double R = nfree > 0 ? fmax(rv, ra) : __builtin_nan("");
    S.sur_last_r = (rv != rv || ra != ra) ? __builtin_nan("") : R;
    const bool ok = S.sur_last_r <= (double)D.sur_thr;  // false for NaN
    if (ok) {
      S.sur_judge_ok += 1;
      S.sur_window = every - 1;
      S.sur_countdown = 0;
    } else {
      S.sur_judge_fail += 1;
      S.sur_window = 0;
      S.sur_countdown = every - 1;
    }
  } else if (mode == kSurPlain) {
    S.sur_countdown -= 1;
  }
}

// A learned step's solid update of the block's scene: the predicted vbar of
// its particles staged in LDS (vb, two doubles each), then per free particle
// dF/dt = sum_b (vbar_b - vbar_a) (x) g_ab B^T (the corrected gradient of
// Section 2.2), F += dt dF/dt, u += dt vbar, v += dt abar, and the predicted
// averages stored as the step's, the acceleration as abar.
__device__ void sur_learned_block(const Dev &D, const ScenePar &P, const SceneState &S, double *vb) {
  const int NS = D.ns, base = P.s_begin, n = P.s_count, nfree = n - P.s_nclamp;
  const int t = threadIdx.x, T = blockDim.x;
  for (int l = t; l < n; l += T) {
    vb[2 * l] = D.sur_vbar[base + l];
    vb[2 * l + 1] = D.sur_vbar[NS + base + l];
  }
  __syncthreads();
  const double dt = S.dt_ac;
  for (int l = t; l < nfree; l += T) {
    const int a = base + l;
    const double va0 = vb[2 * l], va1 = vb[2 * l + 1];
    double G[4] = {0.0, 0.0, 0.0, 0.0};
    const int cnt = D.s_cnt[a];
#pragma unroll 4
    for (int q = 0; q < cnt; ++q) {
      const float4 g = D.s_nbr[(size_t)q * NS + a];
      const int b = __float_as_int(g.w) - base;
      const double d0 = vb[2 * b] - va0, d1 = vb[2 * b + 1] - va1;
      G[0] += d0 * (double)g.x;
      G[1] += d0 * (double)g.y;
      G[2] += d1 * (double)g.x;
      G[3] += d1 * (double)g.y;
    }
    double B[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) B[k] = D.s_B[k * NS + a];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const double dF = G[i * 2] * B[j * 2] + G[i * 2 + 1] * B[j * 2 + 1];
        D.s_H[(i * 2 + j) * NS + a] += dt * dF;
        D.s_dF[(i * 2 + j) * NS + a] = dF;
      }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const float vbk = D.sur_vbar[k * NS + a], abk = D.sur_abar[k * NS + a];
      D.s_u[k * NS + a] += dt * (double)vbk;
      D.s_v[k * NS + a] += dt * (double)abk;
      D.s_a[k * NS + a] = abk;
      D.s_vbar[k * NS + a] = vbk;
      D.s_abar[k * NS + a] = abk;
    }
  }
}

// Split form of the block-resident kernel: the workgroups of one scene meet
// at a barrier on the scene's count in global memory (thread 0 of each; the
// caller brackets it with __syncthreads).  `round` counts the launch's
// barriers from 1.  A wait beyond the spin limit, or one that finds the
// scene already failed, latches ERR_PARTS and returns: the workgroups then
// run to their end without waiting, and the step is reported.
constexpr long long kPartsSpinLimit = 1LL << 22;
__device__ __forceinline__ void parts_barrier(const Dev &D, int s, int nparts, unsigned round) {
  unsigned *bar = D.parts_sync + 4 * s + 2;
  int *err = &D.st[s].err;
  __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned target = round * (unsigned)nparts;
  // poll without ordering, then one acquire: the polls do not drop the caches
  for (long long n = 0; __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++n) {
    if (n > kPartsSpinLimit || (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_PARTS)) {
      atomicOr(err, (int)ERR_PARTS);
      break;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Exchange of `rec` doubles per particle between the workgroups of a scene:
// the own slice [l0, l1) of the LDS records (stride `stride`) to global
// memory, the barrier, then the records of the other free particles in
// [lo, hi), the range that the slice's reference neighbours span.
__device__ __forceinline__ void parts_exchange(const Dev &D, int s, int nparts, unsigned &round, double *lds,
                                               int stride, int rec, double *glob, int base, int l0, int l1, int lo,
                                               int hi) {
  const int t = threadIdx.x, T = blockDim.x;
  for (int i = t; i < (l1 - l0) * rec; i += T) {
    const int l = l0 + i / rec, k = i - (i / rec) * rec;
    glob[(size_t)(base + l) * rec + k] = lds[l * stride + k];
  }
  __syncthreads();
  ++round;
  if (t == 0) parts_barrier(D, s, nparts, round);
  __syncthreads();
  const int before = l0 - lo, others = before + (hi - l1);
  for (int i = t; i < others * rec; i += T) {
    int l = i / rec;
    const int k = i - l * rec;
    l += l < before ? lo : l1 - before;  // [lo, l0) then [l1, hi)
    lds[l * stride + k] = glob[(size_t)(base + l) * rec + k];
  }
  __syncthreads();
}

// The range [lo, hi) of free particles that the reference neighbours of
// each split workgroup's slice span (with the slice itself), packed into the
// map's fourth word as lo | hi << 16; once at set-up.
__global__ void __launch_bounds__(256) k_parts_range(Dev D) {
  __shared__ int sh[2][16];
  int4 &m = D.s_parts[blockIdx.x];
  const ScenePar &P = D.par[m.x];
  const int nfree = P.s_count - P.s_nclamp, base = P.s_begin;
  const int chunk = (nfree + m.z - 1) / m.z;
  const int l0 = min(nfree, m.y * chunk), l1 = min(nfree, l0 + chunk);
  int lo = l0, hi = l1;
  for (int l = l0 + threadIdx.x; l < l1; l += blockDim.x) {
    const int a = base + l, cnt = D.s_cnt[a];
    for (int q = 0; q < cnt; ++q) {
      const int b = __float_as_int(D.s_nbr[(size_t)q * D.ns + a].w) - base;
      if (b < nfree) {
        lo = min(lo, b);
        hi = max(hi, b + 1);
      }
    }
  }
  lo = block_reduce(lo, [](int x, int y) { return min(x, y); }, sh[0]);
  hi = block_reduce(hi, [](int x, int y) { return max(x, y); }, sh[1]);
  if (threadIdx.x == 0) m.w = lo | (hi << 16);
}

// The same sub-steps for 2D scenes whose free solid fits the block with at
// most PPT particles per thread: each thread keeps its particles' own state
// (H, dF/dt, u in FP64; B and the step increments in FP32) in registers for
// the whole launch, v and P B of the scene live in LDS (one record per
// particle, so a neighbour's values arrive in wide reads), and only the fixed
// reference neighbour table is read from (L2-resident) global memory inside
// the sub-step loop.
// Block limits keep the register budget: 1024 threads for one particle per
// thread (4 waves per SIMD), 768 for two (3 waves per SIMD), 512 for four.
// With D.solid_map a scene may run on several workgroups: each keeps a
// contiguous slice of the free particles in registers and the whole scene's
// P B and v in LDS, and the slices' new values are exchanged through global
// memory after each half sub-step (parts_exchange); kappa comes from the
// scene's maxima over all slices.  The sums of every particle are the ones
// of the single-workgroup form, term for term.
template <int DIM, int PPT>
__global__ void __launch_bounds__(PPT == 1 ? 1024 : (PPT == 2 ? 768 : 512)) k_solid_reg(Dev D, int lds_n) {
  extern __shared__ __align__(16) double smem[];
  __shared__ float red[2][16];
  __shared__ int kap_sh;
  __shared__ double del_sh;
  __shared__ unsigned long long end_c[3][16];
  __shared__ double sur_red[4][16];
  constexpr int D2 = DIM * DIM;
  const int nsb = D.solid_map ? D.solid_map_n : D.n_scenes;
  if ((int)blockIdx.x >= nsb) {
    // blocks beside the scenes' solid blocks end the step of the fluid: its
    // speed and pair-count reductions, and the binning of fluid and walls for
    // a rebuild that the closing step sets
    const int b = blockIdx.x - nsb;
    if (b < D.end_fluid_blocks) fluid_step_end(D, b, red[0], end_c);
    else bin_entry<DIM>(D, (b - D.end_fluid_blocks) * blockDim.x + threadIdx.x, true, kBinFluid | kBinWalls);
    return;
  }
  int s = blockIdx.x, part = 0, nparts = 1, span = 0;
  if (D.solid_map) {
    const int4 m = D.solid_map[blockIdx.x];
    s = m.x;
    part = m.y;
    nparts = m.z;
    span = m.w;
  }
  const ScenePar &P = D.par[s];
  SceneState &S = D.st[s];
  const int NS = D.ns;
  const int base = P.s_begin, n = P.s_count, nfree = P.s_count - P.s_nclamp;
  // this workgroup's slice [l0, l1) of the free particles
  const int chunk = (nfree + nparts - 1) / nparts;
  const int l0 = min(nfree, part * chunk), l1 = min(nfree, l0 + chunk);
  // the free particles the slice's neighbours span (split form)
  const int lo = nparts > 1 ? (span & 0xFFFF) : 0, hi = nparts > 1 ? (span >> 16) : nfree;
  unsigned round = 0;
  const int T = blockDim.x, t = threadIdx.x;
  constexpr int PR = solid_pb_record(DIM);
  double *PBx = smem;
  double *Vx = smem + PR * lds_n;
  // one LDS record per particle: a neighbour's P B (or v) arrives in wide reads
  auto PI = [&](int l, int k) { return (int)__umul24((unsigned)l, (unsigned)PR) + k; };
  auto VI = [&](int l, int k) { return l * DIM + k; };
  const int smode = DIM == 2 ? S.sur : kSurOff;  // the surrogate's mode of this step
  if (smode == kSurLearned) {
    // a learned step: the network's averages advance the solid instead of
    // the sub-steps (each thread updates the particles it ends the step of)
    if constexpr (DIM == 2) sur_learned_block(D, P, S, Vx);
    if (t == 0) sur_schedule(D, P, S, smode, 0.0, 0.0, 0.0, 0.0);
    if (D.solid_step_end) {
      const bool rb = rebuilds_next(S);
      float sv = 0.0f, sa = 0.0f;
      for (int l = t; l < nfree; l += T) {
        const int a = base + l;
        hand_over<DIM>(D, a);
        if (rb) bin_entry<DIM>(D, D.nf + P.b_begin + P.w_count + l, true, kBinSolid);
        float v2 = 0.0f, a2 = 0.0f;
        for (int k = 0; k < DIM; ++k) {
          const float v = (float)D.s_v[k * NS + a], q = D.s_a[k * NS + a];
          v2 += v * v;
          a2 += q * q;
        }
        sv = fmaxf(sv, sqrtf(v2));
        sa = fmaxf(sa, sqrtf(a2));
      }
      if (P.single_step) {
        auto fmx = [](float x, float y) { return fmaxf(x, y); };
        sv = block_reduce(sv, fmx, red[0]);
        sa = block_reduce(sa, fmx, red[1]);
        if (t == 0) {
          S.send_v = __float_as_uint(sv);
          S.send_a = __float_as_uint(sa);
        }
      }
    }
    return;
  }
  double dt_ac = S.dt_ac;
  // own particles and their state
  int la[PPT];
  bool own[PPT];
  double H[PPT][D2], dF[PPT][D2], u[PPT][DIM];
  float B[PPT][D2], du[PPT][DIM], dv[PPT][DIM], fF[PPT][DIM], acc_last[PPT][DIM];
  float vm = 0.0f, am = 0.0f;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    la[p] = l0 + t + p * T;
    own[p] = la[p] < l1;
    int a = base + (own[p] ? la[p] : 0);
    float v2 = 0.0f, a2 = 0.0f;
#pragma unroll
    for (int k = 0; k < D2; ++k) {
      H[p][k] = own[p] ? D.s_H[k * NS + a] : 0.0;
      dF[p][k] = own[p] ? D.s_dF[k * NS + a] : 0.0;
      B[p][k] = own[p] ? (float)D.s_B[k * NS + a] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      u[p][k] = own[p] ? D.s_u[k * NS + a] : 0.0;
      du[p][k] = 0.0f;
      dv[p][k] = 0.0f;
      fF[p][k] = own[p] ? D.s_fF[k * NS + a] : 0.0f;
      float vv = own[p] ? (float)D.s_v[k * NS + a] : 0.0f, q = own[p] ? D.s_a[k * NS + a] : 0.0f;
      acc_last[p][k] = q;
      v2 += vv * vv;
      a2 += q * q;
    }
    vm = fmaxf(vm, sqrtf(v2));
    am = fmaxf(am, sqrtf(a2));
  }
  // (Issued before the first barrier so that these loads overlap the state
  // loads above.)  Reference-table rows of the own particles.  Every row is padded past
  // its count with null entries (zero gradient, the particle itself), so the
  // lanes of a wave walk their rows in lockstep up to the wave's longest row
  // without masking; a lane without a particle in slot p walks the first
  // particle's row and discards the sums.  Entries arrive by buffer loads
  // whose vector offset is the lane's particle and whose scalar offset is
  // the row, so addressing costs no vector instructions.
  const __amdgpu_buffer_rsrc_t tab =
      __builtin_amdgcn_make_buffer_rsrc((void *)D.s_nbr, 0, D.nbr_bytes, kBufferWord3);
  const int row_bytes = NS * (int)sizeof(float4);
  unsigned voff[PPT];
  int cnt_max = 0;
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    int lo = own[p] ? la[p] : 0;
    voff[p] = (unsigned)(base + lo) * (unsigned)sizeof(float4);
    if (own[p]) cnt_max = max(cnt_max, D.s_cnt[base + lo]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt_max = max(cnt_max, __shfl_xor(cnt_max, o));
  const int wrows = __builtin_amdgcn_readfirstlane(cnt_max);
  // in 2D z holds the index within the scene: one 12-byte load per entry
  auto entry = [&](int p, int q) -> i4v {
    if constexpr (DIM == 2) {
      i3v e = (i3v)__builtin_amdgcn_raw_buffer_load_b96(tab, voff[p], q * row_bytes, 0);
      return i4v{e[0], e[1], 0, e[2]};
    } else {
      return (i4v)__builtin_amdgcn_raw_buffer_load_b128(tab, voff[p], q * row_bytes, 0);
    }
  };
  // sum_b g_ab of each own particle (stored with the table):
  // sum_b (P_a B_a + P_b B_b) g_ab = P_a B_a sum_b g_ab + sum_b P_b B_b g_ab and
  // sum_b (v_b - v_a) (x) g_ab = sum_b v_b (x) g_ab - v_a (x) sum_b g_ab
  double gs[PPT][DIM];
#pragma unroll
  for (int p = 0; p < PPT; ++p)
#pragma unroll
    for (int k = 0; k < DIM; ++k) gs[p][k] = own[p] ? D.s_gsum[k * NS + base + la[p]] : 0.0;
  // block maxima of |v| and |a|: wave shuffles, then one value per wave
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    vm = fmaxf(vm, __shfl_xor(vm, o));
    am = fmaxf(am, __shfl_xor(am, o));
  }
  if ((t & 63) == 0) {
    red[0][t >> 6] = vm;
    red[1][t >> 6] = am;
  }
  for (int l = t; l < n; l += T) {
    int a = base + l;
#pragma unroll
    for (int k = 0; k < DIM; ++k) Vx[VI(l, k)] = D.s_v[k * NS + a];
    if (l >= nfree)
#pragma unroll
      for (int k = 0; k < D2; ++k) PBx[PI(l, k)] = 0.0;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < (T + 63) / 64; ++w) {
      red[0][0] = fmaxf(red[0][0], red[0][w]);
      red[1][0] = fmaxf(red[1][0], red[1][w]);
    }
    float vmax = red[0][0], amax = red[1][0];
    if (nparts > 1) {
      // the scene's maxima over its workgroups (every one derives the same kappa)
      atomic_max_pos(&D.parts_sync[4 * s], vmax);
      atomic_max_pos(&D.parts_sync[4 * s + 1], amax);
      parts_barrier(D, s, nparts, 1);
      vmax = __uint_as_float(__hip_atomic_load(&D.parts_sync[4 * s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      amax = __uint_as_float(__hip_atomic_load(&D.parts_sync[4 * s + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    int kap;
    double dts;
    solid_kappa(P, S, vmax, amax, dt_ac, kap, dts);
    kap_sh = kap;
    del_sh = dt_ac / kap;
    if (part == 0) {
      S.dt_s = dts;
      S.kappa = kap;
    }
  }
  if (nparts > 1) round = 1;
  __syncthreads();
  const int kap = kap_sh;
  const double del = del_sh;
  const double hd = 0.5 * del;
  const double m_inv = 1.0 / ((double)P.rho0s * (double)P.Vs);
  bool bad_J = false;
  auto first_half = [&](int p) {
    double PB[D2], Bd[D2];
#pragma unroll
    for (int k = 0; k < D2; ++k) {
      H[p][k] += hd * dF[p][k];
      Bd[k] = B[p][k];
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      double inc = hd * Vx[VI(la[p], k)];
      u[p][k] += inc;
      du[p][k] += (float)inc;
    }
    double J;
    solid_PB<DIM, double>(P.material, H[p], Bd, (double)P.mu, (double)P.lam, PB, J);
    bad_J |= !(J > 0.0);
#pragma unroll
    for (int k = 0; k < D2; ++k) PBx[PI(la[p], k)] = PB[k];
  };
#pragma unroll
  for (int p = 0; p < PPT; ++p)
    if (own[p]) first_half(p);
  __syncthreads();
  if (nparts > 1) parts_exchange(D, s, nparts, round, PBx, PR, D2, D.s_xpb, base, l0, l1, lo, hi);
  for (int sub = 0; sub < kap; ++sub) {
    // momentum, velocity
    {
      double acc[PPT][DIM];
#pragma unroll
      for (int p = 0; p < PPT; ++p)
#pragma unroll
        for (int k = 0; k < DIM; ++k) acc[p][k] = 0.0;
      for (int q0 = 0; q0 < wrows; q0 += kSolidBatch) {
        i4v g[kSolidBatch][PPT];
#pragma unroll
        for (int r = 0; r < kSolidBatch; ++r)
#pragma unroll
          for (int p = 0; p < PPT; ++p) g[r][p] = entry(p, q0 + r);
#pragma unroll
        for (int r = 0; r < kSolidBatch; ++r)
#pragma unroll
          for (int p = 0; p < PPT; ++p) {
            const int b = DIM == 2 ? g[r][p][3] : g[r][p][3] - base;
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
              for (int j = 0; j < DIM; ++j) acc[p][i] += PBx[PI(b, i * DIM + j)] * (double)__int_as_float(g[r][p][j]);
          }
      }
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        if (!own[p]) continue;
        int l = la[p];
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          double own_term = 0.0;
#pragma unroll
          for (int j = 0; j < DIM; ++j) own_term += PBx[PI(l, k * DIM + j)] * gs[p][j];
          double ak = ((double)P.Vs * (acc[p][k] + own_term) + (double)fF[p][k]) * m_inv + (double)P.g[k];
          acc_last[p][k] = (float)ak;
          double d_v = del * ak;
          Vx[VI(l, k)] += d_v;
          dv[p][k] += (float)d_v;
        }
      }
    }
    __syncthreads();
    if (nparts > 1) parts_exchange(D, s, nparts, round, Vx, DIM, DIM, D.s_xv, base, l0, l1, lo, hi);
    // deformation rate with the new velocity, second half; then the next
    // sub-step's first half and stress
    const bool more = sub + 1 < kap;
    {
      double G[PPT][D2];
#pragma unroll
      for (int p = 0; p < PPT; ++p)
#pragma unroll
        for (int k = 0; k < D2; ++k) G[p][k] = 0.0;
      for (int q0 = 0; q0 < wrows; q0 += kSolidBatch) {
        i4v g[kSolidBatch][PPT];
#pragma unroll
        for (int r = 0; r < kSolidBatch; ++r)
#pragma unroll
          for (int p = 0; p < PPT; ++p) g[r][p] = entry(p, q0 + r);
#pragma unroll
        for (int r = 0; r < kSolidBatch; ++r)
#pragma unroll
          for (int p = 0; p < PPT; ++p) {
            const int b = DIM == 2 ? g[r][p][3] : g[r][p][3] - base;
#pragma unroll
            for (int i = 0; i < DIM; ++i) {
              double vb = Vx[VI(b, i)];
#pragma unroll
              for (int j = 0; j < DIM; ++j) G[p][i * DIM + j] += vb * (double)__int_as_float(g[r][p][j]);
            }
          }
      }
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        if (!own[p]) continue;
        int l = la[p];
        double va[DIM];
#pragma unroll
        for (int k = 0; k < DIM; ++k) va[k] = Vx[VI(l, k)];
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
          for (int j = 0; j < DIM; ++j) G[p][i * DIM + j] -= va[i] * gs[p][j];
        // (v_b - v_a) (x) (B grad W) summed = G B^T
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
          for (int j = 0; j < DIM; ++j) {
            double sum = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) sum += G[p][i * DIM + k] * (double)B[p][j * DIM + k];
            dF[p][i * DIM + j] = sum;
            H[p][i * DIM + j] += hd * sum;
          }
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          double inc = hd * va[k];
          u[p][k] += inc;
          du[p][k] += (float)inc;
        }
        if (more) first_half(p);
      }
    }
    __syncthreads();
    if (nparts > 1 && more) parts_exchange(D, s, nparts, round, PBx, PR, D2, D.s_xpb, base, l0, l1, lo, hi);
  }
  if (bad_J) atomicOr(&S.err, (int)ERR_JACOBIAN);
  // write back, time averages; where this launch ends the step, the
  // hand-over to the boundary particles, the binning of the solid for a
  // rebuild the closing step sets and the single-step maxima
  const double inv_dt = 1.0 / dt_ac;
  const bool step_end = D.solid_step_end != 0, rb = step_end && rebuilds_next(S);
  float end_v = 0.0f, end_a = 0.0f;
  double jdv = 0.0, jv = 0.0, jda = 0.0, ja = 0.0;  // a judge step's sums
#pragma unroll
  for (int p = 0; p < PPT; ++p) {
    if (!own[p]) continue;
    int l = la[p], a = base + l;
    float vbar[3] = {0.0f, 0.0f, 0.0f}, abar[3] = {0.0f, 0.0f, 0.0f};
    bool bad = false;
#pragma unroll
    for (int k = 0; k < D2; ++k) {
      D.s_H[k * NS + a] = H[p][k];
      D.s_dF[k * NS + a] = dF[p][k];
    }
    float sa = 0.0f;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      D.s_u[k * NS + a] = u[p][k];
      D.s_v[k * NS + a] = Vx[VI(l, k)];
      D.s_a[k * NS + a] = acc_last[p][k];
      vbar[k] = (float)((double)du[p][k] * inv_dt);
      abar[k] = (float)((double)dv[p][k] * inv_dt);
      D.s_vbar[k * NS + a] = vbar[k];
      D.s_abar[k * NS + a] = abar[k];
      bad |= !isfinite(vbar[k]) || !isfinite(abar[k]);
    }
    if (bad) atomicOr(&S.err, (int)ERR_NAN_SOLID);
    if (smode == kSurJudge) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        const double ev = (double)D.sur_vbar[k * NS + a] - vbar[k], ea = (double)D.sur_abar[k * NS + a] - abar[k];
        jdv += ev * ev;
        jv += (double)vbar[k] * vbar[k];
        jda += ea * ea;
        ja += (double)abar[k] * abar[k];
      }
    }
    if (step_end) {
      hand_over_values<DIM>(D, P, a, det_F<DIM>(H[p]), vbar, abar);
      if (rb) bin_entry<DIM>(D, D.nf + P.b_begin + P.w_count + l, true, kBinSolid);
      float v2 = 0.0f, a2 = 0.0f;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        const float v = (float)Vx[VI(l, k)];
        v2 += v * v;
        a2 += acc_last[p][k] * acc_last[p][k];
      }
      end_v = fmaxf(end_v, sqrtf(v2));
      end_a = fmaxf(end_a, sqrtf(a2));
    }
  }
  if (step_end && P.single_step) {
    auto fmx = [](float x, float y) { return fmaxf(x, y); };
    end_v = block_reduce(end_v, fmx, red[0]);
    end_a = block_reduce(end_a, fmx, red[1]);
    if (t == 0) {
      S.send_v = __float_as_uint(end_v);
      S.send_a = __float_as_uint(end_a);
    }
  }
  if (smode != kSurOff) {
    if (smode == kSurJudge) {
      auto add = [](double x, double y) { return x + y; };
      jdv = block_reduce(jdv, add, sur_red[0]);
      jv = block_reduce(jv, add, sur_red[1]);
      jda = block_reduce(jda, add, sur_red[2]);
      ja = block_reduce(ja, add, sur_red[3]);
    }
    if (t == 0) sur_schedule(D, P, S, smode, jdv, jv, jda, ja);
  }
  if (nparts > 1 && t == 0) {
    // the last workgroup of the scene clears its words for the next launch
    const unsigned done =
        __hip_atomic_fetch_add(&D.parts_sync[4 * s + 3], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (done + 1 == (unsigned)nparts)
      for (int k = 0; k < 4; ++k) __hip_atomic_store(&D.parts_sync[4 * s + k], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Max |v| and |a| of the free solid at the end of a step, for scenes that
// take one shared step (their next step size needs the solid step).  A wave
// whose lanes share one scene reduces first; lanes of a wave that straddles
// scenes each post their own maximum.
template <int DIM>
__device__ void single_step_maxima(const Dev &D, int a) {
  const int NS = D.ns;
  int s = -1;
  float vm = 0.0f, am = 0.0f;
  if (a < NS) {
    s = D.s_scene[a];
    const ScenePar &P = D.par[s];
    if (!P.single_step || a - P.s_begin >= P.s_count - P.s_nclamp) {
      s = -1;
    } else {
      float v2 = 0.0f, a2 = 0.0f;
      for (int k = 0; k < DIM; ++k) {
        float v = (float)D.s_v[k * NS + a], q = D.s_a[k * NS + a];
        v2 += v * v;
        a2 += q * q;
      }
      vm = sqrtf(v2);
      am = sqrtf(a2);
    }
  }
  const int s0 = __shfl(s, 0);
  if (__all(s == s0)) {
    if (s0 < 0) return;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      vm = fmaxf(vm, __shfl_xor(vm, o));
      am = fmaxf(am, __shfl_xor(am, o));
    }
    if ((threadIdx.x & 63) == 0) {
      atomic_max_pos(&D.st[s0].send_v, vm);
      atomic_max_pos(&D.st[s0].send_a, am);
    }
  } else if (s >= 0) {
    atomic_max_pos(&D.st[s].send_v, vm);
    atomic_max_pos(&D.st[s].send_a, am);
  }
}

// Step end of the fluid, block blk of the fluid range: max speed for the
// next acoustic step and, after a rebuild, the pair counts, kReduceItems
// particles per thread and one reduction and atomic per scene present in the
// block (scenes own contiguous ranges).  Any block size that is a multiple of
// 64 (at most 1024).
__device__ void fluid_step_end(const Dev &D, int blk, float *shm, unsigned long long (*shc)[16]) {
  const int span = blockDim.x * kReduceItems;
  const int i0 = blk * span, i1 = min(D.nf, i0 + span);
  const int s0 = D.f_scene[i0], s1 = D.f_scene[i1 - 1];
  auto fmx = [](float x, float y) { return fmaxf(x, y); };
  auto add = [](unsigned long long x, unsigned long long y) { return x + y; };
  for (int s = s0; s <= s1; ++s) {
    SceneState &S = D.st[s];
    const bool rebuilt = S.need_rebuild != 0;
    float m = 0.0f;  // fmaxf drops a NaN speed; the continuity pass flags it
    unsigned long long c[3] = {0ull, 0ull, 0ull};
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
      if (D.f_scene[i] != s) continue;
      m = fmaxf(m, D.f_speed[i]);
      if (rebuilt) {
        int4 n = D.f_nnb[i];
        c[0] += (unsigned long long)n.x;
        c[1] += (unsigned long long)n.y;
        c[2] += (unsigned long long)n.z;
      }
    }
    m = block_reduce(m, fmx, shm);
    if (threadIdx.x == 0) atomic_max_pos(&S.vmax_next, m);
    if (rebuilt) {
      for (int k = 0; k < 3; ++k) c[k] = block_reduce(c[k], add, shc[k]);
      if (threadIdx.x == 0) {
        atomicAdd(&S.acc_ff, c[0]);
        atomicAdd(&S.acc_fw, c[1]);
        atomicAdd(&S.acc_fs, c[2]);
      }
    }
  }
}

// End of an acoustic step over all particles, before k_step_close.  Fluid
// blocks: max fluid speed for the next acoustic step and, after a rebuild,
// the pair counts, folded into the scene's accumulators with one atomic per
// block (per thread where a block spans two scenes).  Solid blocks: the
// solid's averaged velocity and acceleration and its current volume are
// handed to the boundary particles seen by the fluid, with the hydrostatic
// factor max(0, (abar - g).n).  Kept apart from the sub-step kernels so that
// the continuity pass, which reads the boundary particles, can run
// concurrently with the coupling and solid passes.
template <int DIM>
__global__ void __launch_bounds__(256) k_step_reduce(Dev D, int bin_blocks, int fluid_blocks) {
  __shared__ float shm[16];
  __shared__ unsigned long long shc[3][16];
  if ((int)blockIdx.x < bin_blocks) {
    // the particles of scenes whose advection step ends with this step are
    // binned for the rebuild that opens the next one (most steps end none:
    // then the blocks leave after reading the scenes' clocks)
    bool any = D.n_scenes > kBinSceneCheck;
    for (int s = 0; s < D.n_scenes && !any; ++s) any = rebuilds_next(D.st[s]);
    if (!any) return;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < D.nf + D.nb; t += bin_blocks * blockDim.x)
      bin_entry<DIM>(D, t, true);
    return;
  }
  const int blk = blockIdx.x - bin_blocks;
  if (blk < fluid_blocks) {
    fluid_step_end(D, blk, shm, shc);
    return;
  }
  const int a = (blk - fluid_blocks) * blockDim.x + threadIdx.x;
  hand_over<DIM>(D, a);
  if (D.any_single) single_step_maxima<DIM>(D, a);
}


// ------------------------------------------------------------------ surrogate
//
// Learned replacement of the kappa solid sub-steps of one acoustic step (2D).
// Per free solid particle the network reads 24 features and predicts the
// change of the time-averaged velocity and acceleration over the step
// (Section 3.2 defines the averages).  With the own values F - I, v, a and
// the pressure and viscous parts fp, fv of the coupling force, their means
// over the reference neighbours (the own values where there are none), the
// row's acceleration scale s = |a| + |mean a| + |g| + |fp + fv| / m + s0
// (m = rho0_S V_S, s0 = 1e-3 m/s^2) and the acoustic step dt, the features
// are F - I, v, a / s, fp / (m s), fv / (m s) and the neighbour mean minus the
// own value of each of the 12 (F's as is, v's over s dt, a's over s, the
// forces' over m s); the network's standardised output y gives, with
// d = y std + mean, vbar = v + s dt d_v and abar = a + s d_a.  The scale puts
// quiet and violent states on one footing; the differences carry what the
// neighbour means add, at the resolution of their own size.
//
// The plain sub-steps judge the network (the schedule and the learned update
// run inside the solid launch, one block per scene; see k_solid_reg).

// Own values of solid particle a: F - I and v (FP64 state), a, fp, fv.
struct SurOwn {
  double h[4], v[2];
  float a[2], fp[2], fv[2];
};
__device__ __forceinline__ SurOwn sur_own(const Dev &D, int a) {
  const int NS = D.ns;
  SurOwn o;
#pragma unroll
  for (int k = 0; k < 4; ++k) o.h[k] = D.s_H[k * NS + a];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    o.v[k] = D.s_v[k * NS + a];
    o.a[k] = D.s_a[k * NS + a];
    const float fp = D.s_fFp[k * NS + a];
    o.fp[k] = fp;
    o.fv[k] = D.s_fF[k * NS + a] - fp;
  }
  return o;
}

// Sums over reference neighbours of (neighbour value - own value).
struct SurDiff {
  double h[4], v[2], a[2], fp[2], fv[2];
};
__device__ __forceinline__ void sur_zero(SurDiff &d) {
#pragma unroll
  for (int k = 0; k < 4; ++k) d.h[k] = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) d.v[k] = d.a[k] = d.fp[k] = d.fv[k] = 0.0;
}
// neighbours q0, q0 + dq, ... of particle a
__device__ __forceinline__ void sur_diffs(const Dev &D, int a, const SurOwn &o, int q0, int dq, SurDiff &d) {
  const int cnt = D.s_cnt[a];
  for (int q = q0; q < cnt; q += dq) {
    const SurOwn b = sur_own(D, __float_as_int(D.s_nbr[(size_t)q * D.ns + a].w));
#pragma unroll
    for (int k = 0; k < 4; ++k) d.h[k] += b.h[k] - o.h[k];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      d.v[k] += b.v[k] - o.v[k];
      d.a[k] += (double)b.a[k] - (double)o.a[k];
      d.fp[k] += (double)b.fp[k] - (double)o.fp[k];
      d.fv[k] += (double)b.fv[k] - (double)o.fv[k];
    }
  }
}
// sum of the partial sums of the 4 consecutive lanes that share a particle
__device__ __forceinline__ void sur_diffs_lanes4(SurDiff &d) {
#pragma unroll
  for (int m = 1; m < 4; m <<= 1) {
#pragma unroll
    for (int k = 0; k < 4; ++k) d.h[k] += __shfl_xor(d.h[k], m);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      d.v[k] += __shfl_xor(d.v[k], m);
      d.a[k] += __shfl_xor(d.a[k], m);
      d.fp[k] += __shfl_xor(d.fp[k], m);
      d.fv[k] += __shfl_xor(d.fv[k], m);
    }
  }
}

constexpr double kSurScaleFloor = 1e-3;  // s0, m/s^2

// The 24 raw features and the scale s of a free particle with cnt neighbours.
__device__ __forceinline__ void sur_finish(const ScenePar &P, double dt, const SurOwn &o, SurDiff d, int cnt,
                                           float *f, double &s) {
  const double inv = cnt > 0 ? 1.0 / (double)cnt : 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) d.h[k] *= inv;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    d.v[k] *= inv;
    d.a[k] *= inv;
    d.fp[k] *= inv;
    d.fv[k] *= inv;
  }
  const double m = (double)P.rho0s * (double)P.Vs;
  const double a0 = o.a[0], a1 = o.a[1];
  const double f0 = (double)o.fp[0] + o.fv[0], f1 = (double)o.fp[1] + o.fv[1];
  s = sqrt(a0 * a0 + a1 * a1) + sqrt((a0 + d.a[0]) * (a0 + d.a[0]) + (a1 + d.a[1]) * (a1 + d.a[1])) +
      sqrt((double)P.g[0] * P.g[0] + (double)P.g[1] * P.g[1]) + sqrt(f0 * f0 + f1 * f1) / m + kSurScaleFloor;
  const double is = 1.0 / s, ims = 1.0 / (m * s), isd = 1.0 / (s * dt);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    f[k] = (float)o.h[k];
    f[12 + k] = (float)d.h[k];
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    f[4 + k] = (float)o.v[k];
    f[6 + k] = (float)(o.a[k] * is);
    f[8 + k] = (float)(o.fp[k] * ims);
    f[10 + k] = (float)(o.fv[k] * ims);
    f[16 + k] = (float)(d.v[k] * isd);
    f[18 + k] = (float)(d.a[k] * is);
    f[20 + k] = (float)(d.fp[k] * ims);
    f[22 + k] = (float)(d.fv[k] * ims);
  }
}

// Training features of every solid particle, in solid order (clamp rows
// zero), standardised by (mean, 1/std) when stats is given; the scale, step,
// v and a of each row are kept for the targets of the same step.
__global__ void __launch_bounds__(256) k_sur_features(Dev D, const float *stats, float *x) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= D.ns) return;
  const int sc = D.s_scene[a];
  const ScenePar &P = D.par[sc];
  float *row = x + (size_t)a * kSurFeat;
  float *aux = D.sur_aux + (size_t)a * 6;
  if (a - P.s_begin >= P.s_count - P.s_nclamp) {
    for (int k = 0; k < kSurFeat; ++k) row[k] = 0.0f;
    for (int k = 0; k < 6; ++k) aux[k] = 0.0f;
    return;
  }
  const double dt = D.st[sc].dt_ac;
  const SurOwn o = sur_own(D, a);
  SurDiff d;
  sur_zero(d);
  sur_diffs(D, a, o, 0, 1, d);
  float f[kSurFeat];
  double s;
  sur_finish(P, dt, o, d, D.s_cnt[a], f, s);
  for (int k = 0; k < kSurFeat; ++k) row[k] = stats ? (f[k] - stats[k]) * stats[kSurFeat + k] : f[k];
  aux[0] = (float)s;
  aux[1] = (float)dt;
  aux[2] = (float)o.v[0];
  aux[3] = (float)o.v[1];
  aux[4] = o.a[0];
  aux[5] = o.a[1];
}

// Training targets after a plain step, from the references its features
// kept: ((vbar - v) / (s dt), (abar - a) / s) per free particle, zero rows
// for the clamp.
__global__ void __launch_bounds__(256) k_sur_targets(Dev D, float *t) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= D.ns) return;
  const ScenePar &P = D.par[D.s_scene[a]];
  const int NS = D.ns;
  float *row = t + (size_t)a * kSurOut;
  const float *aux = D.sur_aux + (size_t)a * 6;
  if (a - P.s_begin >= P.s_count - P.s_nclamp) {
    for (int k = 0; k < kSurOut; ++k) row[k] = 0.0f;
    return;
  }
  const double s = aux[0], dt = aux[1];
  for (int k = 0; k < 2; ++k) {
    row[k] = (float)(((double)D.s_vbar[k * NS + a] - (double)aux[2 + k]) / (s * dt));
    row[2 + k] = (float)(((double)D.s_abar[k * NS + a] - (double)aux[4 + k]) / s);
  }
}

// The surrogate pass of a step, one block per 64 solid rows: each row's
// scene mode (the first row of a scene records it for the solid launch and
// the step's close); for tiles with rows of learned or judge scenes, the
// features (four lanes per row share its neighbours), the network on the
// matrix cores with its weights staged in LDS, and the predicted averages.
__global__ void __launch_bounds__(256) k_sur_net(Dev D, MlpDev M) {
  extern __shared__ __align__(16) unsigned short lds[];
  __shared__ float r_s[kMlpTile], r_dt[kMlpTile], r_v[kMlpTile][2], r_a[kMlpTile][2];
  __shared__ int r_need[kMlpTile];
  const int t = threadIdx.x, l = t & 63;
  const int row0 = blockIdx.x * kMlpTile;
  int need = 0;
  if (t < kMlpTile) {
    const int a = row0 + t;
    if (a < D.ns) {
      const int sc = D.s_scene[a];
      const ScenePar &P = D.par[sc];
      SceneState &S = D.st[sc];
      const int mode = sur_mode(S);
      const int local = a - P.s_begin;
      if (local == 0) {
        S.sur = mode;
        if (mode == kSurLearned) S.kappa = 0;  // no sub-steps this step
      }
      // 1: a free row, 2: a clamp row (zero averages), of a scene that needs the network
      need = mode == kSurPlain ? 0 : (local < P.s_count - P.s_nclamp ? 1 : 2);
    }
    r_need[t] = need;
  }
  if (!__syncthreads_or(need != 0)) return;
  const FwdLds L = fwd_lds_layout(lds);
  stage_weights(M, L);
  const float *mean = D.sur_stats, *istd = D.sur_stats + kSurFeat;
  {
    const int r = t >> 2, q = t & 3, a = row0 + r;
    const int nd = r_need[r];
    SurOwn o;
    SurDiff d;
    sur_zero(d);
    if (nd == 1) {
      o = sur_own(D, a);
      sur_diffs(D, a, o, q, 4, d);
    }
    sur_diffs_lanes4(d);
    unsigned short *hrow = L.HA + r * pitch(kMlpIn);
    if (q == 0) {
      if (nd == 1) {
        const int sc = D.s_scene[a];
        const double dt = D.st[sc].dt_ac;
        float f[kSurFeat];
        double s;
        sur_finish(D.par[sc], dt, o, d, D.s_cnt[a], f, s);
        for (int k = 0; k < kSurFeat; ++k) hrow[k] = f2bf((f[k] - mean[k]) * istd[k]);
        r_s[r] = (float)s;
        r_dt[r] = (float)dt;
        r_v[r][0] = (float)o.v[0];
        r_v[r][1] = (float)o.v[1];
        r_a[r][0] = o.a[0];
        r_a[r][1] = o.a[1];
      } else {
        for (int k = 0; k < kSurFeat; ++k) hrow[k] = 0;
      }
      for (int k = kSurFeat; k < kMlpIn; ++k) hrow[k] = 0;
    }
  }
  __syncthreads();
  const f4 out = forward_tile<false>(L, M, row0, D.ns);
  const float *mo = D.sur_stats + 2 * kSurFeat, *so = mo + kSurOut;
  const int NS = D.ns, r0 = (t >> 6) * 16, c = l & 15;
  if (c < kSurOut) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + (l >> 4) * 4 + j, a = row0 + r;
      const int nd = r_need[r];
      if (nd == 0) continue;
      float val = 0.0f;
      if (nd == 1) {
        const float dd = (out[j] + L.bias[3 * kMlpHid + c]) * so[c] + mo[c];
        val = c < 2 ? r_v[r][c] + r_s[r] * r_dt[r] * dd : r_a[r][c - 2] + r_s[r] * dd;
      }
      if (c < 2) D.sur_vbar[c * NS + a] = val;
      else D.sur_abar[(c - 2) * NS + a] = val;
    }
  }
}

// ------------------------------------------------------------------ state I/O

template <int DIM>
__global__ void k_read_fluid(Dev D, int s, int field, double *out) {
  const ScenePar &P = D.par[s];
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= P.f_count) return;
  int i = P.f_begin + l;
  int id = D.f_id[i];
  switch (field) {
  case 0: {
    double4 o = D.f_off[i];
    for (int k = 0; k < DIM; ++k) out[(size_t)DIM * id + k] = absolute<DIM>(P, D.f_lin[i], get4(o, k), k);
  } break;
  case 1: {
    float4 v = D.f_va[i];
    for (int k = 0; k < DIM; ++k) out[(size_t)DIM * id + k] = get4(v, k);
  } break;
  case 2: out[id] = (double)P.rho0 * (1.0 + (double)D.f_va[i].w); break;
  case 3: out[id] = (double)P.rho0 * (double)D.f_drho[i]; break;
  case 4: {
    float4 v = D.f_acc[i];
    for (int k = 0; k < DIM; ++k) out[(size_t)DIM * id + k] = get4(v, k);
  } break;
  case 5: out[id] = D.f_p[i]; break;
  case 6: {
    int4 c = D.f_nnb[i];
    out[2 * (size_t)id] = c.x;
    out[2 * (size_t)id + 1] = c.y + c.z;
  } break;
  }
}

template <int DIM>
__global__ void k_write_fluid(Dev D, int s, int field, const double *in) {
  const ScenePar &P = D.par[s];
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= P.f_count) return;
  int i = P.f_begin + l;
  int id = D.f_id[i];
  switch (field) {
  case 0: {
    // offset from the particle's current cell; the next rebuild renormalises
    int c[3];
    decode_cell(P, D.f_lin[i], c);
    double o[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < DIM; ++k) {
      double x = in[(size_t)DIM * id + k] - P.lo[k];
      double rel = x - c[k] * P.csd[k];
      if (P.periodic[k]) rel -= P.len[k] * floor(rel / P.len[k] + 0.5);
      o[k] = rel;
    }
    D.f_off[i] = make_double4(o[0], o[1], o[2], 0.0);
  } break;
  case 1: {
    float4 v = D.f_va[i];
    v.x = (float)in[(size_t)DIM * id];
    v.y = (float)in[(size_t)DIM * id + 1];
    if (DIM == 3) v.z = (float)in[(size_t)DIM * id + 2];
    D.f_va[i] = v;
    D.f_speed[i] = sqrtf(v.x * v.x + v.y * v.y + v.z * v.z);
  } break;
  case 2: {
    float4 v = D.f_va[i];
    v.w = (float)(in[id] / (double)P.rho0 - 1.0);
    D.f_va[i] = v;
  } break;
  case 3: D.f_drho[i] = (float)(in[id] / (double)P.rho0); break;
  }
}

template <int DIM>
__global__ void k_read_solid(Dev D, int s, int field, double *out) {
  const ScenePar &P = D.par[s];
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= P.s_count) return;
  int a = P.s_begin + l, NS = D.ns;
  const float *src = nullptr;
  int w = DIM;
  switch (field) {
  case 10:
  case 11: {
    const double *sd = field == 10 ? D.s_u : D.s_v;
    for (int k = 0; k < DIM; ++k) out[(size_t)DIM * l + k] = sd[k * NS + a];
    return;
  }
  case 12: src = D.s_a; break;
  case 14:
  case 19: {
    const double *sd = field == 14 ? D.s_dF : D.s_B;
    for (int k = 0; k < DIM * DIM; ++k) out[(size_t)DIM * DIM * l + k] = sd[k * NS + a];
    return;
  }
  case 15: src = D.s_fF; break;
  case 16: src = D.s_vbar; break;
  case 17: src = D.s_abar; break;
  case 18: src = D.s_n; break;
  case 20: src = D.s_n0; break;
  case 13:
    for (int k = 0; k < DIM * DIM; ++k)
      out[(size_t)DIM * DIM * l + k] = D.s_H[k * NS + a] + ((k % (DIM + 1) == 0) ? 1.0 : 0.0);
    return;
  case 21:
    for (int k = 0; k < DIM; ++k) out[(size_t)DIM * l + k] = D.s_r0d[3 * (size_t)a + k];
    return;
  default: return;
  }
  for (int k = 0; k < w; ++k) out[(size_t)w * l + k] = src[k * NS + a];
}

template <int DIM>
__global__ void k_write_solid(Dev D, int s, int field, const double *in) {
  const ScenePar &P = D.par[s];
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= P.s_count) return;
  int a = P.s_begin + l, NS = D.ns;
  float *dst = nullptr;
  int w = DIM;
  switch (field) {
  case 10:
  case 11: {
    double *dd = field == 10 ? D.s_u : D.s_v;
    for (int k = 0; k < DIM; ++k) dd[k * NS + a] = in[(size_t)DIM * l + k];
    return;
  }
  case 12: dst = D.s_a; break;
  case 14:
    for (int k = 0; k < DIM * DIM; ++k) D.s_dF[k * NS + a] = in[(size_t)DIM * DIM * l + k];
    return;
  case 16: dst = D.s_vbar; break;
  case 17: dst = D.s_abar; break;
  case 13:
    for (int k = 0; k < DIM * DIM; ++k)
      D.s_H[k * NS + a] = in[(size_t)DIM * DIM * l + k] - ((k % (DIM + 1) == 0) ? 1.0 : 0.0);
    return;
  default: return;
  }
  for (int k = 0; k < w; ++k) dst[k * NS + a] = (float)in[(size_t)w * l + k];
}

// ------------------------------------------------------------------ FP64 reductions

// Per-block FP64 partial sums for one scene (deterministic two-pass):
// [0..2] fluid m v, [3..5] solid m v, [6] fluid KE, [7] solid KE,
// [8] strain energy sum V0 W(F), [9..11] sum f^F, [12..14] solid-on-fluid
// coupling force re-evaluated from the mid-point state.
constexpr int NRED = 16;

template <int DIM>
__global__ void __launch_bounds__(256) k_reduce_partial(Dev D, int s, double *part) {
  __shared__ double sh[NRED][256];
  const ScenePar &P = D.par[s];
  double acc[NRED];
  for (int k = 0; k < NRED; ++k) acc[k] = 0.0;
  int NS = D.ns;
  int stride = gridDim.x * blockDim.x;
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < P.f_count; l += stride) {
    int i = P.f_begin + l;
    float4 v = D.f_va[i];
    double m = D.f_pos[i].w;
    double vv[3] = {v.x, v.y, v.z};
    for (int k = 0; k < DIM; ++k) {
      acc[k] += m * vv[k];
      acc[6] += 0.5 * m * vv[k] * vv[k];
    }
    // coupling force of the free solid on this fluid particle, mid-point state
    float4 pi = D.f_pos[i];
    float4 vb = D.f_vs[i];
    float vi[3] = {vb.x, vb.y, vb.z};
    float p_i = D.f_p[i];
    int cb = P.cell_begin;
    visit_cells<DIM>(P, D.f_lin[i], [&](int nl, const float *sh2, int) {
      int2 be = D.bc_se[cb + nl];
      for (int k = be.x; k < be.y; ++k) {
        float4 bn = D.b_nrm[k];
        if (bn.w > 0.0f) continue;  // walls
        float4 pb = D.b_pos[k];
        float r[3] = {(pi.x - pb.x) - sh2[0], (pi.y - pb.y) - sh2[1], DIM == 3 ? (pi.z - pb.z) - sh2[2] : 0.0f};
        float r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (r2 >= P.r2max_f) continue;
        float f[3];
        coupling_force<DIM>(P, pi.w, vb.w, p_i, vi, r, pb, D.b_vbar[k], bn, f);
        for (int q = 0; q < DIM; ++q) acc[12 + q] += f[q];
      }
    });
  }
  for (int l = blockIdx.x * blockDim.x + threadIdx.x; l < P.s_count; l += stride) {
    int a = P.s_begin + l;
    double m = (double)P.rho0s * (double)P.Vs;
    double H[9];
    for (int k = 0; k < DIM * DIM; ++k) H[k] = D.s_H[k * NS + a];
    for (int k = 0; k < DIM; ++k) {
      double v = D.s_v[k * NS + a];
      acc[3 + k] += m * v;
      acc[7] += 0.5 * m * v * v;
      acc[9 + k] += D.s_fF[k * NS + a];
    }
    // strain energy in FP64: Neo-Hookean mu trE - mu lnJ + lambda/2 (lnJ)^2,
    // linear elastic lambda/2 (trE)^2 + mu E:E
    double trE = 0.0, EE = 0.0;
    for (int i = 0; i < DIM; ++i)
      for (int j = 0; j < DIM; ++j) {
        double e = H[i * DIM + j] + H[j * DIM + i];
        for (int k = 0; k < DIM; ++k) e += H[k * DIM + i] * H[k * DIM + j];
        e *= 0.5;
        EE += e * e;
        if (i == j) trE += e;
      }
    if (P.material == 1) {
      acc[8] += (double)P.Vs * (0.5 * (double)P.lam * trE * trE + (double)P.mu * EE);
      continue;
    }
    double J;
    if (DIM == 2) J = (1.0 + H[0]) * (1.0 + H[3]) - H[1] * H[2];
    else {
      double F[9];
      for (int k = 0; k < 9; ++k) F[k] = H[k] + ((k % 4 == 0) ? 1.0 : 0.0);
      J = F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
          F[2] * (F[3] * F[7] - F[4] * F[6]);
    }
    double lj = log(J);
    acc[8] += (double)P.Vs * ((double)P.mu * trE - (double)P.mu * lj + 0.5 * (double)P.lam * lj * lj);
  }
  for (int k = 0; k < NRED; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < NRED; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < NRED; ++k) part[(size_t)blockIdx.x * NRED + k] = sh[k][0];
}

__global__ void k_reduce_final(int nblocks, const double *part, double *out) {
  if (threadIdx.x >= NRED) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * NRED + threadIdx.x];
  out[threadIdx.x] = s;
}

// Block partials of the reductions for callers that cannot allocate
// (sph_reduce_noalloc): one file-scope device array, of which each GPU the
// library runs on holds its own copy until the process ends.  Host code
// never passes the array's name to a kernel (on the host it is a stand-in,
// not a device address): reduce_scratch() takes the device address once per
// device with hipGetSymbolAddress, and the launchers take that pointer.
static __device__ __align__(256) double scratch[kReduceScratchBlocks * NRED];

// Drops the binning done at the end of the last step for scene s (the state
// has changed since, or the rebuild is withdrawn): its cell counts return to
// zero and the scene is binned again when its rebuild starts.
__device__ void unbin_scene(const Dev &D, int s) {
  SceneState &S = D.st[s];
  const int binned = S.binned;  // uniform: read before any thread writes it
  __syncthreads();
  if (binned) {
    const ScenePar &P = D.par[s];
    for (int c = threadIdx.x; c < P.ncell_total; c += blockDim.x) {
      D.fc_count[P.cell_begin + c] = 0;
      D.bc_count[P.cell_begin + c] = 0;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) S.binned = 0;
}

__global__ void __launch_bounds__(256) k_set_rebuild(Dev D, int s) {
  unbin_scene(D, s);
  if (threadIdx.x == 0 && !D.st[s].need_rebuild) {
    D.st[s].need_rebuild = 1;
    atomicAdd(D.rebuild_count, 1);
  }
}

__global__ void __launch_bounds__(256) k_unbin(Dev D, int s) { unbin_scene(D, s); }

// ------------------------------------------------------------------ host-side launchers

#define LAUNCH_DIM(dim, kern, grid, block, stream, ...)                          \
  do {                                                                          \
    if ((dim) == 2) hipLaunchKernelGGL(kern<2>, grid, block, 0, stream, __VA_ARGS__); \
    else hipLaunchKernelGGL(kern<3>, grid, block, 0, stream, __VA_ARGS__);            \
  } while (0)

static inline int nblk(int n, int b) { return n > 0 ? (n + b - 1) / b : 1; }

void launch_init_scene(const Dev &D, int s, const double *x_f, const double *v_f, int has_vf, double gabs,
                       double hydroH, double dpd, int nf, hipStream_t st) {
  LAUNCH_DIM(D.dim, k_init_fluid, dim3(nblk(nf, 256)), dim3(256), st, D, s, x_f, v_f, has_vf, gabs, hydroH, dpd);
}

void launch_init_walls(const Dev &D, int s, const double *x, const double *n, int nw, hipStream_t st) {
  LAUNCH_DIM(D.dim, k_init_walls, dim3(nblk(nw, 256)), dim3(256), st, D, s, x, n);
}

void launch_init_solid(const Dev &D, int s, const double *x, const double *v, int has_v, int ns,
                       hipStream_t st) {
  LAUNCH_DIM(D.dim, k_init_solid, dim3(nblk(ns, 256)), dim3(256), st, D, s, x, v, has_v);
}

void launch_solid_reference(const Dev &D, int s, int ns_scene, hipStream_t st) {
  LAUNCH_DIM(D.dim, k_solid_neighbours, dim3(nblk(ns_scene, 256)), dim3(256), st, D, s);
}

void launch_solid_B(const Dev &D, hipStream_t st) {
  if (D.ns == 0) return;
  LAUNCH_DIM(D.dim, k_solid_B, dim3(nblk(D.ns, 256)), dim3(256), st, D);
}

void launch_parts_range(const Dev &D, hipStream_t st) {
  if (D.n_parts_blocks > 0) hipLaunchKernelGGL(k_parts_range, dim3(D.n_parts_blocks), dim3(256), 0, st, D);
}

void launch_solid_classes(const Dev &D, int s, hipStream_t st) {
  hipLaunchKernelGGL(k_solid_classes, dim3(1), dim3(kNbrClasses), 0, st, D, s);
}

void launch_solid_compact(const Dev &D, int s, int ns_scene, hipStream_t st) {
  if (ns_scene > 0) hipLaunchKernelGGL(k_solid_compact, dim3(nblk(ns_scene, 256)), dim3(256), 0, st, D, s);
}

void launch_solid_gsum_classes(const Dev &D, hipStream_t st) {
  if (D.ns > 0) hipLaunchKernelGGL(k_solid_gsum_classes, dim3(nblk(D.ns, 256)), dim3(256), 0, st, D);
}

void launch_refresh_vmax(const Dev &D, hipStream_t st) {
  hipLaunchKernelGGL(k_refresh_vmax, dim3(D.n_scenes), dim3(256), 0, st, D);
}

#define LAUNCH_LPP(kern, lpp, dim, grid, block, shm, stream, ...)                                    \
  do {                                                                                         \
    switch (lpp) {                                                                             \
    case 1: if ((dim) == 2) hipLaunchKernelGGL((kern<2, 1>), grid, block, shm, stream, __VA_ARGS__);  \
            else hipLaunchKernelGGL((kern<3, 1>), grid, block, shm, stream, __VA_ARGS__); break;       \
    case 2: if ((dim) == 2) hipLaunchKernelGGL((kern<2, 2>), grid, block, shm, stream, __VA_ARGS__);  \
            else hipLaunchKernelGGL((kern<3, 2>), grid, block, shm, stream, __VA_ARGS__); break;       \
    case 4: if ((dim) == 2) hipLaunchKernelGGL((kern<2, 4>), grid, block, shm, stream, __VA_ARGS__);  \
            else hipLaunchKernelGGL((kern<3, 4>), grid, block, shm, stream, __VA_ARGS__); break;       \
    case 8: if ((dim) == 2) hipLaunchKernelGGL((kern<2, 8>), grid, block, shm, stream, __VA_ARGS__);  \
            else hipLaunchKernelGGL((kern<3, 8>), grid, block, shm, stream, __VA_ARGS__); break;       \
    default: if ((dim) == 2) hipLaunchKernelGGL((kern<2, 16>), grid, block, shm, stream, __VA_ARGS__); \
            else hipLaunchKernelGGL((kern<3, 16>), grid, block, shm, stream, __VA_ARGS__); break;      \
    }                                                                                          \
  } while (0)

static inline dim3 grid_for(long long threads, int block) {
  return dim3((unsigned)std::max<long long>(1, (threads + block - 1) / block));
}

// all cells in one tile and at most one close thread per scene in a block:
// the step close also scans the cells of the rebuilds it sets
static inline bool step_end_scan(const Dev &D) { return D.ncell <= kCellTile && D.n_scenes <= 1024; }

void launch_rebuild(const Dev &D, const LaunchCfg &cfg, hipStream_t st, bool with_bin) {
  if (with_bin) launch_bin(D, st);
  const int ntiles = (D.ncell + kCellTile - 1) / kCellTile;
  if (ntiles == 1) {
    if (with_bin || !step_end_scan(D)) hipLaunchKernelGGL(k_cell_one, dim3(1), dim3(1024), 0, st, D);
  } else {
    hipLaunchKernelGGL(k_cell_sum, dim3(ntiles), dim3(1024), 0, st, D);
    hipLaunchKernelGGL(k_cell_prefix, dim3(1), dim3(1024), 0, st, D, ntiles);
    hipLaunchKernelGGL(k_cell_apply, dim3(ntiles), dim3(1024), 0, st, D);
  }
  if (D.nf + D.nb > 0) hipLaunchKernelGGL(k_scatter, grid_for(D.nf + D.nb, 256), dim3(256), 0, st, D);
  if (D.nf + D.nb > 0) LAUNCH_DIM(D.dim, k_rank_move, grid_for(D.nf + D.nb, 256), dim3(256), st, D);
  if (D.nf > 0)
    LAUNCH_LPP(k_reinit, cfg.lpp_reinit, D.dim, grid_for((long long)D.nf * cfg.lpp_reinit, cfg.block_pair),
               dim3(cfg.block_pair), 0, st, D);
  if (D.nf > 0 && D.tile_gp > 0) {
    // one block per group, the rows' lanes per particle (the list width)
    const dim3 grid((D.nf + D.tile_gp - 1) / D.tile_gp), block(D.tile_gp * D.lw);
    switch (D.lw) {
    case 1: hipLaunchKernelGGL(k_tile_union<1>, grid, block, 0, st, D); break;
    case 2: hipLaunchKernelGGL(k_tile_union<2>, grid, block, 0, st, D); break;
    case 4: hipLaunchKernelGGL(k_tile_union<4>, grid, block, 0, st, D); break;
    case 8: hipLaunchKernelGGL(k_tile_union<8>, grid, block, 0, st, D); break;
    default: hipLaunchKernelGGL(k_tile_union<16>, grid, block, 0, st, D); break;
    }
  }
}

// coupling lists ordered by each wave of the force launch's leading blocks
constexpr int kListsPerWave = 2;

void launch_fluid_force(const Dev &D, const LaunchCfg &cfg, hipStream_t st) {
  if (D.nf > 0 && D.fluid_prep) hipLaunchKernelGGL(k_fluid_prep, grid_for(D.nf, 256), dim3(256), 0, st, D);
  if (D.nf > 0) {
    // leading blocks order the coupling lists after a rebuild: kListsPerWave
    // lists per wave, more where that would need over 2048 blocks (each
    // block that only finds no rebuild still costs a dispatch), a multiple
    // of 8 blocks
    Dev Df = D;
    const int waves = cfg.block_pair / 64;
    const int per = std::max(kListsPerWave, (D.ns + waves * 2048 - 1) / (waves * 2048));
    int nsort = D.ns > 0 ? (D.ns + per * waves - 1) / (per * waves) : 0;
    nsort = (nsort + 7) / 8 * 8;
    Df.sort_blocks = nsort;
    dim3 grid = grid_for((long long)D.nf * cfg.lpp_force, cfg.block_pair);
    grid.x += nsort;
    const size_t shm = nsort ? (size_t)waves * D.capf * sizeof(unsigned) : 0;
    LAUNCH_LPP(k_fluid_force, cfg.lpp_force, D.dim, grid, dim3(cfg.block_pair), shm, st, Df);
  }
}

bool launch_fluid_continuity(const Dev &D, const LaunchCfg &cfg, hipStream_t st, bool with_couple) {
  if (D.nf == 0) return false;
  Dev Dc = D;
  Dc.couple_blocks = 0;
  if (with_couple && D.ns > 0 && cfg.lpp_couple == cfg.lpp_cont) {
    const long long threads = (long long)D.ns * cfg.lpp_cont;
    Dc.couple_blocks = (int)((threads + cfg.block_pair - 1) / cfg.block_pair + 7) / 8 * 8;
  }
  dim3 grid = grid_for((long long)D.nf * cfg.lpp_cont, cfg.block_pair);
  grid.x += Dc.couple_blocks;
  LAUNCH_LPP(k_fluid_continuity, cfg.lpp_cont, D.dim, grid, dim3(cfg.block_pair), 0, st, Dc);
  return Dc.couple_blocks > 0;
}

void launch_couple(const Dev &D, const LaunchCfg &cfg, hipStream_t st) {
  if (D.ns > 0)
    LAUNCH_LPP(k_couple, cfg.lpp_couple, D.dim, grid_for((long long)D.ns * cfg.lpp_couple, cfg.block_couple),
               dim3(cfg.block_couple), 0, st, D);
}

#define LAUNCH_SOLID_REG(ppt, ...)                                                        \
  do {                                                                                    \
    if ((ppt) == 1) hipLaunchKernelGGL((k_solid_reg<2, 1>), __VA_ARGS__);                 \
    else if ((ppt) == 2) hipLaunchKernelGGL((k_solid_reg<2, 2>), __VA_ARGS__);            \
    else hipLaunchKernelGGL((k_solid_reg<2, 4>), __VA_ARGS__);                            \
  } while (0)

void launch_solid(const Dev &D, const LaunchCfg &cfg, hipStream_t st, bool step_end, bool parts) {
  size_t bytes = (size_t)cfg.solid_lds_n * solid_lds_bytes_per_particle(D.dim);
  Dev Ds = D;
  Ds.solid_step_end = step_end ? 1 : 0;
  Ds.end_fluid_blocks = 0;
  const bool split = parts && cfg.solid_parts > 0 && D.n_parts_blocks > 0;
  Ds.solid_map = split ? D.s_parts : nullptr;
  Ds.solid_map_n = split ? D.n_parts_blocks : 0;
  int extra = 0;
  if (step_end) {
    const int T = cfg.block_solid;
    Ds.end_fluid_blocks = D.nf > 0 ? (D.nf + T * kReduceItems - 1) / (T * kReduceItems) : 0;
    extra = Ds.end_fluid_blocks + (D.nf + D.nb + T - 1) / T;
  }
  // (the scenes' workgroups come first: they are dispatched, and resident,
  // before the step-end blocks beside them)
  const int scene_blocks = split ? D.n_parts_blocks : D.n_scenes;
  LAUNCH_SOLID_REG(cfg.solid_ppt, dim3(scene_blocks + extra), dim3(cfg.block_solid), bytes, st, Ds,
                   cfg.solid_lds_n);
}

void launch_solid_dt(const Dev &D, hipStream_t st) {
  if (D.ns > 0)
    hipLaunchKernelGGL(k_solid_dt_reduce, dim3((D.ns + 256 * kReduceItems - 1) / (256 * kReduceItems)), dim3(256), 0,
                       st, D);
  hipLaunchKernelGGL(k_solid_dt_close, dim3(nblk(D.n_scenes, 64)), dim3(64), 0, st, D);
}

void launch_solid_first(const Dev &D, bool adopt, hipStream_t st) {
  if (D.ns > 0) LAUNCH_DIM(D.dim, k_solid_first, grid_for(D.ns, 256), dim3(256), st, D, adopt ? 1 : 0);
}

void launch_solid_pass(const Dev &D, int sub, hipStream_t st) {
  if (D.ns == 0) return;
  if (D.dim == 3 && D.lat_nblocks > 0) {
    const int grid = (D.lat_nblocks + kXcds - 1) / kXcds * kXcds;
    if (D.lat_jitter) {
      hipLaunchKernelGGL(k_solid_momentum_lat<true>, dim3(grid), dim3(kLatThreads), 0, st, D, sub);
      hipLaunchKernelGGL(k_solid_rate_lat<true>, dim3(grid), dim3(kLatThreads), 0, st, D, sub);
    } else {
      hipLaunchKernelGGL(k_solid_momentum_lat<false>, dim3(grid), dim3(kLatThreads), 0, st, D, sub);
      hipLaunchKernelGGL(k_solid_rate_lat<false>, dim3(grid), dim3(kLatThreads), 0, st, D, sub);
    }
    return;
  }
  LAUNCH_DIM(D.dim, k_solid_momentum, grid_for(D.ns, 256), dim3(256), st, D, sub);
  LAUNCH_DIM(D.dim, k_solid_rate, grid_for(D.ns, 256), dim3(256), st, D, sub);
}

void launch_solid_average(const Dev &D, int launched, bool maxima, hipStream_t st) {
  if (D.ns > 0)
    LAUNCH_DIM(D.dim, k_solid_average, dim3((D.ns + 256 * kReduceItems - 1) / (256 * kReduceItems)), dim3(256), st,
               D, launched, maxima ? 1 : 0);
}

void launch_sur_features(const Dev &D, const float *stats, float *x, hipStream_t st) {
  if (D.ns > 0) hipLaunchKernelGGL(k_sur_features, grid_for(D.ns, 256), dim3(256), 0, st, D, stats, x);
}

void launch_sur_targets(const Dev &D, float *t, hipStream_t st) {
  if (D.ns > 0) hipLaunchKernelGGL(k_sur_targets, grid_for(D.ns, 256), dim3(256), 0, st, D, t);
}

void launch_sur_net(const Dev &D, const MlpDev &M, hipStream_t st) {
  if (D.ns > 0)
    hipLaunchKernelGGL(k_sur_net, dim3((D.ns + kMlpTile - 1) / kMlpTile), dim3(256), fwd_lds_bytes(), st, D, M);
}

hipError_t allow_sur_net_lds() {
  return hipFuncSetAttribute((const void *)k_sur_net, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)fwd_lds_bytes());
}

void launch_step_end(const Dev &D, hipStream_t st, bool reduced, bool next_kappa) {
  int fb = (D.nf + 256 * kReduceItems - 1) / (256 * kReduceItems), sb = (D.ns + 255) / 256;
  int bb = std::min((D.nf + D.nb + 255) / 256, kBinBlocksMax);
  if (!reduced && bb + fb + sb > 0) LAUNCH_DIM(D.dim, k_step_reduce, dim3(bb + fb + sb), dim3(256), st, D, bb, fb);
  const int nk = next_kappa ? 1 : 0;
  if (step_end_scan(D)) hipLaunchKernelGGL(k_step_close_scan, dim3(1), dim3(1024), 0, st, D, nk);
  else hipLaunchKernelGGL(k_step_close, dim3(nblk(D.n_scenes, 64)), dim3(64), 0, st, D, nk);
}

int solid_lds_bytes_per_particle(int dim) { return (solid_pb_record(dim) + dim) * (int)sizeof(double); }

hipError_t allow_solid_lds(int dim, int ppt, size_t bytes) {
  if (dim != 2 || ppt <= 0) return hipErrorInvalidValue;
  const void *f = ppt == 1 ? (const void *)k_solid_reg<2, 1>
                           : (ppt == 2 ? (const void *)k_solid_reg<2, 2> : (const void *)k_solid_reg<2, 4>);
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

void launch_read(const Dev &D, int s, int field, int n, double *out, hipStream_t st) {
  if (field < 10) LAUNCH_DIM(D.dim, k_read_fluid, dim3(nblk(n, 256)), dim3(256), st, D, s, field, out);
  else LAUNCH_DIM(D.dim, k_read_solid, dim3(nblk(n, 256)), dim3(256), st, D, s, field, out);
}

void launch_write(const Dev &D, int s, int field, int n, const double *in, hipStream_t st) {
  if (field < 10) LAUNCH_DIM(D.dim, k_write_fluid, dim3(nblk(n, 256)), dim3(256), st, D, s, field, in);
  else LAUNCH_DIM(D.dim, k_write_solid, dim3(nblk(n, 256)), dim3(256), st, D, s, field, in);
}

void launch_reduce(const Dev &D, int s, int nblocks, double *part, double *out, hipStream_t st) {
  LAUNCH_DIM(D.dim, k_reduce_partial, dim3(nblocks), dim3(256), st, D, s, part);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, st, nblocks, (const double *)part, out);
}

hipError_t reduce_scratch(double **ptr) {
  // device address of `scratch` on the current device, taken once per device
  constexpr int kMaxDevices = 64;
  static std::mutex lock;
  static double *addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> guard(lock);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double *>(p);
  }
  *ptr = addr[dev];
  return hipSuccess;
}

void launch_set_rebuild(const Dev &D, int s, hipStream_t st) {
  hipLaunchKernelGGL(k_set_rebuild, dim3(1), dim3(256), 0, st, D, s);
}

void launch_unbin(const Dev &D, int s, hipStream_t st) {
  hipLaunchKernelGGL(k_unbin, dim3(1), dim3(256), 0, st, D, s);
}

void launch_bin(const Dev &D, hipStream_t st) {
  if (D.nf + D.nb > 0) LAUNCH_DIM(D.dim, k_bin, grid_for(D.nf + D.nb, 256), dim3(256), st, D);
}

void launch_prebin(const Dev &D, hipStream_t st) {
  launch_bin(D, st);
  if (step_end_scan(D)) hipLaunchKernelGGL(k_cell_one, dim3(1), dim3(1024), 0, st, D);
}

}  // namespace mrsph
