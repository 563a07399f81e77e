// HIP kernels for gfx950 and the C ABI of include/hweno.h.
//
// One workgroup advances one tile of cells through one Runge-Kutta stage
// (or evaluates the right-hand side on it):
//   1. the tile plus a two-cell halo of every field is staged in LDS with
//      coalesced row loads (boundary conditions are index maps on these
//      loads; there is no ghost-fill pass);
//   2. one thread per x-interface computes all interface fluxes
//      (characteristic HWENO f-hat, linear h-hat, mixed eta-hat) into an LDS
//      flux buffer; each thread then differences the two interfaces of its
//      own cell;
//   3. the same for the y-interfaces (same code, momenta swapped on load);
//   4. each thread limits the derivatives of its cell, applies the SSP-RK3
//      combination, stores its cell, and contributes its wave speeds to a
//      workgroup max that is folded into the next stage's global speed with
//      one 64-bit atomic max on the IEEE bit pattern.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/hweno.h"
#include "hweno_adjoint.h"
#include "hweno_math.h"

namespace hweno {

// ---------------------------------------------------------------------------
// launch arguments
// ---------------------------------------------------------------------------
template <typename T>
struct StageArgs {
  const T* in;        // stage input S_k (state layout)
  T* out;             // S_{k+1}, or the right-hand side (K == 0)
  const T* st0;       // S^n (stages 2 and 3 read U^n, and all of S^n without limiter)
  T* base;            // limited derivatives of S^n (written by stage 1, read by 2, 3)
  double* ctrl;       // step control block (stages only)
  unsigned long long* status;  // status word, or NULL
  const double* alpha;  // speeds for K == 0
  int nx, ny, bc_x, bc_y;
  long long fs;       // field stride nx * ny
  double dx, dy;
  double dt_fixed, t_end, cfl;
  int replay;
  int fold_next;      // stage 3 folds the new state's speeds into ctrl[10..11]
};

__device__ __forceinline__ int map_index(int i, int n, int bc) {
  if (bc == HWENO_BC_PERIODIC) {
    i %= n;
    return i < 0 ? i + n : i;
  }
  if (bc == HWENO_BC_REFLECT) {
    // mirror images repeat with period 2n; reducing first keeps every index
    // in range (halo loads deeper than n are never used in a result)
    i %= 2 * n;
    if (i < 0) i += 2 * n;
    return i < n ? i : 2 * n - 1 - i;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// map_index for the stage kernels, whose results use halos at most 2 deep: a
// reflecting wall has n >= 2 cells across, so one mirror step is exact for
// -2 <= i <= n + 1.  A partial tile also stages cells further out that no
// result uses; the clamp keeps those loads inside the grid.
__device__ __forceinline__ int map_index2(int i, int n, int bc) {
  if (bc == HWENO_BC_PERIODIC) {
    i %= n;
    return i < 0 ? i + n : i;
  }
  if (bc == HWENO_BC_REFLECT) i = i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// true when index i is a ghost that a reflecting boundary fills with signs
__device__ __forceinline__ bool mirrored(int i, int n, int bc) {
  return bc == HWENO_BC_REFLECT && (i < 0 || i >= n);
}

// Sign of field f (layout U[0..m), U_x[0..m), U_y[0..m)) in a ghost mirrored
// across a wall normal to direction d (0 = x, 1 = y): the wall-normal momentum
// (Euler component 1 + d) is odd, and so is every derivative along d; the
// two parities multiply.
__host__ __device__ __forceinline__ int mirror_sign(int f, int m, bool euler, int d) {
  const int c = f % m, g = f / m;
  int s = (euler && c == 1 + d) ? -1 : 1;
  if (g == 1 + d) s = -s;
  return s;
}

// Sides described by hweno_edge (HWENO_BC_EDGES) in kernel-argument form;
// sides 0..3 = x_lo, x_hi, y_lo, y_hi.
struct EdgeArgs {
  int kind[4][2];
  int mirror[4];  // the side stages with the mirror map (it has a wall segment)
  double split[4][3];
  double state[4][2][4];
  double t0;      // time of the state read by the right-hand side and the limiter entry points
  int oi, oj;     // solid cells i >= oi, j < oj (oj == 0: no obstacle)
};

// cell (i, j) of the grid is solid
__device__ __forceinline__ bool solid_cell(const EdgeArgs& e, int i, int j) {
  return j < e.oj && i >= e.oi && j >= 0;
}

// map_index2 with a per-side choice between mirror and copy on edge-described
// directions; always inside the grid
__device__ __forceinline__ int map_edge(int i, int n, int bc, int mlo, int mhi) {
  if (bc != HWENO_BC_EDGES) return map_index2(i, n, bc);
  if (i < 0)
    i = mlo ? -1 - i : 0;
  else if (i >= n)
    i = mhi ? 2 * n - 1 - i : n - 1;
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Segment (0 or 1) of side `side` taken by a ghost cell at position `pos`
// along the side, `depth` beyond it, at time t: split = s0 + s1 t + s2 depth,
// evaluated in that order with separately rounded products and sums.
__device__ __forceinline__ int edge_segment(const EdgeArgs& e, int side, double pos, double depth,
                                            double t) {
  const double sp = __dadd_rn(__dadd_rn(e.split[side][0], __dmul_rn(e.split[side][1], t)),
                              __dmul_rn(e.split[side][2], depth));
  return pos < sp ? 0 : 1;
}

// Loads and stores through the global address space.  Pointers that arrive
// through memory (the batched instance descriptors) are generic to the
// compiler, which then cannot rule out aliasing with the LDS tile and
// serialises every HBM load against the LDS writes around it.
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

__device__ __forceinline__ unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}

// workgroup reduction of two non-negative speeds (as bit patterns, so NaN
// wins) and of status flags; thread 0 folds them into global memory.
template <int NT>
__device__ __forceinline__ void block_fold(double sx, double sy, uint32_t flags,
                                           double* slot, unsigned long long* status,
                                           bool do_speeds) {
  __shared__ unsigned long long red[NT / 64][2];
  __shared__ uint32_t redf[NT / 64];
  unsigned long long bx = dbits(sx), by = dbits(sy);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    unsigned long long ox = __shfl_xor(bx, off);
    unsigned long long oy = __shfl_xor(by, off);
    uint32_t of = __shfl_xor(flags, off);
    bx = ox > bx ? ox : bx;
    by = oy > by ? oy : by;
    flags |= of;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[wv][0] = bx;
    red[wv][1] = by;
    redf[wv] = flags;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < NT / 64; ++q) {
      bx = red[q][0] > bx ? red[q][0] : bx;
      by = red[q][1] > by ? red[q][1] : by;
      flags |= redf[q];
    }
    // global-address-space atomics (see gld): the slot may come from memory.
    // The slots only grow during a launch, so a value read from them is a
    // lower bound of the final maximum: a workgroup whose maximum does not
    // exceed it has nothing to add.  Once the first workgroups have folded
    // theirs, almost every later one skips its atomic, and tens of thousands
    // of read-modify-writes no longer queue on one address.
    using gu64 = __attribute__((address_space(1))) unsigned long long;
    if (do_speeds) {
      const unsigned long long cx =
          __hip_atomic_load((gu64*)slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned long long cy =
          __hip_atomic_load((gu64*)slot + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (bx > cx) __hip_atomic_fetch_max((gu64*)slot, bx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (by > cy)
        __hip_atomic_fetch_max((gu64*)slot + 1, by, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (flags && status)
      __hip_atomic_fetch_or((gu64*)status, (unsigned long long)flags, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// Tile order.  Workgroups are dispatched round-robin over the 8 XCDs (each
// with its own L2); renumbering so that each XCD receives a contiguous band
// of tiles keeps the halo rows shared by neighbouring tiles in one L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_band(int b, int nb) {
  constexpr int NXCD = 8;
  const int per = nb / NXCD;
  if (b >= per * NXCD) return b;
  return (b % NXCD) * per + (b / NXCD);
}

// Persistent variant: the tile list is cut into 8 contiguous bands, band x
// is processed by the workgroups on XCD x (blockIdx % 8 == x), in order.
// Visits every t in [0, total) exactly once; `it` counts the iterations.
struct BandIter {
  int lb, nlb, band_lo, band_hi;
  __device__ __forceinline__ BandIter(int total) {
    constexpr int NXCD = 8;
    const int nb = (int)gridDim.x;
    if (nb < NXCD) {  // too few workgroups for one band each: plain striding
      nlb = nb;
      lb = (int)blockIdx.x;
      band_lo = 0;
      band_hi = total;
      return;
    }
    const int x = (int)blockIdx.x % NXCD;
    // workgroups of XCD x: x, x+8, ... (the last band may get fewer)
    nlb = nb / NXCD + ((nb % NXCD) > x ? 1 : 0);
    lb = (int)blockIdx.x / NXCD;
    const int per = (total + NXCD - 1) / NXCD;
    band_lo = min(x * per, total);
    band_hi = min(band_lo + per, total);
  }
  __device__ __forceinline__ int tile(int it) const { return band_lo + lb + it * nlb; }
  __device__ __forceinline__ bool valid(int it) const { return tile(it) < band_hi; }
};

// time step of stage K and the speeds it splits with (uniform per grid)
template <int DIM, int K>
__device__ __forceinline__ bool stage_dt(const StageArgs<double>* unused, double* ctrl,
                                         double dt_fixed, double t_end, double cfl, double dx,
                                         double dy, int replay, bool leader,
                                         unsigned long long* status, double& dt) {
  (void)unused;
  if constexpr (K == 1) {
    if (replay) {
      dt = ctrl[6];
    } else {
      const double alx = ctrl[0], aly = ctrl[1];
      if (dt_fixed > 0.0) {
        dt = dt_fixed;
      } else if (DIM == 1) {
        dt = cfl * dx / alx;
      } else {
        dt = cfl / (alx / dx + aly / dy);
      }
      if (t_end > 0.0) dt = fmin(dt, t_end - ctrl[7]);
      if (!(dt > 0.0) || !isfinite(dt)) dt = 0.0;
      if (leader) {
        ctrl[6] = dt;
        if (dt == 0.0) atomicOr(status, (unsigned long long)HWENO_ST_SKIPPED);
      }
    }
  } else {
    dt = ctrl[6];
  }
  return dt > 0.0;
}

// the LDS rectangle of columns [c0, c1) and rows [r0, r1) holds solid cells
__device__ __forceinline__ bool obstacle_near(const EdgeArgs& e, int c0, int c1, int r0, int r1) {
  return e.oj > 0 && c1 > e.oi && r0 < e.oj && r1 > 0;
}

// Solid cells of the staged tile take the mirror image of the fluid across the
// obstacle's front face (d = 0) or top face (d = 1), with the wall signs of
// that direction, read from the stage input.  Cells deeper than two inside the
// obstacle take a clamped, finite copy; no stencil that enters a result reads
// them.  Each thread rewrites the entries it staged.
template <typename T, int M, int NF, int HR, int W, int NT>
__device__ __forceinline__ void obstacle_mirror(const StageArgs<T>& a, const EdgeArgs& e, T* sm,
                                                int i0, int j0, int HY, int d) {
  const int nx = a.nx, ny = a.ny;
  for (int q = threadIdx.x; q < W * HR; q += NT) {
    const int lr = q / W, lc = q - lr * W;
    const int ii = i0 - 2 + lc, jj = j0 - HY + lr;
    if (!solid_cell(e, ii, jj)) continue;
    int si = d == 0 ? 2 * e.oi - 1 - ii : ii;
    int sj = d == 0 ? jj : 2 * e.oj - 1 - jj;
    si = si < 0 ? 0 : (si >= nx ? nx - 1 : si);
    sj = sj < 0 ? 0 : (sj >= ny ? ny - 1 : sj);
    const long long g = (long long)sj * nx + si;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const T x = gld(a.in + f * a.fs + g);
      sm[f * HR * W + q] = mirror_sign(f, M, true, d) < 0 ? -x : x;
    }
  }
}

// Where the stage kernels sum the linear derivative fluxes of an x-interface
// over its four stencil points: in registers in FP64 (two waves per SIMD leave
// room; the sums of the y-interfaces stay in LDS, as the x results held there
// leave none), in their flux-buffer slots in FP32 (at five waves per SIMD the
// registers spill 136-144 B per lane).
template <typename T>
struct LinReg {
  static constexpr bool value = sizeof(T) == 8;
};

// ---------------------------------------------------------------------------
// One tile of one stage (K = 1, 2, 3) or of the right-hand side (K = 0).
// NT threads; TX x TY cells (TX*TY <= NT); sm, fb: LDS staging buffers.
// Returns this thread's contribution to the next stage's speeds.
// ---------------------------------------------------------------------------
// CL: the characteristic variant of the limiter (Euler; a separate
// instantiation so the default kernels carry none of its code).
// EDG: edge-described sides (2D Euler; a separate instantiation), read from *e.
template <typename T, int PHYS, int DIM, int K, int TX, int TY, int NT, bool CL, bool EDG = false>
__device__ __forceinline__ void stage_tile(const StageArgs<T>& a, const Consts<T>& k,
                                           int tile_x, int tile_y, double dt, double alx,
                                           double aly, T* __restrict__ sm, T* __restrict__ fb,
                                           T& sx, T& sy, uint32_t& flags,
                                           const EdgeArgs* e = nullptr) {
  constexpr int M = Comps<PHYS, DIM>::M;
  constexpr int NF = Comps<PHYS, DIM>::NF;
  constexpr int HY = (DIM == 2) ? 2 : 0;
  constexpr int W = TX + 4;           // LDS row length (2-cell x halo each side)
  constexpr int HR = TY + 2 * HY;     // LDS rows
  constexpr int FW = TX + 1;          // flux buffer row length
  constexpr int FR = TY + 1;          // flux buffer rows
  constexpr bool LR = LinReg<T>::value;
  static_assert(TX * TY <= NT, "one cell per thread");

  const int tid = threadIdx.x;
  const int i0 = tile_x * TX;
  const int j0 = tile_y * TY;
  const int nx = a.nx, ny = a.ny;
  const long long fs = a.fs;

  // ---- stage the tile and its halo in LDS ----
  // All rounds' loads are issued before the first LDS write.
  constexpr int NS = (W * HR + NT - 1) / NT;
  T v[NS][NF];
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int q = tid + r * NT;
    if (q < W * HR) {
      const int lr = q / W, lc = q - lr * W;
      const int ii = i0 - 2 + lc, jj = j0 - HY + lr;
      int gi, gj;
      if constexpr (EDG) {
        gi = map_edge(ii, nx, a.bc_x, e->mirror[0], e->mirror[1]);
        gj = map_edge(jj, ny, a.bc_y, e->mirror[2], e->mirror[3]);
      } else {
        gi = map_index2(ii, nx, a.bc_x);
        gj = (DIM == 2) ? map_index2(jj, ny, a.bc_y) : 0;
      }
      const long long g = (long long)gj * nx + gi;
#pragma unroll
      for (int f = 0; f < NF; ++f) v[r][f] = gld(a.in + f * fs + g);
    }
  }
#pragma unroll
  for (int r = 0; r < NS; ++r) {
    const int q = tid + r * NT;
    if (q < W * HR) {
#pragma unroll
      for (int f = 0; f < NF; ++f) sm[f * HR * W + q] = v[r][f];
    }
  }
  if constexpr (PHYS == PH_EULER) {
    // Reflecting walls: a ghost cell holds the mirror image of an interior
    // cell with its odd fields negated.  Only tiles whose halo crosses such a
    // wall (a uniform decision) fix their LDS entries, each thread the ones it
    // stored itself, so the staging above stays the same for every tile.
    const bool wx = a.bc_x == HWENO_BC_REFLECT && (i0 - 2 < 0 || i0 - 2 + W > nx);
    const bool wy = DIM == 2 && a.bc_y == HWENO_BC_REFLECT && (j0 - HY < 0 || j0 - HY + HR > ny);
    if (wx || wy) {
      for (int q = tid; q < W * HR; q += NT) {
        const int lr = q / W, lc = q - lr * W;
        const int ii = i0 - 2 + lc, jj = j0 - HY + lr;
        const bool mx = wx && (ii < 0 || ii >= nx), my = wy && (jj < 0 || jj >= ny);
        if (!(mx || my)) continue;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          const int sg = (mx ? mirror_sign(f, M, true, 0) : 1) * (my ? mirror_sign(f, M, true, 1) : 1);
          if (sg < 0) sm[f * HR * W + q] = -sm[f * HR * W + q];
        }
      }
    }
  }
  if constexpr (EDG) {
    // Edge-described sides, at the time of this stage's input: ghost cells of
    // a wall segment take the mirror signs, those of an inflow segment the
    // prescribed state with zero derivatives; outflow segments keep the copy
    // staged above.  Corner ghosts take both rules; no stencil reads them.
    const bool ex = a.bc_x == HWENO_BC_EDGES && (i0 - 2 < 0 || i0 - 2 + W > nx);
    const bool ey = a.bc_y == HWENO_BC_EDGES && (j0 - HY < 0 || j0 - HY + HR > ny);
    if (ex || ey) {
      const double te = (K == 0) ? e->t0 : a.ctrl[7] + (K == 1 ? 0.0 : (K == 2 ? dt : 0.5 * dt));
      for (int q = tid; q < W * HR; q += NT) {
        const int lr = q / W, lc = q - lr * W;
        const int ii = i0 - 2 + lc, jj = j0 - HY + lr;
        auto apply = [&](int side, int d, double pos, double depth) {
          const int sg = edge_segment(*e, side, pos, depth, te);
          const int kd = e->kind[side][sg];
          if (kd == HWENO_SEG_REFLECT) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
              if (mirror_sign(f, M, true, d) < 0) sm[f * HR * W + q] = -sm[f * HR * W + q];
          } else if (kd == HWENO_SEG_STATE) {
#pragma unroll
            for (int f = 0; f < NF; ++f)
              sm[f * HR * W + q] = f < M ? T(e->state[side][sg][f]) : T(0);
          }
        };
        if (ex && ii < 0) apply(0, 0, (jj + 0.5) * a.dy, (-ii - 0.5) * a.dx);
        if (ex && ii >= nx) apply(1, 0, (jj + 0.5) * a.dy, (ii - nx + 0.5) * a.dx);
        if (ey && jj < 0) apply(2, 1, (ii + 0.5) * a.dx, (-jj - 0.5) * a.dy);
        if (ey && jj >= ny) apply(3, 1, (ii + 0.5) * a.dx, (jj - ny + 0.5) * a.dy);
      }
    }
    // Obstacle, x-interfaces: a solid cell holds the mirror image of the fluid
    // across the front face x = oi dx (read from the stage input, wall signs)
    if (obstacle_near(*e, i0 - 2, i0 - 2 + W, j0 - HY, j0 - HY + HR))
      obstacle_mirror<T, M, NF, HR, W, NT>(a, *e, sm, i0, j0, HY, 0);
  }
  __syncthreads();

  const T idx = T(1.0 / a.dx);
  const T hx = T(a.dx);
  const bool owner = tid < TX * TY;
  const int tx = tid % TX, ty = tid / TX;
  T LU[M], LV[M], LW[M];

  // ---- x-interfaces: between local cells ix-1 and ix, ix = 0..TX ----
  for (int q = tid; q < FW * TY; q += NT) {
    const int r = q / FW, ix = q - r * FW;
    const T* row = sm + (r + HY) * W + ix;
    auto ld = [&](int s, T* U, T* Dn, T* Dt) {
#pragma unroll
      for (int c = 0; c < M; ++c) {
        U[c] = row[(c * HR) * W + s];
        Dn[c] = row[((M + c) * HR) * W + s];
        if constexpr (DIM == 2) Dt[c] = row[((2 * M + c) * HR) * W + s];
      }
    };
    // linear fluxes: their flux-buffer slots belong to this lane; the last
    // stencil point (s = 3) completes them
    T ha[M], xa[M];
    auto lin = [&](int s, int c, T dh, T dx) {
      T& h1 = fb[((M + c) * FR + r) * FW + ix];
      T* x1 = DIM == 2 ? &fb[((2 * M + c) * FR + r) * FW + ix] : nullptr;  // 2D only
      if constexpr (LR) {
        if (s == 0) ha[c] = dh, xa[c] = dx;
        else if (s < 3) ha[c] += dh, xa[c] += dx;
        else {
          h1 = ha[c] + dh;
          if constexpr (DIM == 2) *x1 = xa[c] + dx;
        }
      } else {
        h1 = (s == 0) ? dh : h1 + dh;
        if constexpr (DIM == 2) *x1 = (s == 0) ? dx : *x1 + dx;
      }
    };
    T fh[M];
    interface_fluxes<T, PHYS, M, DIM == 2>(ld, lin, T(alx), hx, idx, k.ax, k, fh);
#pragma unroll
    for (int c = 0; c < M; ++c) fb[(c * FR + r) * FW + ix] = fh[c];
  }
  __syncthreads();
  if (owner) {
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const int b0 = (c * FR + ty) * FW + tx;
      LU[c] = -(fb[b0 + 1] - fb[b0]) * idx;
      const int b1 = ((M + c) * FR + ty) * FW + tx;
      LV[c] = -(fb[b1 + 1] - fb[b1]) * idx;
      if constexpr (DIM == 2) {
        const int b2 = ((2 * M + c) * FR + ty) * FW + tx;
        LW[c] = -(fb[b2 + 1] - fb[b2]) * idx;
      }
    }
  }

  if constexpr (DIM == 2) {
    const T idy = T(1.0 / a.dy);
    const T hy = T(a.dy);
    __syncthreads();
    if constexpr (EDG) {
      // Obstacle, y-interfaces: the mirror image across the top face y = oj dy
      if (obstacle_near(*e, i0 - 2, i0 - 2 + W, j0 - HY, j0 - HY + HR)) {
        obstacle_mirror<T, M, NF, HR, W, NT>(a, *e, sm, i0, j0, HY, 1);
        __syncthreads();
      }
    }
    // ---- y-interfaces: between local rows iy-1 and iy, iy = 0..TY ----
    for (int q = tid; q < TX * FR; q += NT) {
      const int iy = q / TX, cc = q - iy * TX;
      const T* col = sm + iy * W + cc + 2;
      auto ld = [&](int s, T* U, T* Dn, T* Dt) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          // normal frame: swap the two momenta; Dn = U_y, Dt = U_x
          const int cs = (PHYS == PH_EULER && (c == 1 || c == 2)) ? 3 - c : c;
          U[c] = col[(cs * HR + s) * W];
          Dn[c] = col[((2 * M + cs) * HR + s) * W];
          Dt[c] = col[((M + cs) * HR + s) * W];
        }
      };
      auto lin = [&](int s, int c, T dh, T dx) {
        const int cs = (PHYS == PH_EULER && (c == 1 || c == 2)) ? 3 - c : c;
        T& h1 = fb[((M + cs) * FR + iy) * FW + cc];      // theta-hat -> L_W
        h1 = (s == 0) ? dh : h1 + dh;
        T& x1 = fb[((2 * M + cs) * FR + iy) * FW + cc];  // xi-hat -> L_V
        x1 = (s == 0) ? dx : x1 + dx;
      };
      T fh[M];
      interface_fluxes<T, PHYS, M, true>(ld, lin, T(aly), hy, idy, k.ay, k, fh);
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const int cs = (PHYS == PH_EULER && (c == 1 || c == 2)) ? 3 - c : c;
        fb[(cs * FR + iy) * FW + cc] = fh[c];
      }
    }
    __syncthreads();
    if (owner) {
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const int b0 = (c * FR + ty) * FW + tx;
        LU[c] -= (fb[b0 + FW] - fb[b0]) * idy;
        const int b1 = ((M + c) * FR + ty) * FW + tx;
        LW[c] -= (fb[b1 + FW] - fb[b1]) * idy;
        const int b2 = ((2 * M + c) * FR + ty) * FW + tx;
        LV[c] -= (fb[b2 + FW] - fb[b2]) * idy;
      }
    }
  }

  // ---- own cell: limiter, Runge-Kutta combination, store ----
  const int gi = i0 + tx, gj = j0 + ty;
  const bool inside = owner && gi < nx && gj < ny;
  const long long g = (long long)gj * nx + gi;
  const T* own = sm + (ty + HY) * W + tx + 2;
  if (!inside) return;
  if constexpr (EDG) {
    if (solid_cell(*e, gi, gj)) {
      // solid: zero right-hand side, the state carried through unchanged
#pragma unroll
      for (int f = 0; f < NF; ++f) gst(a.out + f * fs + g, K == 0 ? T(0) : gld(a.in + f * fs + g));
      return;
    }
  }

  if constexpr (K == 0) {
#pragma unroll
    for (int c = 0; c < M; ++c) {
      gst(a.out + c * fs + g, LU[c]);
      gst(a.out + (M + c) * fs + g, LV[c]);
      if constexpr (DIM == 2) gst(a.out + (2 * M + c) * fs + g, LW[c]);
    }
  } else {
    // S^_k = (U_k, limited derivatives of S_k)
    T Sh[NF];
    constexpr bool charlim = CL && PHYS == PH_EULER;
    const bool complim = k.limiter_on && !charlim;
    // the x-neighbour of a fluid cell next to the obstacle's front face is that
    // cell's own mirror image (the stage buffer holds the y-image there)
    bool front = false;
    if constexpr (EDG) front = gi == e->oi - 1 && gj < e->oj;
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const T* u = own + (c * HR) * W;
      const T* v = own + ((M + c) * HR) * W;
      Sh[c] = u[0];
      T up = u[1], vp = v[1];
      if constexpr (EDG) {
        if (front) {
          up = mirror_sign(c, M, true, 0) < 0 ? -u[0] : u[0];
          vp = mirror_sign(M + c, M, true, 0) < 0 ? -v[0] : v[0];
        }
      }
      Sh[M + c] = complim ? limit1(u[-1], u[0], up, v[-1], vp, hx, idx, k.lw) : v[0];
      if constexpr (DIM == 2) {
        const T* w = own + ((2 * M + c) * HR) * W;
        Sh[2 * M + c] = complim ? limit1(u[-W], u[0], u[W], w[-W], w[W], T(a.dy),
                                         T(1.0 / a.dy), k.lw)
                                : w[0];
      }
    }
    if constexpr (charlim) {
      if (k.limiter_on) {
        // characteristic variant of the limiter, x then y (normal frame:
        // the two momenta swap places for y)
        T um[M], u0[M], up[M], vm[M], vp[M], r[M];
#pragma unroll
        for (int c = 0; c < M; ++c) {
          const T* u = own + (c * HR) * W;
          const T* v = own + ((M + c) * HR) * W;
          um[c] = u[-1], u0[c] = u[0], up[c] = u[1], vm[c] = v[-1], vp[c] = v[1];
          if constexpr (EDG) {
            if (front) {
              up[c] = mirror_sign(c, M, true, 0) < 0 ? -u[0] : u[0];
              vp[c] = mirror_sign(M + c, M, true, 0) < 0 ? -v[0] : v[0];
            }
          }
        }
        limit_char<T, M>(um, u0, up, vm, vp, hx, idx, k.lw, k.gm1, r);
#pragma unroll
        for (int c = 0; c < M; ++c) Sh[M + c] = r[c];
        if constexpr (DIM == 2) {
#pragma unroll
          for (int c = 0; c < M; ++c) {
            const int q = (c == 1) ? 2 : (c == 2) ? 1 : c;
            const T* u = own + (q * HR) * W;
            const T* w = own + ((2 * M + q) * HR) * W;
            um[c] = u[-W], u0[c] = u[0], up[c] = u[W], vm[c] = w[-W], vp[c] = w[W];
          }
          limit_char<T, M>(um, u0, up, vm, vp, T(a.dy), T(1.0 / a.dy), k.lw, k.gm1, r);
#pragma unroll
          for (int c = 0; c < M; ++c) Sh[2 * M + ((c == 1) ? 2 : (c == 2) ? 1 : c)] = r[c];
        }
      }
    }
    T L[NF];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      L[c] = LU[c];
      L[M + c] = LV[c];
      if constexpr (DIM == 2) L[2 * M + c] = LW[c];
    }
    const T tdt = T(dt);
    T out[NF];
    if constexpr (K == 1) {
#pragma unroll
      for (int f = 0; f < NF; ++f) out[f] = Sh[f] + tdt * L[f];
      if (k.limiter_on) {
#pragma unroll
        for (int f = M; f < NF; ++f) gst(a.base + (f - M) * fs + g, Sh[f]);
      }
    } else {
      const T w0 = (K == 2) ? T(0.75) : T(1.0 / 3.0);
      const T w1 = (K == 2) ? T(0.25) : T(2.0 / 3.0);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const T s0 = (f < M || !k.limiter_on) ? gld(a.st0 + f * fs + g) : gld(a.base + (f - M) * fs + g);
        out[f] = w0 * s0 + w1 * (Sh[f] + tdt * L[f]);
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) gst(a.out + f * fs + g, out[f]);
    point_speeds<T, PHYS, DIM>(out, k, sx, sy, flags);
  }
  (void)alx;
  (void)aly;
}

// ---------------------------------------------------------------------------
// stage / right-hand-side kernel over one grid
// K = 0: right-hand side only; K = 1, 2, 3: SSP-RK3 stage K.
// ---------------------------------------------------------------------------
// Resident waves per SIMD the stage kernels are compiled for (the register
// budget is 512 / WAVES per lane; LDS allows five FP32 and two FP64
// workgroups per CU).  Runge-Kutta stages: five waves in FP32 (96 VGPRs),
// two in FP64.  The right-hand-side-only FP32 kernel (K = 0) keeps three:
// at four it spills and runs 4 % slower; the FP64 one runs two waves with a
// small spill, 30 % faster than at one wave.
template <typename T, int K>
struct StageOcc {
  static constexpr int WAVES = sizeof(T) == 4 ? (K == 0 ? 3 : 5) : 2;
};

template <typename T, int PHYS, int DIM, int K, int TX, int TY, int NT, bool CL>
__global__ __launch_bounds__(NT, (StageOcc<T, K>::WAVES)) void k_stage(StageArgs<T> a, Consts<T> k) {
  constexpr int M = Comps<PHYS, DIM>::M;
  constexpr int NF = Comps<PHYS, DIM>::NF;
  constexpr int HY = (DIM == 2) ? 2 : 0;
  constexpr int NQ = (DIM == 2) ? 3 : 2;
  __shared__ T sm[NF * (TY + 2 * HY) * (TX + 4)];
  __shared__ T fb[NQ * M * (TY + 1) * (TX + 1)];

  double dt = 0.0, alx, aly;
  if constexpr (K == 0) {
    alx = a.alpha[0];
    aly = a.alpha[1];
  } else {
    alx = a.ctrl[2 * (K - 1)];
    aly = a.ctrl[2 * (K - 1) + 1];
    if (!stage_dt<DIM, K>(nullptr, a.ctrl, a.dt_fixed, a.t_end, a.cfl, a.dx, a.dy, a.replay,
                          blockIdx.x == 0 && threadIdx.x == 0, a.status, dt))
      return;  // uniform over the grid: the step is skipped
  }
  const int ntx = (a.nx + TX - 1) / TX;
  const int t = xcd_band(blockIdx.x, gridDim.x);
  const int tile_y = t / ntx, tile_x = t - tile_y * ntx;
  T sx = T(0), sy = T(0);
  uint32_t flags = 0;
  stage_tile<T, PHYS, DIM, K, TX, TY, NT, CL>(a, k, tile_x, tile_y, dt, alx, aly, sm, fb, sx, sy,
                                              flags);
  if constexpr (K > 0) {
    // speeds of the new stage state feed the next stage's splitting; after
    // stage 3 they are the next step's stage-1 speeds (multi-step calls)
    block_fold<NT>(double(sx), double(sy), flags, a.ctrl + (K < 3 ? 2 * K : 10), a.status,
                   !a.replay && (K < 3 || a.fold_next));
  }
}

// 2D Euler with edge-described sides (CL: the characteristic limiter).  The body
// repeats k_stage's: handing the kernel parameters to a shared device
// function by reference costs k_stage its register allocation (spills).
// Three waves per SIMD in FP32: at five the boundary fix-up spills.
template <typename T>
struct EdgeOcc {
  static constexpr int WAVES = sizeof(T) == 4 ? 3 : 2;
};

template <typename T, int K, int TX, int TY, int NT, bool CL>
__global__ __launch_bounds__(NT, (EdgeOcc<T>::WAVES)) void k_stage_edges(StageArgs<T> a,
                                                                             Consts<T> k,
                                                                             EdgeArgs e) {
  constexpr int PHYS = PH_EULER, DIM = 2;
  constexpr int M = Comps<PHYS, DIM>::M;
  constexpr int NF = Comps<PHYS, DIM>::NF;
  constexpr int HY = (DIM == 2) ? 2 : 0;
  constexpr int NQ = (DIM == 2) ? 3 : 2;
  __shared__ T sm[NF * (TY + 2 * HY) * (TX + 4)];
  __shared__ T fb[NQ * M * (TY + 1) * (TX + 1)];

  double dt = 0.0, alx, aly;
  if constexpr (K == 0) {
    alx = a.alpha[0];
    aly = a.alpha[1];
  } else {
    alx = a.ctrl[2 * (K - 1)];
    aly = a.ctrl[2 * (K - 1) + 1];
    if (!stage_dt<DIM, K>(nullptr, a.ctrl, a.dt_fixed, a.t_end, a.cfl, a.dx, a.dy, a.replay,
                          blockIdx.x == 0 && threadIdx.x == 0, a.status, dt))
      return;  // uniform over the grid: the step is skipped
  }
  const int ntx = (a.nx + TX - 1) / TX;
  const int t = xcd_band(blockIdx.x, gridDim.x);
  const int tile_y = t / ntx, tile_x = t - tile_y * ntx;
  T sx = T(0), sy = T(0);
  uint32_t flags = 0;
  stage_tile<T, PH_EULER, 2, K, TX, TY, NT, CL, true>(a, k, tile_x, tile_y, dt, alx, aly, sm, fb,
                                                      sx, sy, flags, &e);
  if constexpr (K > 0) {
    // speeds of the new stage state feed the next stage's splitting; after
    // stage 3 they are the next step's stage-1 speeds (multi-step calls)
    block_fold<NT>(double(sx), double(sy), flags, a.ctrl + (K < 3 ? 2 * K : 10), a.status,
                   !a.replay && (K < 3 || a.fold_next));
  }
}

// ---------------------------------------------------------------------------
// Batched 2D Euler: persistent kernels striding over the flattened tile list
// of many independent instances.
// ---------------------------------------------------------------------------
template <int V>
struct BatchTile;
template <>
struct BatchTile<0> {  // 255 x- and 256 y-interfaces: one pass each
  static constexpr int TX = 16, TY = 15, NT = 256;
};
template <>
struct BatchTile<1> {  // 231 x- and 256 y-interfaces: one pass each, wider rows
  static constexpr int TX = 32, TY = 7, NT = 256;
};


template <typename T, int K>
__device__ __forceinline__ StageArgs<T> instance_args(const hweno_instance& I, double cfl) {
  StageArgs<T> a;
  char* ws = (char*)I.ws;
  a.ctrl = (double*)ws;
  a.status = (unsigned long long*)(a.ctrl + 8);
  a.alpha = nullptr;
  a.nx = I.nx;
  a.ny = I.ny;
  a.bc_x = I.bc_x;
  a.bc_y = I.bc_y;
  a.fs = (long long)I.nx * I.ny;
  a.dx = I.dx;
  a.dy = I.dy;
  a.dt_fixed = I.dt_fixed;
  a.t_end = I.t_end;
  a.cfl = cfl;
  a.replay = 0;
  a.st0 = (const T*)I.state;
  a.base = (T*)(ws + I.off_base);
  T* s1 = (T*)(ws + I.off_s1);
  T* s2 = (T*)(ws + I.off_s2);
  a.in = (K <= 1) ? (const T*)I.state : (K == 2 ? s1 : s2);
  a.out = (K <= 1) ? s1 : (K == 2 ? s2 : (T*)I.state);
  return a;
}

// One tile t of the flattened list; nothing is done when its instance's step
// is skipped (a decision uniform over the workgroup).
template <typename T, int V, int K, bool CL>
__device__ __forceinline__ void batched_tile(const hweno_instance* __restrict__ inst,
                                             const int* __restrict__ tile_map, int t, double cfl,
                                             const Consts<T>& k, T* sm, T* fb) {
  constexpr int TX = BatchTile<V>::TX, TY = BatchTile<V>::TY, NT = BatchTile<V>::NT;
  const hweno_instance& I = inst[tile_map[t]];
  StageArgs<T> a = instance_args<T, K>(I, cfl);
  double dt;
  if (!stage_dt<2, K>(nullptr, a.ctrl, a.dt_fixed, a.t_end, cfl, a.dx, a.dy, 0,
                      t == I.tile_begin[V] && threadIdx.x == 0, a.status, dt))
    return;  // this instance's step is skipped
  const double alx = a.ctrl[2 * (K - 1)], aly = a.ctrl[2 * (K - 1) + 1];
  const int lt = t - I.tile_begin[V];
  const int ntx = (I.nx + TX - 1) / TX;
  const int tile_y = lt / ntx, tile_x = lt - tile_y * ntx;
  T sx = T(0), sy = T(0);
  uint32_t flags = 0;
  stage_tile<T, PH_EULER, 2, K, TX, TY, NT, CL>(a, k, tile_x, tile_y, dt, alx, aly, sm, fb, sx,
                                                sy, flags);
  block_fold<NT>(double(sx), double(sy), flags, a.ctrl + 2 * K, a.status, K < 3);
}

// ONE: exactly one tile per workgroup (grid = tile count, XCD-banded order).
// Nothing is written before the descriptor and control words are read, so
// those reads stay scalar and never queue behind the other workgroups'
// atomics on the same control line.  Otherwise: persistent, striding over
// XCD bands of the tile list.
template <typename T, int V, int K, bool ONE, bool CL>
__global__ __launch_bounds__(256, (StageOcc<T, K>::WAVES)) void k_stage_batched(
    const hweno_instance* __restrict__ inst, const int* __restrict__ tile_map, int total,
    double cfl, Consts<T> k) {
  constexpr int TX = BatchTile<V>::TX, TY = BatchTile<V>::TY;
  __shared__ T sm[12 * (TY + 4) * (TX + 4)];
  __shared__ T fb[12 * (TY + 1) * (TX + 1)];
  if constexpr (ONE) {
    batched_tile<T, V, K, CL>(inst, tile_map, xcd_band(blockIdx.x, gridDim.x), cfl, k, sm, fb);
  } else {
    const BandIter bi(total);
    for (int it = 0; bi.valid(it); ++it) {
      batched_tile<T, V, K, CL>(inst, tile_map, bi.tile(it), cfl, k, sm, fb);
      __syncthreads();  // LDS tile and fold slots are reused by the next tile
    }
  }
}

// speeds of every instance's state (slots pre-zeroed by k_begin_batched).
// Each workgroup walks one contiguous chunk of the tile list, keeps a running
// maximum while consecutive tiles belong to the same instance and folds it
// into that instance's slot only when the instance changes (cells are read
// once, so no halo locality is at stake here).
template <typename T, int V>
__global__ __launch_bounds__(256) void k_alpha_batched(const hweno_instance* __restrict__ inst,
                                                       const int* __restrict__ tile_map,
                                                       int total, Consts<T> k) {
  constexpr int TX = BatchTile<V>::TX, TY = BatchTile<V>::TY;
  const long long nb = gridDim.x;
  const int t_lo = (int)(total * (long long)blockIdx.x / nb);
  const int t_hi = (int)(total * ((long long)blockIdx.x + 1) / nb);
  int cur = -1;
  T sx = T(0), sy = T(0);
  uint32_t flags = 0;
  for (int t = t_lo; t < t_hi; ++t) {
    const int q = tile_map[t];
    if (q != cur) {  // uniform over the workgroup
      if (cur >= 0) {
        double* ctrl = (double*)inst[cur].ws;
        block_fold<256>(double(sx), double(sy), flags, ctrl, (unsigned long long*)(ctrl + 8), true);
        __syncthreads();  // the fold's LDS slots are reused by the next fold
        sx = sy = T(0);
        flags = 0;
      }
      cur = q;
    }
    const hweno_instance& I = inst[q];
    const int lt = t - I.tile_begin[V];
    const int ntx = (I.nx + TX - 1) / TX;
    const int tile_y = lt / ntx, tile_x = lt - tile_y * ntx;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int gi = tile_x * TX + tx, gj = tile_y * TY + ty;
    if (threadIdx.x < TX * TY && gi < I.nx && gj < I.ny) {
      const long long n = (long long)I.nx * I.ny;
      const long long g = (long long)gj * I.nx + gi;
      const T* S = (const T*)I.state;
      T U[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) U[c] = gld(S + c * n + g);
      T ax, ay;
      point_speeds<T, PH_EULER, 2>(U, k, ax, ay, flags);
      // bit-pattern max keeps NaN
      sx = (dbits(double(ax)) > dbits(double(sx))) ? ax : sx;
      sy = (dbits(double(ay)) > dbits(double(sy))) ? ay : sy;
    }
  }
  if (cur >= 0) {
    double* ctrl = (double*)inst[cur].ws;
    block_fold<256>(double(sx), double(sy), flags, ctrl, (unsigned long long*)(ctrl + 8), true);
  }
}

__global__ void k_begin_batched(const hweno_instance* __restrict__ inst, int n_inst) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n_inst) {
    double* ctrl = (double*)inst[q].ws;
#pragma unroll
    for (int j = 0; j < 6; ++j) ctrl[j] = 0.0;
  }
}

__global__ void k_finish_batched(const hweno_instance* __restrict__ inst, int n_inst) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n_inst) {
    double* ctrl = (double*)inst[q].ws;
    if (ctrl[6] > 0.0) {
      ctrl[7] += ctrl[6];
      ctrl[9] += 1.0;
    }
  }
}

// Fold the ghost-padded adjoint onto the grid and apply the pointwise
// Runge-Kutta transposes:
//   out  = [out] + fold(E) + cu * XU   (XU on U only, or on all fields when
//                                       identity_all; nothing when XU is NULL)
//   L0   = ca * A + cb * B + out       (when L0 is non-NULL)
template <typename T>
struct FoldArgs {
  const T* E;
  int nxe, nye;
  int nx, ny, bc_x, bc_y, dim, nf, m, euler;
  long long fs;
  T* out;
  int accumulate;
  const T* XU;
  double cu;
  int identity_all;
  T* L0;
  const T* A;
  const T* B;
  double ca, cb;
};

// The Runge-Kutta transposes of the NF fields of cell index q, given their
// folded adjoints v[].  Every load is issued before the first store: the
// output may not be proven distinct from the inputs, and interleaving them
// would serialise one memory round trip per field.
template <typename T, int NF>
__device__ __forceinline__ void fold_finish(const FoldArgs<T>& a, long long q, const T* v) {
  T r[NF], av[NF], bv[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const long long o = (long long)f * a.fs + q;
    r[f] = v[f];
    if (a.accumulate) r[f] += a.out[o];
    if (a.XU && (f < a.m || a.identity_all)) r[f] += T(a.cu) * a.XU[o];
    if (a.L0) {
      av[f] = a.A[o];
      bv[f] = a.B[o];
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const long long o = (long long)f * a.fs + q;
    a.out[o] = r[f];
    if (a.L0) a.L0[o] = T(a.ca) * av[f] + T(a.cb) * bv[f] + r[f];
  }
}

// field f of cell (i, j): its own entry of E plus every ghost entry the
// boundary maps read from it, then the Runge-Kutta transposes
template <typename T>
__device__ __forceinline__ void fold_cell_field(const FoldArgs<T>& a, int i, int j, int f) {
  const int GX = 2, GY = (a.dim == 2) ? 2 : 0;
  const int gx[4] = {-2, -1, a.nx, a.nx + 1};
  const int gy[4] = {-2, -1, a.ny, a.ny + 1};
  const long long q = (long long)j * a.nx + i;
  const T* Ef = a.E + (long long)f * a.nye * a.nxe;
  T v = Ef[(long long)(j + GY) * a.nxe + (i + GX)];
  // ghosts copied from this cell; a reflecting wall copied them with a sign
  const T sx = (a.bc_x == HWENO_BC_REFLECT) ? T(mirror_sign(f, a.m, a.euler, 0)) : T(1);
#pragma unroll
  for (int g = 0; g < 4; ++g)
    if (map_index(gx[g], a.nx, a.bc_x) == i) v += sx * Ef[(long long)(j + GY) * a.nxe + (gx[g] + GX)];
  if (a.dim == 2) {
    const T sy = (a.bc_y == HWENO_BC_REFLECT) ? T(mirror_sign(f, a.m, a.euler, 1)) : T(1);
#pragma unroll
    for (int g = 0; g < 4; ++g)
      if (map_index(gy[g], a.ny, a.bc_y) == j) v += sy * Ef[(long long)(gy[g] + GY) * a.nxe + (i + GX)];
  }
  const long long o = (long long)f * a.fs + q;
  T r = v;
  if (a.accumulate) r += a.out[o];
  if (a.XU && (f < a.m || a.identity_all)) r += T(a.cu) * a.XU[o];
  T av = T(0), bv = T(0);
  if (a.L0) {
    av = a.A[o];
    bv = a.B[o];
  }
  a.out[o] = r;
  if (a.L0) a.L0[o] = T(a.ca) * av + T(a.cb) * bv + r;
}

// one thread per (field, cell)
template <typename T>
__global__ __launch_bounds__(256) void k_fold(FoldArgs<T> a) {
  const long long t = blockIdx.x * 256ll + threadIdx.x;
  if (t >= a.fs * a.nf) return;
  const int f = (int)(t / a.fs);
  const long long q = t - (long long)f * a.fs;
  const int j = (int)(q / a.nx), i = (int)(q - (long long)j * a.nx);
  fold_cell_field(a, i, j, f);
}

// 2D grids with nx, ny >= 4 after a fused adjoint: only the cells within two of
// a boundary (the only ones the boundary maps read ghost entries from) are
// folded here; every other cell was finished by the adjoint kernel itself.
// Band cells are enumerated as the four columns 0, 1, nx-2, nx-1 (4*ny cells)
// and then the four rows 0, 1, ny-2, ny-1 of the columns 2..nx-3; one thread
// per (field, band cell).
template <typename T>
__global__ __launch_bounds__(256) void k_fold_band(FoldArgs<T> a) {
  const int nxb = 4 * a.ny, nb = nxb + 4 * (a.nx - 4);
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= nb * a.nf) return;
  const int f = t / nb, q = t - f * nb;
  int i, j;
  if (q < nxb) {
    const int r = q & 3;
    j = q >> 2;
    i = r < 2 ? r : a.nx - 4 + r;
  } else {
    const int r = (q - nxb) & 3;
    i = 2 + ((q - nxb) >> 2);
    j = r < 2 ? r : a.ny - 4 + r;
  }
  fold_cell_field(a, i, j, f);
}

// ---------------------------------------------------------------------------
// Discrete adjoint.  The forward operator reads ghost cells through the
// boundary index maps; its adjoint scatters into a ghost-padded buffer E
// ([nf][ny+4][nx+4] in 2D, [nf][1][nx+4] in 1D) and k_fold then adds every
// ghost entry onto the cell it was copied from.
// ---------------------------------------------------------------------------
template <typename T>
struct AdjArgs {
  const T* S;           // state the operator is linearised at
  const T* XL;          // adjoint of L is cr * XL (nf fields)
  const T* XM;          // adjoint of the limited derivatives is cl * XM (m*dim fields) or NULL
  T* E;                 // ghost-padded output
  const double* alpha;  // speeds used by the forward evaluation
  const double* dtp;    // if non-NULL, cr is multiplied by *dtp
  double cr, cl;
  int nx, ny, bc_x, bc_y;
  long long fs;
  int nxe, nye;
  double dx, dy;
  // fused: entries of real cells at least two away from every boundary are
  // folded and finished (fo's transposes) here instead of being stored in E
  int fused;
  FoldArgs<T> fo;
};

// a lane's column of an LDS buffer, read as an array
template <typename T>
struct Col {
  const T* p;
  int stride;
  __device__ T operator[](int c) const { return p[c * stride]; }
};

template <typename T>
struct AdjOcc {
  static constexpr int WAVES = sizeof(T) == 4 ? 3 : 1;
};

constexpr int cmax(int x, int y) { return x > y ? x : y; }

// One output tile of E per workgroup (TX x TY entries, ghost entries
// included).  Every interface and limiter stencil that touches the tile is
// differentiated by one lane.  Its contributions to the stencil's cells are
// handed over point by point: at each emit every lane writes the values for
// one stencil point (or one group of points) into its own column of a small
// LDS buffer, and after a barrier the owner of each output entry adds the
// column that points at it to its accumulators, one LDS slot per field and entry
// (held in registers they made the kernel spill).
// No atomics, and the buffer holds one point's contributions instead of a
// whole stencil's, so several workgroups fit on a compute unit.  The barriers
// also keep the compiler from holding the staged stencil in registers across
// the reverse pass (loads after a barrier are reloads).  Lanes without an
// interface or with a zero adjoint run the same code on a valid stencil (every
// lane takes part in every barrier) and emit exact zeros.  The state tile is
// staged cell-interleaved ([row][col][field]) so that one stencil point's
// fields are read with a few wide LDS loads.
// CL: the characteristic limiter variant (Euler), a separate instantiation.
template <typename T, int PHYS, int DIM, int TX, int TY, int NT, bool CL>
__global__ __launch_bounds__(NT, AdjOcc<T>::WAVES) void k_adjoint(AdjArgs<T> a, Consts<T> k) {
  constexpr int M = Comps<PHYS, DIM>::M;
  constexpr int NF = Comps<PHYS, DIM>::NF;
  constexpr int GX = 2, GY = (DIM == 2) ? 2 : 0;  // ghost width of E
  constexpr int HX = 3, HY = (DIM == 2) ? 3 : 0;  // state halo around the tile
  constexpr int W = TX + 2 * HX, HR = TY + 2 * HY;
  constexpr int NIX = TY * (TX + 3);                   // x-interfaces touching the tile
  constexpr int NIY = (DIM == 2) ? TX * (TY + 3) : 0;  // y-interfaces
  constexpr int NLX = TY * (TX + 2);                   // cells whose x-limiter touches it
  constexpr int NLY = (DIM == 2) ? TX * (TY + 2) : 0;
  constexpr int NR = cmax(NF, 3 * M);                  // rows of the hand-over buffer
  static_assert(TX * TY <= NT, "one output entry per thread");
  static_assert(NIX <= NT && NIY <= NT && NLX <= NT && NLY <= NT, "one stencil per lane");
  __shared__ __align__(16) T sm[HR * W * NF];
  __shared__ T pt[NR * NT];
  __shared__ T accs[NF * TX * TY];
  __shared__ T gin[2 * M * NT];  // this lane's adjoints of h-hat and of the mixed flux
  const int nx = a.nx, ny = a.ny;
  const long long fs = a.fs;
  const int ntx = (a.nxe + TX - 1) / TX;
  const int t = xcd_band(blockIdx.x, gridDim.x);
  const int bty = t / ntx, btx = t - bty * ntx;
  const int rx0 = btx * TX - GX, ry0 = bty * TY - GY;  // real coordinates of tile entry (0, 0)
  const int tid = threadIdx.x;
  const T cr = T(a.cr * (a.dtp ? *a.dtp : 1.0));
  const T cl = T(a.cl);
  for (int q = tid; q < W * HR; q += NT) {
    const int lr = q / W, lc = q - lr * W;
    const int ii = rx0 - HX + lc, jj = ry0 - HY + lr;
    const int gi = map_index(ii, nx, a.bc_x);
    const int gj = (DIM == 2) ? map_index(jj, ny, a.bc_y) : 0;
    const long long g = (long long)gj * nx + gi;
    const bool mx = mirrored(ii, nx, a.bc_x), my = DIM == 2 && mirrored(jj, ny, a.bc_y);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const T x = a.S[f * fs + g];
      const int sg = (mx ? mirror_sign(f, M, PHYS == PH_EULER, 0) : 1) *
                     (my ? mirror_sign(f, M, PHYS == PH_EULER, 1) : 1);
      sm[q * NF + f] = sg < 0 ? -x : x;
    }
  }
  __syncthreads();

  auto xl = [&](int f, int i, int j) -> T {
    return (i >= 0 && i < nx && j >= 0 && j < ny) ? a.XL[f * fs + (long long)j * nx + i] : T(0);
  };
  // cell (i, j) of the staged state
  auto cell = [&](int i, int j) -> const T* {
    return sm + ((j - (ry0 - HY)) * W + (i - (rx0 - HX))) * NF;
  };
  const bool owner = tid < TX * TY;
  const int lx = tid % TX, ly = tid / TX;
  const T idx = T(1.0 / a.dx), hx = T(a.dx);
  T* acc = accs + (owner ? tid : 0);
  constexpr int AS = TX * TY;  // stride of the accumulator fields
  if (owner) {
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f * AS] = T(0);
  }
  // row r of this lane's column of the hand-over buffer
  auto put = [&](int r, T v) { pt[r * NT + tid] = v; };
  auto col = [&](int r, int q) -> T { return pt[r * NT + q]; };

  // ---- x-interfaces I (between cells I and I+1) that touch the tile ----
  {
    // lanes past the last interface take the last one, with a zero adjoint
    const int q = tid < NIX ? tid : NIX - 1;
    const int r = q / (TX + 3), ii = q - r * (TX + 3);
    const int j = ry0 + r, I = rx0 - 2 + ii;
    T gf[M], gh[M], gx[M];
    bool any = false;
    const bool live = tid < NIX && j >= 0 && j < ny && I >= -1 && I <= nx - 1;
#pragma unroll
    for (int c = 0; c < M; ++c) {
      gf[c] = live ? cr * (xl(c, I + 1, j) - xl(c, I, j)) * idx : T(0);
      gh[c] = live ? cr * (xl(M + c, I + 1, j) - xl(M + c, I, j)) * idx : T(0);
      gx[c] = (DIM == 2 && live) ? cr * (xl(2 * M + c, I + 1, j) - xl(2 * M + c, I, j)) * idx : T(0);
      any = any || gf[c] != T(0) || gh[c] != T(0) || gx[c] != T(0);
    }
#pragma unroll
    for (int c = 0; c < M; ++c) {
      gin[c * NT + tid] = gh[c];
      gin[(M + c) * NT + tid] = gx[c];
    }
    const Col<T> ghc{gin + tid, NT}, gxc{gin + M * NT + tid, NT};
    const T* row = cell(I - 1, j);
    auto ld = [&](int s, T* U, T* Dn, T* Dt) {
      const T* p = row + s * NF;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        U[c] = p[c];
        Dn[c] = p[M + c];
        Dt[c] = (DIM == 2) ? p[2 * M + c] : T(0);
      }
    };
    // entry (lx, ly) is point s of interface ii = lx + 3 - s in its row
    const int qo = ly * (TX + 3) + lx + 3;
    auto emit = [&](int s, int mode, const T* gU, const T* gDn, const T* gDt) {
      if (mode == EMIT_ADD_U) {
        // the Roe-average contributions to points 1 and 2 share one hand-over
#pragma unroll
        for (int c = 0; c < M; ++c) put((s == 1 ? 0 : M) + c, any ? gU[c] : T(0));
        if (s == 1) return;
      } else {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          put(c, any ? gU[c] : T(0));
          put(M + c, any ? gDn[c] : T(0));
          if constexpr (DIM == 2) put(2 * M + c, any ? gDt[c] : T(0));
        }
      }
      __syncthreads();
      if (owner) {
        if (mode == EMIT_ADD_U) {
#pragma unroll
          for (int c = 0; c < M; ++c) acc[(c) * AS] += col(c, qo - 1) + col(M + c, qo - 2);
        } else {
#pragma unroll
          for (int f = 0; f < NF; ++f) acc[(f) * AS] += col(f, qo - s);
        }
      }
      __syncthreads();
    };
    interface_vjp<T, PHYS, M, DIM == 2>(ld, T(a.alpha[0]), hx, idx, k.ax, k, gf, ghc, gxc, emit);
  }

  if constexpr (DIM == 2) {
    const T idy = T(1.0 / a.dy), hy = T(a.dy);
    // ---- y-interfaces J (between rows J and J+1) that touch the tile ----
    const int q = tid < NIY ? tid : NIY - 1;
    const int jj = q / TX, cc = q - jj * TX;
    const int i = rx0 + cc, J = ry0 - 2 + jj;
    T gf[M], gh[M], gx[M];
    bool any = false;
    const bool live = tid < NIY && i >= 0 && i < nx && J >= -1 && J <= ny - 1;
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const int cs = (PHYS == PH_EULER && (c == 1 || c == 2)) ? 3 - c : c;
      gf[c] = live ? cr * (xl(cs, i, J + 1) - xl(cs, i, J)) * idy : T(0);
      gh[c] = live ? cr * (xl(2 * M + cs, i, J + 1) - xl(2 * M + cs, i, J)) * idy : T(0);  // theta-hat
      gx[c] = live ? cr * (xl(M + cs, i, J + 1) - xl(M + cs, i, J)) * idy : T(0);          // xi-hat
      any = any || gf[c] != T(0) || gh[c] != T(0) || gx[c] != T(0);
    }
    __syncthreads();  // the x pass's last readers of gin are done
#pragma unroll
    for (int c = 0; c < M; ++c) {
      gin[c * NT + tid] = gh[c];
      gin[(M + c) * NT + tid] = gx[c];
    }
    const Col<T> ghc{gin + tid, NT}, gxc{gin + M * NT + tid, NT};
    const T* colp = cell(i, J - 1);
    auto ld = [&](int s, T* U, T* Dn, T* Dt) {
      const T* p = colp + s * (W * NF);
#pragma unroll
      for (int c = 0; c < M; ++c) {
        // normal frame: swap the two momenta; Dn = U_y, Dt = U_x
        const int cs = (PHYS == PH_EULER && (c == 1 || c == 2)) ? 3 - c : c;
        U[c] = p[cs];
        Dn[c] = p[2 * M + cs];
        Dt[c] = p[M + cs];
      }
    };
    // entry (lx, ly) is point s of interface jj = ly + 3 - s in its column
    const int qo = (ly + 3) * TX + lx;
    auto emit = [&](int s, int mode, const T* gU, const T* gDn, const T* gDt) {
      if (mode == EMIT_ADD_U) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          const int cs = (PHYS == PH_EULER && (c == 1 || c == 2)) ? 3 - c : c;
          put((s == 1 ? 0 : M) + cs, any ? gU[c] : T(0));
        }
        if (s == 1) return;
      } else {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          const int cs = (PHYS == PH_EULER && (c == 1 || c == 2)) ? 3 - c : c;
          put(cs, any ? gU[c] : T(0));
          put(2 * M + cs, any ? gDn[c] : T(0));
          put(M + cs, any ? gDt[c] : T(0));
        }
      }
      __syncthreads();
      if (owner) {
        if (mode == EMIT_ADD_U) {
#pragma unroll
          for (int c = 0; c < M; ++c) acc[(c) * AS] += col(c, qo - TX) + col(M + c, qo - 2 * TX);
        } else {
#pragma unroll
          for (int f = 0; f < NF; ++f) acc[(f) * AS] += col(f, qo - s * TX);
        }
      }
      __syncthreads();
    };
    interface_vjp<T, PHYS, M, true>(ld, T(a.alpha[1]), hy, idy, k.ay, k, gf, ghc, gxc, emit);
  }

  // ---- limiter: U_x along x (and U_y along y) of cells near the tile ----
  // contributions of the limiter at cell C, component c: U at C-1, C, C+1
  // (handed over together), then the derivative at C-1 and C+1
  if (a.XM) {
    {
      const int q = tid < NLX ? tid : NLX - 1;
      const int r = q / (TX + 2), ii = q - r * (TX + 2);
      const int j = ry0 + r, C = rx0 - 1 + ii;
      const bool live = tid < NLX && j >= 0 && j < ny && C >= 0 && C < nx;
      const T* p = live ? cell(C, j) : sm + NF;
      T g[5][M];
#pragma unroll
      for (int c = 0; c < M; ++c)
#pragma unroll
        for (int s5 = 0; s5 < 5; ++s5) g[s5][c] = T(0);
      if constexpr (CL && PHYS == PH_EULER) {
        T mu[M];
        bool any = false;
#pragma unroll
        for (int c = 0; c < M; ++c) {
          mu[c] = live ? cl * a.XM[c * fs + (long long)j * nx + C] : T(0);
          any = any || mu[c] != T(0);
        }
        if (any) {
          T um[M], u0[M], up[M], vm[M], vp[M];
#pragma unroll
          for (int c = 0; c < M; ++c) {
            um[c] = p[-NF + c], u0[c] = p[c], up[c] = p[NF + c];
            vm[c] = p[-NF + M + c], vp[c] = p[NF + M + c];
          }
          limit_char_vjp<T, M>(um, u0, up, vm, vp, hx, idx, k.lw, k.gm1, mu, g[0], g[1], g[2],
                               g[3], g[4]);
        }
      } else {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          const T mu = live ? cl * a.XM[c * fs + (long long)j * nx + C] : T(0);
          if (mu != T(0))
            limit1_vjp(p[-NF + c], p[c], p[NF + c], p[-NF + M + c], p[NF + M + c], hx, idx, k.lw,
                       mu, g[0][c], g[1][c], g[2][c], g[3][c], g[4][c]);
        }
      }
      // entry P = rx0 + lx: the limiter of cell C sits at ii = C - rx0 + 1
      const int qb = ly * (TX + 2) + lx + 1;
#pragma unroll
      for (int c = 0; c < M; ++c) {
        put(c, g[0][c]);
        put(M + c, g[1][c]);
        put(2 * M + c, g[2][c]);
      }
      __syncthreads();
      if (owner) {
#pragma unroll
        for (int c = 0; c < M; ++c)
          acc[(c) * AS] += col(c, qb + 1) + col(M + c, qb) + col(2 * M + c, qb - 1);
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < M; ++c) {
        put(c, g[3][c]);
        put(M + c, g[4][c]);
      }
      __syncthreads();
      if (owner) {
#pragma unroll
        for (int c = 0; c < M; ++c) acc[(M + c) * AS] += col(c, qb + 1) + col(M + c, qb - 1);
      }
      __syncthreads();
    }
    if constexpr (DIM == 2) {
      const T idy = T(1.0 / a.dy), hy = T(a.dy);
      const int q = tid < NLY ? tid : NLY - 1;
      const int jj = q / TX, cc = q - jj * TX;
      const int i = rx0 + cc, C = ry0 - 1 + jj;
      const bool live = tid < NLY && i >= 0 && i < nx && C >= 0 && C < ny;
      const T* p = live ? cell(i, C) : sm + W * NF;
      constexpr int S = W * NF;
      T g[5][M];
#pragma unroll
      for (int c = 0; c < M; ++c)
#pragma unroll
        for (int s5 = 0; s5 < 5; ++s5) g[s5][c] = T(0);
      if constexpr (CL && PHYS == PH_EULER) {
        // normal frame: the two momenta swap places (as in the forward); the
        // gradients come back in that frame and are swapped on hand-over
        T mu[M];
        bool any = false;
#pragma unroll
        for (int c = 0; c < M; ++c) {
          const int qc = (c == 1) ? 2 : (c == 2) ? 1 : c;
          mu[c] = live ? cl * a.XM[(M + qc) * fs + (long long)C * nx + i] : T(0);
          any = any || mu[c] != T(0);
        }
        if (any) {
          T um[M], u0[M], up[M], vm[M], vp[M];
#pragma unroll
          for (int c = 0; c < M; ++c) {
            const int qc = (c == 1) ? 2 : (c == 2) ? 1 : c;
            um[c] = p[-S + qc], u0[c] = p[qc], up[c] = p[S + qc];
            vm[c] = p[-S + 2 * M + qc], vp[c] = p[S + 2 * M + qc];
          }
          limit_char_vjp<T, M>(um, u0, up, vm, vp, hy, idy, k.lw, k.gm1, mu, g[0], g[1], g[2],
                               g[3], g[4]);
        }
      } else {
#pragma unroll
        for (int c = 0; c < M; ++c) {
          const T mu = live ? cl * a.XM[(M + c) * fs + (long long)C * nx + i] : T(0);
          if (mu != T(0))
            limit1_vjp(p[-S + c], p[c], p[S + c], p[-S + 2 * M + c], p[S + 2 * M + c], hy, idy,
                       k.lw, mu, g[0][c], g[1][c], g[2][c], g[3][c], g[4][c]);
        }
      }
      auto fc = [&](int c) { return (CL && PHYS == PH_EULER) ? ((c == 1) ? 2 : (c == 2) ? 1 : c) : c; };
      const int qb = (ly + 1) * TX + lx;  // jj of C = P
#pragma unroll
      for (int c = 0; c < M; ++c) {
        put(fc(c), g[0][c]);
        put(M + fc(c), g[1][c]);
        put(2 * M + fc(c), g[2][c]);
      }
      __syncthreads();
      if (owner) {
#pragma unroll
        for (int c = 0; c < M; ++c)
          acc[(c) * AS] += col(c, qb + TX) + col(M + c, qb) + col(2 * M + c, qb - TX);
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < M; ++c) {
        put(fc(c), g[3][c]);
        put(M + fc(c), g[4][c]);
      }
      __syncthreads();
      if (owner) {
#pragma unroll
        for (int c = 0; c < M; ++c) acc[(2 * M + c) * AS] += col(c, qb + TX) + col(M + c, qb - TX);
      }
    }
  }
  if (owner) {
    const int ex = btx * TX + lx, ey = bty * TY + ly;
    if (ex < a.nxe && ey < a.nye) {
      const int i = ex - GX, j = ey - GY;
      const bool inner = i >= 2 && i < nx - 2 && (DIM == 1 || (j >= 2 && j < ny - 2));
      T v[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) v[f] = acc[f * AS];
      if (a.fused && inner) {
        fold_finish<T, NF>(a.fo, (long long)j * nx + i, v);
      } else {
#pragma unroll
        for (int f = 0; f < NF; ++f) a.E[((long long)f * a.nye + ey) * a.nxe + ex] = v[f];
      }
    }
  }
}

// global speeds of a state: alpha[0..1] = max over cells (target pre-zeroed)
template <typename T, int PHYS, int DIM>
__global__ __launch_bounds__(256) void k_alpha(const T* __restrict__ S, long long n,
                                               Consts<T> k, double* alpha,
                                               unsigned long long* status) {
  constexpr int M = Comps<PHYS, DIM>::M;
  T mx = T(0), my = T(0);
  uint32_t flags = 0;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
    T U[M];
#pragma unroll
    for (int c = 0; c < M; ++c) U[c] = S[c * n + i];
    T sx, sy;
    point_speeds<T, PHYS, DIM>(U, k, sx, sy, flags);
    // bit-pattern max keeps NaN
    mx = (dbits(double(sx)) > dbits(double(mx))) ? sx : mx;
    my = (dbits(double(sy)) > dbits(double(my))) ? sy : my;
  }
  block_fold<256>(double(mx), double(my), flags, alpha, status, true);
}

// k_alpha over the fluid cells of a 2D Euler grid with an obstacle (solid
// cells enter no speed)
template <typename T>
__global__ __launch_bounds__(256) void k_alpha_obstacle(const T* __restrict__ S, int nx, int ny,
                                                        int oi, int oj, Consts<T> k,
                                                        double* alpha, unsigned long long* status) {
  const long long n = (long long)nx * ny;
  T mx = T(0), my = T(0);
  uint32_t flags = 0;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += 256ll * gridDim.x) {
    const int j = (int)(i / nx), c = (int)(i - (long long)j * nx);
    if (j < oj && c >= oi) continue;
    T U[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) U[q] = S[q * n + i];
    T sx, sy;
    point_speeds<T, PH_EULER, 2>(U, k, sx, sy, flags);
    mx = (dbits(double(sx)) > dbits(double(mx))) ? sx : mx;
    my = (dbits(double(sy)) > dbits(double(my))) ? sy : my;
  }
  block_fold<256>(double(mx), double(my), flags, alpha, status, true);
}

// Start of a step: stage speeds and dt from the replay record, or speeds
// cleared for the speed reduction; the next-step speed slots ctrl[10..11]
// are cleared for this step's stage 3 (multi-step calls fold into them).
__global__ void k_begin(double* ctrl, const double* replay) {
  const int t = threadIdx.x;
  if (replay) {
    if (t < 7) ctrl[t] = replay[t];
  } else if (t < 6) {
    ctrl[t] = 0.0;
  }
  if (t == 10 || t == 11) ctrl[t] = 0.0;
}

__global__ void k_zero(double* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

// End of a step: time and step count, tape record.  begin_next: also start
// the next step of a multi-step call (what k_begin does with take_next), so
// consecutive steps need one small launch between them instead of two.
__global__ void k_finish(double* ctrl, double* tape, int begin_next) {
  if (threadIdx.x == 0) {
    if (ctrl[6] > 0.0) {
      ctrl[7] += ctrl[6];
      ctrl[9] += 1.0;
    } else {
      // skipped step: the state is unchanged, so the next step's stage-1
      // speeds (taken from ctrl[10..11] in multi-step calls) are this step's
      ctrl[10] = ctrl[0];
      ctrl[11] = ctrl[1];
    }
    if (tape) {
      for (int q = 0; q < 10; ++q) tape[q] = ctrl[q];
    }
  }
  if (begin_next) {
    __syncthreads();
    const int t = threadIdx.x;
    const double nxt = t < 2 ? ctrl[10 + t] : 0.0;
    __syncthreads();
    if (t < 6) ctrl[t] = nxt;
    if (t == 10 || t == 11) ctrl[t] = 0.0;
  }
}

// limited derivatives (Section 2.2), one thread per cell, all components
// One neighbour of a cell for the limiter: its cell index and what a ghost
// there holds (0: a copy, 1: the mirror image with the wall signs, 2: the
// prescribed state `st` with zero derivatives).
struct LimNb {
  long long at;
  int mode;
  const double* st;
};

template <typename T, int PHYS, int DIM>
__global__ __launch_bounds__(256) void k_limit(const T* __restrict__ S, T* __restrict__ out,
                                               int nx, int ny, int bc_x, int bc_y,
                                               double dx, double dy, Consts<T> k, EdgeArgs e) {
  constexpr int M = Comps<PHYS, DIM>::M;
  const long long n = (long long)nx * ny;
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= n) return;
  const int gj = (int)(i / nx), gi = (int)(i - (long long)gj * nx);
  constexpr bool EU = PHYS == PH_EULER;
  if (e.oj > 0 && solid_cell(e, gi, gj)) {
    // solid cells keep their derivatives
    for (int f = 0; f < M * DIM; ++f) out[f * n + i] = S[(M + f) * n + i];
    return;
  }
  // neighbour at index q (column or row) along direction d; one cell deep,
  // so mirror and copy read the same interior cell
  auto neighbour = [&](int q, int d) -> LimNb {
    const int nn = d == 0 ? nx : ny, bc = d == 0 ? bc_x : bc_y;
    const int mq = map_index(q, nn, bc);
    LimNb r;
    r.at = d == 0 ? (long long)gj * nx + mq : (long long)mq * nx + gi;
    r.mode = mirrored(q, nn, bc) ? 1 : 0;
    r.st = nullptr;
    if (e.oj > 0 && (d == 0 ? solid_cell(e, q, gj) : solid_cell(e, gi, q))) {
      // a solid neighbour is the cell's own mirror image across the obstacle's face
      r.at = i;
      r.mode = 1;
      return r;
    }
    if (bc == HWENO_BC_EDGES && (q < 0 || q >= nn)) {
      const int side = 2 * d + (q < 0 ? 0 : 1);
      const double pos = d == 0 ? (gj + 0.5) * dy : (gi + 0.5) * dx;
      const int sg = edge_segment(e, side, pos, 0.5 * (d == 0 ? dx : dy), e.t0);
      const int kd = e.kind[side][sg];
      r.mode = kd == HWENO_SEG_REFLECT ? 1 : (kd == HWENO_SEG_STATE ? 2 : 0);
      r.st = e.state[side][sg];
    }
    return r;
  };
  const LimNb nxm = neighbour(gi - 1, 0), nxp = neighbour(gi + 1, 0);
  // value of field f at a neighbour: a copy, the wall signs of a mirrored
  // ghost, or an inflow state
  auto nbv = [&](int f, const LimNb& b, int d) -> T {
    if (b.mode == 2) return f < M ? T(b.st[f]) : T(0);
    const T x = S[f * n + b.at];
    return (b.mode == 1 && mirror_sign(f, M, EU, d) < 0) ? -x : x;
  };
  if (EU && k.limiter_char) {
    // characteristic variant (normal frame: the momenta swap places for y)
    T um[M], u0[M], up[M], vm[M], vp[M], r[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      um[c] = nbv(c, nxm, 0), u0[c] = S[c * n + i], up[c] = nbv(c, nxp, 0);
      vm[c] = nbv(M + c, nxm, 0), vp[c] = nbv(M + c, nxp, 0);
    }
    limit_char<T, M>(um, u0, up, vm, vp, T(dx), T(1.0 / dx), k.lw, k.gm1, r);
#pragma unroll
    for (int c = 0; c < M; ++c) out[c * n + i] = r[c];
    if constexpr (DIM == 2) {
      const LimNb nym = neighbour(gj - 1, 1), nyp = neighbour(gj + 1, 1);
#pragma unroll
      for (int c = 0; c < M; ++c) {
        const int q = (c == 1) ? 2 : (c == 2) ? 1 : c;
        um[c] = nbv(q, nym, 1), u0[c] = S[q * n + i], up[c] = nbv(q, nyp, 1);
        vm[c] = nbv(2 * M + q, nym, 1), vp[c] = nbv(2 * M + q, nyp, 1);
      }
      limit_char<T, M>(um, u0, up, vm, vp, T(dy), T(1.0 / dy), k.lw, k.gm1, r);
#pragma unroll
      for (int c = 0; c < M; ++c) out[(M + ((c == 1) ? 2 : (c == 2) ? 1 : c)) * n + i] = r[c];
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < M; ++c) {
    out[c * n + i] = limit1(nbv(c, nxm, 0), S[c * n + i], nbv(c, nxp, 0), nbv(M + c, nxm, 0),
                            nbv(M + c, nxp, 0), T(dx), T(1.0 / dx), k.lw);
  }
  if constexpr (DIM == 2) {
    const LimNb nym = neighbour(gj - 1, 1), nyp = neighbour(gj + 1, 1);
#pragma unroll
    for (int c = 0; c < M; ++c) {
      out[(M + c) * n + i] = limit1(nbv(c, nym, 1), S[c * n + i], nbv(c, nyp, 1),
                                    nbv(2 * M + c, nym, 1), nbv(2 * M + c, nyp, 1), T(dy),
                                    T(1.0 / dy), k.lw);
    }
  }
}

}  // namespace hweno

// ===========================================================================
// host side
// ===========================================================================
using namespace hweno;

// Stage states and limited base derivatives of the allocation-free step
// (hweno_rk3_step_static).  Each GPU that runs the library holds its own copy
// for the life of the process.  On the host this name is only a handle for
// hipGetSymbolAddress: kernels receive the device address it returns.
static __device__ __align__(256) unsigned char scratch[HWENO_STATIC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

// stage-kernel timing (diagnostics, per host thread)
struct Timing {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t used = 0;
};
thread_local Timing g_timing;

hipEvent_t* timing_pair(hipStream_t s, bool start) {
  (void)s;
  if (!g_timing.on) return nullptr;
  if (start) {
    if (g_timing.used == g_timing.ev.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) return nullptr;
      if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return nullptr; }
      g_timing.ev.emplace_back(a, b);
    }
    return &g_timing.ev[g_timing.used].first;
  }
  return &g_timing.ev[g_timing.used++].second;
}

void timing_release() {
  for (auto& e : g_timing.ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  g_timing.ev.clear();
  g_timing.used = 0;
  g_timing.on = false;
}

// launches one stage kernel, bracketed by timing events when enabled
template <typename Launch>
void timed(hipStream_t s, Launch&& launch) {
  hipEvent_t* a = timing_pair(s, true);
  if (a) (void)hipEventRecord(*a, s);
  launch();
  if (a) (void)hipEventRecord(*timing_pair(s, false), s);
}

hweno_status fail(hweno_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

hweno_status ok() {
  g_last_error.clear();
  return HWENO_OK;
}

int n_comp(const hweno_problem* p) {
  if (p->physics == HWENO_EULER) return p->dim == 1 ? 3 : 4;
  return 1;
}

int n_fields(const hweno_problem* p) { return n_comp(p) * (1 + p->dim); }

size_t elem_size(const hweno_problem* p) { return p->dtype == HWENO_F64 ? 8 : 4; }

bool weights_ok(const double* w) {
  if (!(w[0] > 0.0 && w[1] > 0.0 && w[2] > 0.0)) return false;
  if (!std::isfinite(w[0] + w[1] + w[2])) return false;
  return std::fabs(w[0] + w[1] + w[2] - 1.0) <= 1e-12;
}

bool has_edges(const hweno_problem* p) {
  return p->bc_x == HWENO_BC_EDGES || (p->dim == 2 && p->bc_y == HWENO_BC_EDGES);
}

hweno_status validate(const hweno_problem* p) {
  if (!p) return fail(HWENO_ERR_INVALID_ARG, "problem pointer is NULL");
  if (p->dim != 1 && p->dim != 2) return fail(HWENO_ERR_INVALID_ARG, "dim must be 1 or 2 (got %d)", p->dim);
  if (p->nx < 0 || p->ny < 0) return fail(HWENO_ERR_INVALID_ARG, "nx, ny must be >= 0");
  if (p->dim == 1 && p->ny != 1 && p->ny != 0)
    return fail(HWENO_ERR_INVALID_ARG, "ny must be 1 for dim == 1 (got %d)", p->ny);
  if (p->physics < HWENO_LINADV || p->physics > HWENO_EULER)
    return fail(HWENO_ERR_INVALID_ARG, "unknown physics %d", p->physics);
  if (p->dtype != HWENO_F32 && p->dtype != HWENO_F64)
    return fail(HWENO_ERR_INVALID_ARG, "unknown dtype %d", p->dtype);
  auto bc_ok = [](int b) {
    return b == HWENO_BC_PERIODIC || b == HWENO_BC_OUTFLOW || b == HWENO_BC_REFLECT ||
           b == HWENO_BC_EDGES;
  };
  if (!bc_ok(p->bc_x) || (p->dim == 2 && !bc_ok(p->bc_y)))
    return fail(HWENO_ERR_INVALID_ARG, "unknown boundary condition");
  if (p->obstacle[0] != 0 || p->obstacle[1] != 0) {
    if (p->dim != 2 || p->bc_x != HWENO_BC_EDGES)
      return fail(HWENO_ERR_UNSUPPORTED, "an obstacle needs a 2D grid with edge-described x sides");
    if (p->obstacle[0] < 2 || p->obstacle[0] > p->nx || p->obstacle[1] < 1 ||
        p->obstacle[1] > p->ny - 2)
      return fail(HWENO_ERR_INVALID_ARG,
                  "obstacle {%d, %d}: needs 2 <= i_s <= nx and 1 <= j_s <= ny - 2",
                  p->obstacle[0], p->obstacle[1]);
  }
  if (has_edges(p)) {
    if (p->physics != HWENO_EULER || p->dim != 2)
      return fail(HWENO_ERR_UNSUPPORTED, "edge-described sides are built for 2D Euler");
    for (int d = 0; d < 2; ++d) {
      if ((d == 0 ? p->bc_x : p->bc_y) != HWENO_BC_EDGES) continue;
      const int across = d == 0 ? p->nx : p->ny;
      for (int side = 0; side < 2; ++side) {
        const hweno_edge& e = p->edges[2 * d + side];
        bool out = false, wall = false;
        for (int sg = 0; sg < 2; ++sg) {
          const int kd = e.kind[sg];
          if (kd != HWENO_SEG_OUTFLOW && kd != HWENO_SEG_REFLECT && kd != HWENO_SEG_STATE)
            return fail(HWENO_ERR_INVALID_ARG, "edge %d: unknown segment kind %d", 2 * d + side, kd);
          out = out || kd == HWENO_SEG_OUTFLOW;
          wall = wall || kd == HWENO_SEG_REFLECT;
          if (kd == HWENO_SEG_STATE) {
            const double* q = e.state[sg];
            for (int c = 0; c < 4; ++c)
              if (!std::isfinite(q[c]))
                return fail(HWENO_ERR_INVALID_ARG, "edge %d: state %d is not finite", 2 * d + side, sg);
            const double pr =
                (p->gamma_gas - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);
            if (!(q[0] > 0.0) || !(pr > 0.0))
              return fail(HWENO_ERR_INVALID_ARG,
                          "edge %d: state %d needs positive density and pressure", 2 * d + side, sg);
          }
        }
        for (int k = 0; k < 3; ++k)
          if (!std::isfinite(e.split[k]))
            return fail(HWENO_ERR_INVALID_ARG, "edge %d: split is not finite", 2 * d + side);
        if (out && wall)
          return fail(HWENO_ERR_INVALID_ARG, "edge %d combines an outflow and a wall segment",
                      2 * d + side);
        if (wall && across < 2)
          return fail(HWENO_ERR_INVALID_ARG, "a reflecting wall needs at least 2 cells across");
      }
    }
  }
  if (p->physics != HWENO_EULER &&
      (p->bc_x == HWENO_BC_REFLECT || (p->dim == 2 && p->bc_y == HWENO_BC_REFLECT)))
    return fail(HWENO_ERR_UNSUPPORTED, "reflecting walls are defined for the Euler equations only");
  // the two ghost cells mirror two distinct interior cells
  if ((p->bc_x == HWENO_BC_REFLECT && p->nx == 1) ||
      (p->dim == 2 && p->bc_y == HWENO_BC_REFLECT && p->ny == 1))
    return fail(HWENO_ERR_INVALID_ARG, "a reflecting wall needs at least 2 cells across");
  if (p->limiter_characteristic != 0 && p->limiter_characteristic != 1)
    return fail(HWENO_ERR_INVALID_ARG, "limiter_characteristic must be 0 or 1");
  if (!(p->dx > 0.0) || !std::isfinite(p->dx)) return fail(HWENO_ERR_INVALID_ARG, "dx must be > 0");
  if (p->dim == 2 && (!(p->dy > 0.0) || !std::isfinite(p->dy)))
    return fail(HWENO_ERR_INVALID_ARG, "dy must be > 0");
  if (!weights_ok(p->lin_w))
    return fail(HWENO_ERR_INVALID_ARG, "linear weights gamma must be > 0 and sum to 1 (got %.17g %.17g %.17g)",
                p->lin_w[0], p->lin_w[1], p->lin_w[2]);
  if (!weights_ok(p->lim_w))
    return fail(HWENO_ERR_INVALID_ARG, "limiter weights d must be > 0 and sum to 1 (got %.17g %.17g %.17g)",
                p->lim_w[0], p->lim_w[1], p->lim_w[2]);
  if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return fail(HWENO_ERR_INVALID_ARG, "eps must be > 0");
  if (!(p->cfl > 0.0) || !std::isfinite(p->cfl)) return fail(HWENO_ERR_INVALID_ARG, "cfl must be > 0");
  if (p->physics == HWENO_EULER && (!(p->gamma_gas > 1.0) || !std::isfinite(p->gamma_gas)))
    return fail(HWENO_ERR_INVALID_ARG, "gamma_gas must be > 1");
  if (p->physics == HWENO_LINADV &&
      (!std::isfinite(p->adv_speed[0]) || !std::isfinite(p->adv_speed[1])))
    return fail(HWENO_ERR_INVALID_ARG, "advection speeds must be finite");
  const double cells = (double)p->nx * (double)(p->dim == 2 ? p->ny : 1);
  if (cells * n_fields(p) > 9.0e18 / 8.0) return fail(HWENO_ERR_INVALID_ARG, "grid too large");
  if (p->nx > (1 << 28) || p->ny > (1 << 28)) return fail(HWENO_ERR_INVALID_ARG, "grid side too large");
  return ok();
}

bool empty(const hweno_problem* p) { return p->nx == 0 || (p->dim == 2 && p->ny == 0); }

long long cells_of(const hweno_problem* p) {
  return (long long)p->nx * (p->dim == 2 ? p->ny : 1);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct WsLayout {
  size_t ctrl, s1, s2, base, total;
};

WsLayout ws_layout(const hweno_problem* p) {
  WsLayout L;
  const size_t fb = (size_t)cells_of(p) * elem_size(p);
  L.ctrl = 0;
  L.s1 = align256(HWENO_CTRL_LEN * sizeof(double));
  L.s2 = L.s1 + align256(fb * n_fields(p));
  L.base = L.s2 + align256(fb * n_fields(p));
  L.total = L.base + align256(fb * n_comp(p) * p->dim);
  return L;
}

template <typename T>
Consts<T> make_consts(const hweno_problem* p) {
  Consts<T> k;
  k.rw = {T(p->lin_w[0]), T(p->lin_w[1]), T(p->lin_w[2]), T(p->eps),
          T(p->lin_w[0]) + T(p->lin_w[1]) + T(p->lin_w[2])};
  k.lw = {T(p->lim_w[0]), T(p->lim_w[1]), T(p->lim_w[2]), T(p->eps),
          T(p->lim_w[0]) + T(p->lim_w[1]) + T(p->lim_w[2])};
  k.gm1 = T(p->gamma_gas - 1.0);
  k.gam = T(p->gamma_gas);
  k.ax = T(p->adv_speed[0]);
  k.ay = T(p->adv_speed[1]);
  k.characteristic = p->characteristic ? 1 : 0;
  k.limiter_on = p->limiter_on ? 1 : 0;
  k.limiter_char = p->limiter_characteristic ? 1 : 0;
  return k;
}

// the characteristic limiter variant is in force (Euler with the limiter on)
bool char_limiter(const hweno_problem* p) {
  return p->physics == HWENO_EULER && p->limiter_on && p->limiter_characteristic;
}

hweno_status launch_check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(HWENO_ERR_LAUNCH, "%s: %s", what, hipGetErrorString(e));
  return HWENO_OK;
}

// 2D tile: 16 x 15 cells on 256 threads gives 255 x-interfaces and 256
// y-interfaces, i.e. one balanced pass per direction.  1D tile: 255 cells have
// 256 interfaces, one per thread (with 256 cells the first wave took a second
// pass for the 257th, doubling the stage's critical path on small grids).
template <int DIM>
struct Tile {
  static constexpr int TX = (DIM == 2) ? 16 : 255;
  static constexpr int TY = (DIM == 2) ? 15 : 1;
  static constexpr int NT = 256;
};

// dispatch helper: calls F::template run<T, PHYS, DIM>(args...)
template <typename F, typename... Args>
hweno_status dispatch(const hweno_problem* p, Args&&... args) {
#define HWENO_CASE(TT, PH, D)                                                  \
  if (p->dtype == (sizeof(TT) == 8 ? HWENO_F64 : HWENO_F32) && p->physics == PH && \
      p->dim == D)                                                             \
    return F::template run<TT, PH, D>(p, args...);
  HWENO_CASE(double, HWENO_LINADV, 1)
  HWENO_CASE(double, HWENO_BURGERS, 1)
  HWENO_CASE(double, HWENO_EULER, 1)
  HWENO_CASE(double, HWENO_LINADV, 2)
  HWENO_CASE(double, HWENO_BURGERS, 2)
  HWENO_CASE(double, HWENO_EULER, 2)
  HWENO_CASE(float, HWENO_LINADV, 1)
  HWENO_CASE(float, HWENO_BURGERS, 1)
  HWENO_CASE(float, HWENO_EULER, 1)
  HWENO_CASE(float, HWENO_LINADV, 2)
  HWENO_CASE(float, HWENO_BURGERS, 2)
  HWENO_CASE(float, HWENO_EULER, 2)
#undef HWENO_CASE
  return fail(HWENO_ERR_UNSUPPORTED, "unsupported combination");
}

EdgeArgs edge_args(const hweno_problem* p) {
  EdgeArgs e;
  std::memset(&e, 0, sizeof e);
  for (int side = 0; side < 4; ++side) {
    const hweno_edge& h = p->edges[side];
    for (int sg = 0; sg < 2; ++sg) {
      e.kind[side][sg] = h.kind[sg];
      for (int c = 0; c < 4; ++c) e.state[side][sg][c] = h.state[sg][c];
    }
    e.mirror[side] = h.kind[0] == HWENO_SEG_REFLECT || h.kind[1] == HWENO_SEG_REFLECT;
    for (int q = 0; q < 3; ++q) e.split[side][q] = h.split[q];
  }
  e.t0 = 0.0;
  e.oi = p->obstacle[0];
  e.oj = p->obstacle[1];
  return e;
}

template <typename T, int PHYS, int DIM>
StageArgs<T> base_args(const hweno_problem* p) {
  StageArgs<T> a;
  std::memset(&a, 0, sizeof a);
  a.nx = p->nx;
  a.ny = DIM == 2 ? p->ny : 1;
  a.bc_x = p->bc_x;
  a.bc_y = p->bc_y;
  a.fs = cells_of(p);
  a.dx = p->dx;
  a.dy = DIM == 2 ? p->dy : 1.0;
  a.cfl = p->cfl;
  return a;
}

dim3 stage_grid(int dim, int nx, int ny) {
  if (dim == 2)
    return dim3(((nx + Tile<2>::TX - 1) / Tile<2>::TX) * ((ny + Tile<2>::TY - 1) / Tile<2>::TY));
  return dim3((nx + Tile<1>::TX - 1) / Tile<1>::TX);
}

// eight cells per thread: every workgroup ends in one atomic max on the same
// two words, and at small grids a thousand workgroups finishing together
// serialise there (512^2: 24 us with one cell per thread, 11 us with eight)
unsigned alpha_blocks(long long n) {
  long long b = (n + 2047) / 2048;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (unsigned)b;
}

struct RunAlpha {
  template <typename T, int PHYS, int DIM>
  static hweno_status run(const hweno_problem* p, const void* state, double* alpha,
                          unsigned long long* status, hipStream_t s) {
    const long long n = cells_of(p);
    k_zero<<<1, 64, 0, s>>>(alpha, 2);
    if constexpr (PHYS == PH_EULER && DIM == 2) {
      if (p->obstacle[1] > 0) {
        k_alpha_obstacle<T><<<alpha_blocks(n), 256, 0, s>>>(
            (const T*)state, p->nx, p->ny, p->obstacle[0], p->obstacle[1], make_consts<T>(p),
            alpha, status);
        return launch_check("alpha");
      }
    }
    k_alpha<T, PHYS, DIM><<<alpha_blocks(n), 256, 0, s>>>((const T*)state, n,
                                                          make_consts<T>(p), alpha, status);
    return launch_check("alpha");
  }
};

struct RunRhs {
  template <typename T, int PHYS, int DIM>
  static hweno_status run(const hweno_problem* p, const void* state, void* rhs,
                          double* alpha, int compute, hipStream_t s) {
    if (compute) {
      hweno_status st = RunAlpha::run<T, PHYS, DIM>(p, state, alpha, nullptr, s);
      if (st) return st;
    }
    StageArgs<T> a = base_args<T, PHYS, DIM>(p);
    a.in = (const T*)state;
    a.out = (T*)rhs;
    a.alpha = alpha;
    constexpr int TX = Tile<DIM>::TX, TY = Tile<DIM>::TY, NT = Tile<DIM>::NT;
    if constexpr (PHYS == PH_EULER && DIM == 2) {
      if (has_edges(p)) {
        k_stage_edges<T, 0, TX, TY, NT, false><<<stage_grid(DIM, a.nx, a.ny), NT, 0, s>>>(
            a, make_consts<T>(p), edge_args(p));
        return launch_check("rhs");
      }
    }
    k_stage<T, PHYS, DIM, 0, TX, TY, NT, false><<<stage_grid(DIM, a.nx, a.ny), NT, 0, s>>>(
        a, make_consts<T>(p));
    return launch_check("rhs");
  }
};

struct RunLimit {
  template <typename T, int PHYS, int DIM>
  static hweno_status run(const hweno_problem* p, const void* state, void* out, hipStream_t s) {
    const long long n = cells_of(p);
    const unsigned blocks = (unsigned)((n + 255) / 256);
    k_limit<T, PHYS, DIM><<<blocks, 256, 0, s>>>((const T*)state, (T*)out, p->nx,
                                                 DIM == 2 ? p->ny : 1, p->bc_x, p->bc_y,
                                                 p->dx, DIM == 2 ? p->dy : 1.0,
                                                 make_consts<T>(p), edge_args(p));
    return launch_check("limit");
  }
};

// where one step keeps its control block, its two stage states and the
// limited base derivatives
struct StepBufs {
  double* ctrl;
  void* s1;
  void* s2;
  void* base;
};

StepBufs ws_bufs(const hweno_problem* p, void* ws) {
  const WsLayout L = ws_layout(p);
  char* w = (char*)ws;
  return StepBufs{(double*)(w + L.ctrl), w + L.s1, w + L.s2, w + L.base};
}

struct RunStep {
  template <typename T, int PHYS, int DIM>
  // take_next: stage-1 speeds come from the previous step's stage 3 (the state
  // has not changed since); fold_next: this step's stage 3 provides them
  // (multi-step calls: the previous step's k_finish already began this one when
  // take_next, and this one's k_finish begins the next when fold_next).
  // may_time: stage launches may be bracketed by the diagnostic timer's events
  static hweno_status run(const hweno_problem* p, void* state, StepBufs b, double dt_fixed,
                          double t_end, double* tape, const double* replay, bool take_next,
                          bool fold_next, bool may_time, hipStream_t s) {
    double* ctrl = b.ctrl;
    auto timed = [&](hipStream_t st, auto&& launch) {
      if (may_time)
        ::timed(st, launch);
      else
        launch();
    };
    const long long n = cells_of(p);
    const Consts<T> k = make_consts<T>(p);
    if (!(take_next && !replay)) k_begin<<<1, 64, 0, s>>>(ctrl, replay);
    if (!replay && !take_next) {
      bool done = false;
      if constexpr (PHYS == PH_EULER && DIM == 2) {
        if (p->obstacle[1] > 0) {
          k_alpha_obstacle<T><<<alpha_blocks(n), 256, 0, s>>>(
              (const T*)state, p->nx, p->ny, p->obstacle[0], p->obstacle[1], k, ctrl,
              (unsigned long long*)(ctrl + 8));
          done = true;
        }
      }
      if (!done)
        k_alpha<T, PHYS, DIM><<<alpha_blocks(n), 256, 0, s>>>(
            (const T*)state, n, k, ctrl, (unsigned long long*)(ctrl + 8));
    }
    StageArgs<T> a = base_args<T, PHYS, DIM>(p);
    a.ctrl = ctrl;
    a.status = (unsigned long long*)(ctrl + 8);
    a.st0 = (const T*)state;
    a.base = (T*)b.base;
    a.dt_fixed = dt_fixed;
    a.t_end = t_end;
    a.replay = replay ? 1 : 0;
    a.fold_next = (fold_next && !replay) ? 1 : 0;
    T* s1 = (T*)b.s1;
    T* s2 = (T*)b.s2;
    constexpr int TX = Tile<DIM>::TX, TY = Tile<DIM>::TY, NT = Tile<DIM>::NT;
    const dim3 grid = stage_grid(DIM, a.nx, a.ny);
    auto stages = [&](auto cl) {
      constexpr bool CL = decltype(cl)::value;
      a.in = (const T*)state;
      a.out = s1;
      timed(s, [&] { k_stage<T, PHYS, DIM, 1, TX, TY, NT, CL><<<grid, NT, 0, s>>>(a, k); });
      a.in = s1;
      a.out = s2;
      timed(s, [&] { k_stage<T, PHYS, DIM, 2, TX, TY, NT, CL><<<grid, NT, 0, s>>>(a, k); });
      a.in = s2;
      a.out = (T*)state;
      timed(s, [&] { k_stage<T, PHYS, DIM, 3, TX, TY, NT, CL><<<grid, NT, 0, s>>>(a, k); });
    };
    if constexpr (PHYS == PH_EULER) {
      if constexpr (DIM == 2) {
        if (has_edges(p)) {
          const EdgeArgs e = edge_args(p);
          auto edge_stages = [&](auto cl) {
            constexpr bool CLE = decltype(cl)::value;
            a.in = (const T*)state;
            a.out = s1;
            timed(s, [&] { k_stage_edges<T, 1, TX, TY, NT, CLE><<<grid, NT, 0, s>>>(a, k, e); });
            a.in = s1;
            a.out = s2;
            timed(s, [&] { k_stage_edges<T, 2, TX, TY, NT, CLE><<<grid, NT, 0, s>>>(a, k, e); });
            a.in = s2;
            a.out = (T*)state;
            timed(s, [&] { k_stage_edges<T, 3, TX, TY, NT, CLE><<<grid, NT, 0, s>>>(a, k, e); });
          };
          if (char_limiter(p))
            edge_stages(std::true_type{});
          else
            edge_stages(std::false_type{});
          k_finish<<<1, 64, 0, s>>>(ctrl, tape, fold_next && !replay ? 1 : 0);
          return launch_check("rk3_step");
        }
      }
      if (char_limiter(p))
        stages(std::true_type{});
      else
        stages(std::false_type{});
    } else {
      stages(std::false_type{});
    }
    k_finish<<<1, 64, 0, s>>>(ctrl, tape, fold_next && !replay ? 1 : 0);
    return launch_check("rk3_step");
  }
};

// 2D adjoint tile: 15 x 14 cells, so the 18 x 14 x-interfaces and the
// 15 x 17 y-interfaces touching it each fit one pass of 256 threads
template <int DIM>
struct AdjTile {
  static constexpr int TX = (DIM == 2) ? 15 : 253;
  static constexpr int TY = (DIM == 2) ? 14 : 1;
  static constexpr int NT = 256;
};

struct AdjLayout {
  size_t e, y2, y1, l0, total;
  int nxe, nye;
};

AdjLayout adj_layout(const hweno_problem* p) {
  AdjLayout L;
  L.nxe = p->nx + 4;
  L.nye = p->dim == 2 ? p->ny + 4 : 1;
  const size_t es = elem_size(p);
  const size_t st = (size_t)cells_of(p) * es * n_fields(p);
  L.e = 0;
  L.y2 = align256((size_t)L.nxe * L.nye * es * n_fields(p));
  L.y1 = L.y2 + align256(st);
  L.l0 = L.y1 + align256(st);
  L.total = L.l0 + align256(st);
  return L;
}

// one adjoint evaluation into E followed by one fold
struct RunAdj {
  template <typename T, int PHYS, int DIM>
  // fuse: finish interior cells inside the adjoint kernel (the fold's output
  // buffers must then not alias S, XL or XM)
  static hweno_status run(const hweno_problem* p, const void* S, const void* XL, double cr,
                          const double* dtp, const void* XM, double cl, const double* alpha,
                          void* ws, FoldArgs<T> fo, bool fuse, hipStream_t s) {
    const AdjLayout L = adj_layout(p);
    AdjArgs<T> a;
    a.S = (const T*)S;
    a.XL = (const T*)XL;
    a.XM = (const T*)XM;
    a.E = (T*)((char*)ws + L.e);
    a.alpha = alpha;
    a.dtp = dtp;
    a.cr = cr;
    a.cl = cl;
    a.nx = p->nx;
    a.ny = DIM == 2 ? p->ny : 1;
    a.bc_x = p->bc_x;
    a.bc_y = p->bc_y;
    a.fs = cells_of(p);
    a.nxe = L.nxe;
    a.nye = L.nye;
    a.dx = p->dx;
    a.dy = DIM == 2 ? p->dy : 1.0;
    fo.E = a.E;
    fo.nxe = L.nxe;
    fo.nye = L.nye;
    fo.nx = a.nx;
    fo.ny = a.ny;
    fo.bc_x = p->bc_x;
    fo.bc_y = p->bc_y;
    fo.dim = DIM;
    fo.nf = Comps<PHYS, DIM>::NF;
    fo.m = Comps<PHYS, DIM>::M;
    fo.euler = PHYS == PH_EULER;
    fo.fs = a.fs;
    a.fused = (fuse && DIM == 2 && a.nx >= 4 && a.ny >= 4) ? 1 : 0;
    a.fo = fo;
    constexpr int TX = AdjTile<DIM>::TX, TY = AdjTile<DIM>::TY, NT = AdjTile<DIM>::NT;
    const unsigned tiles = (unsigned)(((L.nxe + TX - 1) / TX) * ((L.nye + TY - 1) / TY));
    if constexpr (PHYS == PH_EULER) {
      if (char_limiter(p))
        timed(s, [&] { k_adjoint<T, PHYS, DIM, TX, TY, NT, true><<<tiles, NT, 0, s>>>(a, make_consts<T>(p)); });
      else
        timed(s, [&] { k_adjoint<T, PHYS, DIM, TX, TY, NT, false><<<tiles, NT, 0, s>>>(a, make_consts<T>(p)); });
    } else {
      timed(s, [&] { k_adjoint<T, PHYS, DIM, TX, TY, NT, false><<<tiles, NT, 0, s>>>(a, make_consts<T>(p)); });
    }
    if (a.fused) {
      const long long nb = (4ll * a.ny + 4ll * (a.nx - 4)) * fo.nf;
      k_fold_band<T><<<(unsigned)((nb + 255) / 256), 256, 0, s>>>(fo);
    } else {
      k_fold<T><<<(unsigned)((a.fs * fo.nf + 255) / 256), 256, 0, s>>>(fo);
    }
    return launch_check("adjoint");
  }
};

template <typename T>
FoldArgs<T> fold_args(void* out, int accumulate, const void* XU, double cu, int identity_all) {
  FoldArgs<T> f;
  std::memset(&f, 0, sizeof f);
  f.out = (T*)out;
  f.accumulate = accumulate;
  f.XU = (const T*)XU;
  f.cu = cu;
  f.identity_all = identity_all;
  return f;
}

struct RunRhsAdj {
  template <typename T, int PHYS, int DIM>
  static hweno_status run(const hweno_problem* p, const void* state, const double* alpha,
                          const void* lam_rhs, const void* lam_lim, void* lam_state, void* ws,
                          hipStream_t s) {
    // the caller's buffers may alias: fold in a separate pass
    return RunAdj::run<T, PHYS, DIM>(p, state, lam_rhs, 1.0, nullptr, lam_lim, 1.0, alpha, ws,
                                     fold_args<T>(lam_state, 1, nullptr, 0.0, 0), false, s);
  }
};

struct RunStepAdj {
  template <typename T, int PHYS, int DIM>
  static hweno_status run(const hweno_problem* p, const void* state0, const void* step_ws,
                          const double* tape, void* lam, void* ws, hipStream_t s) {
    const WsLayout F = ws_layout(p);
    const AdjLayout L = adj_layout(p);
    const char* sw = (const char*)step_ws;
    const void* S1 = sw + F.s1;
    const void* S2 = sw + F.s2;
    char* w = (char*)ws;
    T* Y2 = (T*)(w + L.y2);
    T* Y1 = (T*)(w + L.y1);
    T* L0 = (T*)(w + L.l0);
    const bool lim = p->limiter_on != 0;
    const long long mN = (long long)n_comp(p) * cells_of(p);
    const int ida = lim ? 0 : 1;
    hweno_status st;
    // stage 3: S^{n+1} = 1/3 S^0 + 2/3 (S^2 + dt L(S2)),  S^ = (U, Lim(S))
    // (each stage's fold writes a buffer its adjoint kernel does not read: fused)
    st = RunAdj::run<T, PHYS, DIM>(p, S2, lam, 2.0 / 3.0, tape + 6,
                                   lim ? (const T*)lam + mN : nullptr, 2.0 / 3.0, tape + 4, ws,
                                   fold_args<T>(Y2, 0, lam, 2.0 / 3.0, ida), true, s);
    if (st) return st;
    // stage 2: S2 = 3/4 S^0 + 1/4 (S^1 + dt L(S1));  L0 = lam/3 + 3/4 Y2 + Y1
    FoldArgs<T> f2 = fold_args<T>(Y1, 0, Y2, 0.25, ida);
    f2.L0 = L0;
    f2.A = (const T*)lam;
    f2.B = Y2;
    f2.ca = 1.0 / 3.0;
    f2.cb = 0.75;
    st = RunAdj::run<T, PHYS, DIM>(p, S1, Y2, 0.25, tape + 6, lim ? Y2 + mN : nullptr, 0.25,
                                   tape + 2, ws, f2, true, s);
    if (st) return st;
    // stage 1: S1 = S^0 + dt L(S0); the base S^0 collects L0
    return RunAdj::run<T, PHYS, DIM>(p, state0, Y1, 1.0, tape + 6, lim ? L0 + mN : nullptr, 1.0,
                                     tape + 0, ws, fold_args<T>(lam, 0, L0, 1.0, ida), true, s);
  }
};

int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
  }
  return cus;
}

template <int V>
int tiles_of(int nx, int ny) {
  return ((nx + BatchTile<V>::TX - 1) / BatchTile<V>::TX) *
         ((ny + BatchTile<V>::TY - 1) / BatchTile<V>::TY);
}

// workgroups of one batched stage launch: `blocks`, or (0) exactly the
// workgroups that can be resident at once, never more than the tiles
template <typename T, int V>
int batched_grid(int blocks, int total) {
  int grid = blocks;
  if (grid <= 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_stage_batched<T, V, 1, false, false>, 256, 0) !=
            hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    grid = per_cu * device_cus();
  }
  return std::min(grid, total);
}

template <typename T, int V>
hweno_status run_batched(const hweno_problem* p, const hweno_instance* inst, const int* map, int n,
                         int total, int blocks, hipStream_t s) {
  const Consts<T> k = make_consts<T>(p);
  const int grid = batched_grid<T, V>(blocks, total);
  const unsigned small = (unsigned)((n + 255) / 256);
  k_begin_batched<<<small, 256, 0, s>>>(inst, n);
  k_alpha_batched<T, V><<<std::min(total, 4 * device_cus()), 256, 0, s>>>(inst, map, total, k);
  auto stages = [&](auto one, auto cl) {
    constexpr bool ONE = decltype(one)::value, CL = decltype(cl)::value;
    timed(s, [&] { k_stage_batched<T, V, 1, ONE, CL><<<grid, 256, 0, s>>>(inst, map, total, p->cfl, k); });
    timed(s, [&] { k_stage_batched<T, V, 2, ONE, CL><<<grid, 256, 0, s>>>(inst, map, total, p->cfl, k); });
    timed(s, [&] { k_stage_batched<T, V, 3, ONE, CL><<<grid, 256, 0, s>>>(inst, map, total, p->cfl, k); });
  };
  const bool cl = char_limiter(p);
  if (grid == total) {
    if (cl)
      stages(std::true_type{}, std::true_type{});
    else
      stages(std::true_type{}, std::false_type{});
  } else {
    if (cl)
      stages(std::false_type{}, std::true_type{});
    else
      stages(std::false_type{}, std::false_type{});
  }
  k_finish_batched<<<small, 256, 0, s>>>(inst, n);
  return launch_check("rk3_step_batched");
}

hweno_status run_batched_any(const hweno_problem* p, const hweno_instance* inst, const int* map,
                             int n, int total, int variant, int blocks, hipStream_t s) {
  if (p->dtype == HWENO_F64)
    return variant == 0 ? run_batched<double, 0>(p, inst, map, n, total, blocks, s)
                        : run_batched<double, 1>(p, inst, map, n, total, blocks, s);
  return variant == 0 ? run_batched<float, 0>(p, inst, map, n, total, blocks, s)
                      : run_batched<float, 1>(p, inst, map, n, total, blocks, s);
}

int batched_grid_any(const hweno_problem* p, int variant, int blocks, int total) {
  if (p->dtype == HWENO_F64)
    return variant == 0 ? batched_grid<double, 0>(blocks, total) : batched_grid<double, 1>(blocks, total);
  return variant == 0 ? batched_grid<float, 0>(blocks, total) : batched_grid<float, 1>(blocks, total);
}

// the autotuner's grid-size candidates for one tile variant: the resident
// capacity (0), two and four workgroups per compute unit, one per tile
void autotune_candidates(int total, int out[HWENO_AUTOTUNE_CANDIDATES]) {
  const int cus = device_cus();
  out[0] = 0;
  out[1] = 2 * cus;
  out[2] = 4 * cus;
  out[3] = total;
}

// timing of the autotuner's steps: two events, destroyed on every path
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

hweno_status batch_common_ok(const hweno_problem* common) {
  if (!common) return fail(HWENO_ERR_INVALID_ARG, "problem pointer is NULL");
  if (common->dim != 2 || common->physics != HWENO_EULER)
    return fail(HWENO_ERR_UNSUPPORTED, "batched stepping is built for 2D Euler only");
  if (has_edges(common))
    return fail(HWENO_ERR_UNSUPPORTED, "batched stepping has no edge-described sides");
  hweno_problem q = *common;
  if (q.nx < 1) q.nx = 1;
  if (q.ny < 1) q.ny = 1;
  return validate(&q);
}

// device address of `scratch` on every device, looked up once per device
// with that device current (each device holds its own copy of the array)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hweno_status static_scratch(hipStream_t s, void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(HWENO_ERR_LAUNCH, "hipGetDevice: %s", hipGetErrorString(e));
  if (s) {
    hipDevice_t sdev = -1;
    e = hipStreamGetDevice(s, &sdev);
    if (e != hipSuccess) return fail(HWENO_ERR_LAUNCH, "hipStreamGetDevice: %s", hipGetErrorString(e));
    if ((int)sdev != dev)
      return fail(HWENO_ERR_INVALID_ARG, "the stream belongs to device %d but device %d is current",
                  (int)sdev, dev);
  }
  if (dev < 0 || dev >= kMaxDevices) return fail(HWENO_ERR_UNSUPPORTED, "device index %d", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(HWENO_ERR_LAUNCH, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HWENO_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

hweno_status hweno_validate(const hweno_problem* prob) { return validate(prob); }

size_t hweno_workspace_bytes(const hweno_problem* prob) {
  if (validate(prob) != HWENO_OK) return 0;
  return ws_layout(prob).total;
}

hweno_status hweno_alpha(const hweno_problem* prob, const void* state, double* alpha,
                         void* stream) {
  hweno_status st = validate(prob);
  if (st) return st;
  if (empty(prob)) return ok();
  if (!state || !alpha) return fail(HWENO_ERR_INVALID_ARG, "state and alpha must be non-NULL");
  st = dispatch<RunAlpha>(prob, state, alpha, (unsigned long long*)nullptr, (hipStream_t)stream);
  if (st) return st;
  return ok();
}

hweno_status hweno_rhs(const hweno_problem* prob, const void* state, void* rhs,
                       double* alpha, int32_t compute_alpha, void* stream) {
  hweno_status st = validate(prob);
  if (st) return st;
  if (empty(prob)) return ok();
  if (!state || !rhs || !alpha) return fail(HWENO_ERR_INVALID_ARG, "state, rhs and alpha must be non-NULL");
  if (state == rhs) return fail(HWENO_ERR_INVALID_ARG, "state and rhs must not alias");
  st = dispatch<RunRhs>(prob, state, rhs, alpha, (int)compute_alpha, (hipStream_t)stream);
  if (st) return st;
  return ok();
}

hweno_status hweno_limit(const hweno_problem* prob, const void* state, void* dlim,
                         void* stream) {
  hweno_status st = validate(prob);
  if (st) return st;
  if (empty(prob)) return ok();
  if (!state || !dlim) return fail(HWENO_ERR_INVALID_ARG, "state and dlim must be non-NULL");
  st = dispatch<RunLimit>(prob, state, dlim, (hipStream_t)stream);
  if (st) return st;
  return ok();
}

hweno_status hweno_rk3_step(const hweno_problem* prob, void* state, void* ws, size_t ws_bytes,
                            double dt_fixed, double t_end, double* tape, const double* replay,
                            void* stream) {
  hweno_status st = validate(prob);
  if (st) return st;
  if (empty(prob)) return ok();
  if (!state || !ws) return fail(HWENO_ERR_INVALID_ARG, "state and ws must be non-NULL");
  const size_t need = ws_layout(prob).total;
  if (ws_bytes < need)
    return fail(HWENO_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  if (((uintptr_t)ws & 255u) != 0) return fail(HWENO_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (!std::isfinite(dt_fixed) || !std::isfinite(t_end))
    return fail(HWENO_ERR_INVALID_ARG, "dt_fixed and t_end must be finite");
  st = dispatch<RunStep>(prob, state, ws_bufs(prob, ws), dt_fixed, t_end, tape, replay, false,
                         false, true, (hipStream_t)stream);
  if (st) return st;
  return ok();
}

hweno_status hweno_rk3_steps(const hweno_problem* prob, void* state, void* ws, size_t ws_bytes,
                             int32_t n_steps, double dt_fixed, double t_end, double* tapes,
                             void* stream) {
  hweno_status st = validate(prob);
  if (st) return st;
  if (n_steps < 0) return fail(HWENO_ERR_INVALID_ARG, "n_steps must be >= 0");
  if (empty(prob) || n_steps == 0) return ok();
  if (!state || !ws) return fail(HWENO_ERR_INVALID_ARG, "state and ws must be non-NULL");
  const size_t need = ws_layout(prob).total;
  if (ws_bytes < need)
    return fail(HWENO_ERR_WORKSPACE, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  if (((uintptr_t)ws & 255u) != 0) return fail(HWENO_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  if (!std::isfinite(dt_fixed) || !std::isfinite(t_end))
    return fail(HWENO_ERR_INVALID_ARG, "dt_fixed and t_end must be finite");
  for (int32_t q = 0; q < n_steps; ++q) {
    st = dispatch<RunStep>(prob, state, ws_bufs(prob, ws), dt_fixed, t_end,
                           tapes ? tapes + (size_t)q * HWENO_CTRL_LEN : (double*)nullptr,
                           (const double*)nullptr, q > 0, q + 1 < n_steps, true,
                           (hipStream_t)stream);
    if (st) return st;
  }
  return ok();
}

hweno_status hweno_rk3_step_static(const hweno_problem* prob, void* state, double* ctrl,
                                   double dt_fixed, double t_end, double* tape,
                                   const double* replay, void* stream) {
  hweno_status st = validate(prob);
  if (st) return st;
  if (empty(prob)) return ok();
  if (!state || !ctrl) return fail(HWENO_ERR_INVALID_ARG, "state and ctrl must be non-NULL");
  if (((uintptr_t)ctrl & 7u) != 0) return fail(HWENO_ERR_INVALID_ARG, "ctrl must be 8-byte aligned");
  if (!std::isfinite(dt_fixed) || !std::isfinite(t_end))
    return fail(HWENO_ERR_INVALID_ARG, "dt_fixed and t_end must be finite");
  // the stage states and base derivatives, laid out as in a workspace but
  // without its control block
  const WsLayout L = ws_layout(prob);
  const size_t need = L.total - L.s1;
  if (need > (size_t)HWENO_STATIC_SCRATCH_BYTES)
    return fail(HWENO_ERR_WORKSPACE,
                "grid too large for the static scratch: needs %zu bytes, the maximum is %zu",
                need, (size_t)HWENO_STATIC_SCRATCH_BYTES);
  void* base = nullptr;
  st = static_scratch((hipStream_t)stream, &base);
  if (st) return st;
  char* w = (char*)base;
  const StepBufs b{ctrl, w, w + (L.s2 - L.s1), w + (L.base - L.s1)};
  st = dispatch<RunStep>(prob, state, b, dt_fixed, t_end, tape, replay, false, false, false,
                         (hipStream_t)stream);
  if (st) return st;
  return ok();
}

size_t hweno_adjoint_workspace_bytes(const hweno_problem* prob) {
  if (validate(prob) != HWENO_OK || has_edges(prob)) return 0;
  return adj_layout(prob).total;
}

hweno_status hweno_rhs_adjoint(const hweno_problem* prob, const void* state, const double* alpha,
                               const void* lam_rhs, const void* lam_lim, void* lam_state, void* ws,
                               size_t ws_bytes, void* stream) {
  hweno_status st = validate(prob);
  if (st) return st;
  if (has_edges(prob)) return fail(HWENO_ERR_UNSUPPORTED, "the adjoint has no edge-described sides");
  if (empty(prob)) return ok();
  if (!state || !alpha || !lam_rhs || !lam_state || !ws)
    return fail(HWENO_ERR_INVALID_ARG, "state, alpha, lam_rhs, lam_state and ws must be non-NULL");
  if (ws_bytes < adj_layout(prob).total)
    return fail(HWENO_ERR_WORKSPACE, "adjoint workspace too small: %zu < %zu bytes", ws_bytes,
                adj_layout(prob).total);
  if (((uintptr_t)ws & 255u) != 0) return fail(HWENO_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  st = dispatch<RunRhsAdj>(prob, state, alpha, lam_rhs, lam_lim, lam_state, ws, (hipStream_t)stream);
  if (st) return st;
  return ok();
}

hweno_status hweno_rk3_step_adjoint(const hweno_problem* prob, const void* state0,
                                    const void* step_ws, size_t step_ws_bytes, const double* tape,
                                    void* lam, void* ws, size_t ws_bytes, void* stream) {
  hweno_status st = validate(prob);
  if (st) return st;
  if (has_edges(prob)) return fail(HWENO_ERR_UNSUPPORTED, "the adjoint has no edge-described sides");
  if (empty(prob)) return ok();
  if (!state0 || !step_ws || !tape || !lam || !ws)
    return fail(HWENO_ERR_INVALID_ARG, "state0, step_ws, tape, lam and ws must be non-NULL");
  if (step_ws_bytes < ws_layout(prob).total)
    return fail(HWENO_ERR_WORKSPACE, "step workspace too small");
  if (ws_bytes < adj_layout(prob).total)
    return fail(HWENO_ERR_WORKSPACE, "adjoint workspace too small: %zu < %zu bytes", ws_bytes,
                adj_layout(prob).total);
  if (((uintptr_t)ws & 255u) != 0 || ((uintptr_t)step_ws & 255u) != 0)
    return fail(HWENO_ERR_WORKSPACE, "workspaces must be 256-byte aligned");
  {
    // the stage adjoints read state0, step_ws and lam while writing lam and ws
    const size_t sb = (size_t)cells_of(prob) * elem_size(prob) * n_fields(prob);
    auto overlap = [](const void* a, size_t na, const void* b, size_t nb) {
      const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
      return x < y + nb && y < x + na;
    };
    if (overlap(lam, sb, state0, sb) || overlap(lam, sb, step_ws, step_ws_bytes) ||
        overlap(lam, sb, ws, ws_bytes) || overlap(ws, ws_bytes, state0, sb) ||
        overlap(ws, ws_bytes, step_ws, step_ws_bytes))
      return fail(HWENO_ERR_INVALID_ARG, "lam, state0, step_ws and ws must not overlap");
  }
  st = dispatch<RunStepAdj>(prob, state0, step_ws, tape, lam, ws, (hipStream_t)stream);
  if (st) return st;
  return ok();
}

hweno_status hweno_batch_prepare(const hweno_problem* common, hweno_instance* inst,
                                 int32_t n_inst, int32_t* total_tiles) {
  hweno_status st = batch_common_ok(common);
  if (st) return st;
  if (!inst || !total_tiles || n_inst < 1)
    return fail(HWENO_ERR_INVALID_ARG, "inst, total_tiles must be non-NULL and n_inst >= 1");
  long long tot[HWENO_BATCH_VARIANTS] = {0, 0};
  for (int q = 0; q < n_inst; ++q) {
    hweno_instance& I = inst[q];
    hweno_problem p = *common;
    p.nx = I.nx;
    p.ny = I.ny;
    p.bc_x = I.bc_x;
    p.bc_y = I.bc_y;
    p.dx = I.dx;
    p.dy = I.dy;
    if (has_edges(&p))
      return fail(HWENO_ERR_UNSUPPORTED, "instance %d: batched stepping has no edge-described sides", q);
    st = validate(&p);
    if (st) return fail(st, "instance %d: %s", q, g_last_error.c_str());
    if (I.nx < 1 || I.ny < 1) return fail(HWENO_ERR_INVALID_ARG, "instance %d: nx, ny must be >= 1", q);
    if (!std::isfinite(I.dt_fixed) || !std::isfinite(I.t_end))
      return fail(HWENO_ERR_INVALID_ARG, "instance %d: dt_fixed, t_end must be finite", q);
    const WsLayout L = ws_layout(&p);
    I.ws_bytes = (int64_t)L.total;
    I.off_s1 = (int64_t)L.s1;
    I.off_s2 = (int64_t)L.s2;
    I.off_base = (int64_t)L.base;
    const int nt[HWENO_BATCH_VARIANTS] = {tiles_of<0>(I.nx, I.ny), tiles_of<1>(I.nx, I.ny)};
    for (int v = 0; v < HWENO_BATCH_VARIANTS; ++v) {
      I.tile_begin[v] = (int32_t)tot[v];
      I.n_tiles[v] = nt[v];
      tot[v] += nt[v];
      if (tot[v] > (1ll << 30)) return fail(HWENO_ERR_INVALID_ARG, "too many tiles");
    }
  }
  for (int v = 0; v < HWENO_BATCH_VARIANTS; ++v) total_tiles[v] = (int32_t)tot[v];
  return ok();
}

hweno_status hweno_batch_tile_map(const hweno_instance* inst, int32_t n_inst, int32_t variant,
                                  int32_t* map, int32_t total_tiles) {
  if (!inst || !map || n_inst < 1 || variant < 0 || variant >= HWENO_BATCH_VARIANTS)
    return fail(HWENO_ERR_INVALID_ARG, "inst, map must be non-NULL, n_inst >= 1, variant valid");
  long long filled = 0;
  for (int q = 0; q < n_inst; ++q) {
    const int b = inst[q].tile_begin[variant], n = inst[q].n_tiles[variant];
    if (b != filled || n < 1 || (long long)b + n > total_tiles)
      return fail(HWENO_ERR_INVALID_ARG, "instance %d: descriptors not prepared for %d tiles", q,
                  total_tiles);
    for (int t = 0; t < n; ++t) map[b + t] = q;
    filled += n;
  }
  if (filled != total_tiles) return fail(HWENO_ERR_INVALID_ARG, "tile count mismatch");
  return ok();
}

hweno_status hweno_rk3_step_batched(const hweno_problem* common, const hweno_instance* inst_dev,
                                    const int32_t* tile_map_dev, int32_t n_inst,
                                    int32_t total_tiles, int32_t variant, int32_t blocks,
                                    void* stream) {
  hweno_status st = batch_common_ok(common);
  if (st) return st;
  if (!inst_dev || !tile_map_dev || n_inst < 1 || total_tiles < n_inst)
    return fail(HWENO_ERR_INVALID_ARG,
                "inst_dev, tile_map_dev must be non-NULL, n_inst >= 1, total_tiles >= n_inst");
  if (variant < 0 || variant >= HWENO_BATCH_VARIANTS)
    return fail(HWENO_ERR_INVALID_ARG, "variant must be in [0, %d)", HWENO_BATCH_VARIANTS);
  if (blocks < 0) return fail(HWENO_ERR_INVALID_ARG, "blocks must be >= 0");
  st = run_batched_any(common, inst_dev, tile_map_dev, n_inst, total_tiles, variant, blocks,
                       (hipStream_t)stream);
  if (st) return st;
  return ok();
}

hweno_status hweno_autotune(const hweno_problem* common, const hweno_instance* inst_dev,
                            const int32_t* const* tile_maps_dev, int32_t n_inst,
                            const int32_t* total_tiles, int32_t trials, void* stream,
                            int32_t* variant, int32_t* blocks, double* times_ms,
                            int32_t* grid_sizes) {
  hweno_status st = batch_common_ok(common);
  if (st) return st;
  if (!inst_dev || !tile_maps_dev || !total_tiles || !variant || !blocks || n_inst < 1)
    return fail(HWENO_ERR_INVALID_ARG,
                "inst_dev, tile_maps_dev, total_tiles, variant, blocks must be non-NULL, n_inst >= 1");
  if (trials < 1 || trials > 1000) return fail(HWENO_ERR_INVALID_ARG, "trials must be in [1, 1000]");
  for (int v = 0; v < HWENO_BATCH_VARIANTS; ++v) {
    if (!tile_maps_dev[v]) return fail(HWENO_ERR_INVALID_ARG, "tile map of variant %d is NULL", v);
    if (total_tiles[v] < n_inst)
      return fail(HWENO_ERR_INVALID_ARG, "variant %d: total_tiles must be >= n_inst", v);
  }
  hipStream_t s = (hipStream_t)stream;
  // the diagnostic stage timer must not see the autotuner's launches
  const bool timing_was_on = g_timing.on;
  g_timing.on = false;
  struct Restore {
    bool on;
    ~Restore() { g_timing.on = on; }
  } restore{timing_was_on};
  EventPair ev;
  hipError_t e = hipEventCreate(&ev.a);
  if (e == hipSuccess) e = hipEventCreate(&ev.b);
  if (e != hipSuccess) return fail(HWENO_ERR_LAUNCH, "hipEventCreate: %s", hipGetErrorString(e));
  double best = 0.0;
  int best_v = -1, best_b = 0;
  for (int v = 0; v < HWENO_BATCH_VARIANTS; ++v) {
    int cand[HWENO_AUTOTUNE_CANDIDATES];
    autotune_candidates(total_tiles[v], cand);
    for (int c = 0; c < HWENO_AUTOTUNE_CANDIDATES; ++c) {
      const int b = cand[c];
      // one warm-up step, then `trials` timed steps between two events
      st = run_batched_any(common, inst_dev, tile_maps_dev[v], n_inst, total_tiles[v], v, b, s);
      if (st) return st;
      if ((e = hipEventRecord(ev.a, s)) != hipSuccess)
        return fail(HWENO_ERR_LAUNCH, "hipEventRecord: %s", hipGetErrorString(e));
      for (int q = 0; q < trials; ++q) {
        st = run_batched_any(common, inst_dev, tile_maps_dev[v], n_inst, total_tiles[v], v, b, s);
        if (st) return st;
      }
      if ((e = hipEventRecord(ev.b, s)) != hipSuccess ||
          (e = hipEventSynchronize(ev.b)) != hipSuccess)
        return fail(HWENO_ERR_LAUNCH, "event: %s", hipGetErrorString(e));
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, ev.a, ev.b)) != hipSuccess)
        return fail(HWENO_ERR_LAUNCH, "hipEventElapsedTime: %s", hipGetErrorString(e));
      const double per = (double)ms / trials;
      const int k = v * HWENO_AUTOTUNE_CANDIDATES + c;
      if (times_ms) times_ms[k] = per;
      if (grid_sizes) grid_sizes[k] = batched_grid_any(common, v, b, total_tiles[v]);
      if (best_v < 0 || per < best) {
        best = per;
        best_v = v;
        best_b = b;
      }
    }
  }
  *variant = best_v;
  // the grid size itself (the resident capacity resolved), which launches the
  // same kernels as the candidate when passed back as `blocks`
  *blocks = batched_grid_any(common, best_v, best_b, total_tiles[best_v]);
  return ok();
}

hweno_status hweno_timing_begin(int32_t enable) {
  timing_release();
  g_timing.on = enable != 0;
  return ok();
}

hweno_status hweno_timing_end(int64_t* launches, double* total_ms) {
  double tot = 0.0;
  for (size_t q = 0; q < g_timing.used; ++q) {
    if (hipEventSynchronize(g_timing.ev[q].second) != hipSuccess) {
      timing_release();
      return fail(HWENO_ERR_LAUNCH, "event synchronisation failed");
    }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_timing.ev[q].first, g_timing.ev[q].second) != hipSuccess) {
      timing_release();
      return fail(HWENO_ERR_LAUNCH, "event timing failed");
    }
    tot += ms;
  }
  if (launches) *launches = (int64_t)g_timing.used;
  if (total_ms) *total_ms = tot;
  timing_release();
  return ok();
}

const char* hweno_status_string(int32_t s) {
  switch (s) {
    case HWENO_OK: return "HWENO_OK";
    case HWENO_ERR_INVALID_ARG: return "HWENO_ERR_INVALID_ARG";
    case HWENO_ERR_UNSUPPORTED: return "HWENO_ERR_UNSUPPORTED";
    case HWENO_ERR_WORKSPACE: return "HWENO_ERR_WORKSPACE";
    case HWENO_ERR_LAUNCH: return "HWENO_ERR_LAUNCH";
    default: return "HWENO_ERR_UNKNOWN";
  }
}

const char* hweno_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
