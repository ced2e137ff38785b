// mcv_reduce.hip -- powder reduction of detector data to I(Q, E) on gfx950.
//
// The reduction step of the simulation workflow (Sec. 3): intensities per
// (pixel, time-of-flight) bin, or detector events, are rebinned into
// momentum transfer |Q| and energy transfer E for a direct-geometry powder
// measurement, with the scattering taken at the sample position.  For a
// pixel centre r_p and a time t: v_f = |r_p| / t, E = E_i - m v_f^2 / 2,
// Q^2 = k_i^2 + k_f^2 - 2 k_i k_f cos(2theta), cos(2theta) = z_p / |r_p|.
//
// Histogram mode streams the histogram once (HBM bound).  Every lane walks
// runs of 4 consecutive bins (two 16-byte non-temporal loads; the next
// run's loads are issued before the current run is binned); a workgroup
// covers a contiguous range of the histogram, 1024 bins per step.
// Consecutive time bins of one pixel fall into the same (Q, E) bin for
// several steps, so a lane sums runs of equal destination bins (zero bins
// are skipped).  Neighbouring pixels of a tube see nearly the same
// scattering angle, so the runs of a workgroup's range land on one narrow
// band of the (Q, E) plane: runs go into a per-workgroup LDS cache of output
// bins (direct mapped, a slot claimed by compare-and-swap of its tag;
// binary64 LDS atomics), flushed with one global atomic per slot at the end;
// runs whose slot another bin holds go straight to global atomics.  Device-
// wide binary64 atomics are executed at the memory side, so the cache is
// what keeps the kernel near the bandwidth of its single read.  The pixel
// centres (distance, cos 2theta) come from a table the plan builds in
// binary64 and stores in binary32 (8 bytes per pixel, cache resident).
//
// Event mode reads 16-byte events and adds each into its bin.
//
// Q and E in binary32 (a few ulp; bins are 1e-3 to 1e-2 of the range), sums
// in binary64.

#include <hip/hip_runtime.h>

#include "mcv_internal.h"

namespace mcv {
namespace red {

typedef double dvec2 __attribute__((ext_vector_type(2)));

constexpr int kBlock = 256;
constexpr int kPerLane = 4;                  // consecutive bins per lane
constexpr int kTile = kBlock * kPerLane;     // bins per workgroup step
constexpr int kCache = 2048;                 // LDS output-bin cache slots

// adds (v, v2) for output bin b into the workgroup's cache, or into the
// output when another bin holds b's slot
template <bool W2>
__device__ __forceinline__ void put(double* cv, double* cw, int* ct, double* __restrict__ iqe,
                                    double* __restrict__ iqe_w2, int b, double v, double v2) {
  const int slot = b & (kCache - 1);
  int t = ct[slot];
  if (t < 0) {
    const int old = atomicCAS(&ct[slot], -1, b);
    t = old < 0 ? b : old;
  }
  if (t == b) {
    atomicAdd(&cv[slot], v);
    if (W2) atomicAdd(&cw[slot], v2);
  } else {
    unsafeAtomicAdd(iqe + b, v);
    if (W2) unsafeAtomicAdd(iqe_w2 + b, v2);
  }
}

typedef float fvec2 __attribute__((ext_vector_type(2)));

// centre of pixel `pid`: distance from the sample and cos(2theta)
__device__ __forceinline__ void pixel_geom(const float* __restrict__ geo, uint32_t pid, float& L2,
                                           float& c2t) {
  const fvec2 g = reinterpret_cast<const fvec2*>(geo)[pid];
  L2 = g.x;
  c2t = g.y;
}

// pixel of flat bin i (i < 2^53) and its time bin
__device__ __forceinline__ void pixel_of(uint64_t i, uint64_t ntof, double inv_ntof,
                                         uint32_t& pid, uint32_t& tb) {
  uint64_t p = (uint64_t)((double)i * inv_ntof);
  int64_t r = (int64_t)(i - p * ntof);
  if (r < 0) {
    --p;
    r += (int64_t)ntof;
  } else if (r >= (int64_t)ntof) {
    ++p;
    r -= (int64_t)ntof;
  }
  pid = (uint32_t)p;
  tb = (uint32_t)r;
}

// (Q, E) bin of a time t at a pixel, or -1 outside the grid
__device__ __forceinline__ int qe_bin(const QEMap& M, float L2, float c2t, float t) {
  const float vf = L2 / t;
  const float E = M.Ei - M.e_per_v2 * vf * vf;
  const float kf = M.k_per_v * vf;
  const float Q = sqrtf(fmaxf(M.ki2 + kf * (kf - M.two_ki * c2t), 0.0f));
  const float fq = (Q - M.q_lo) * M.q_scale;
  const float fe = (E - M.e_lo) * M.e_scale;
  if (!(fq >= 0.0f && fq < (float)M.nq && fe >= 0.0f && fe < (float)M.ne)) return -1;
  const int iq = min((int)fq, M.nq - 1);
  const int ie = min((int)fe, M.ne - 1);
  return iq * M.ne + ie;
}

// the kPerLane bins of run i0 (zeros past the end)
__device__ __forceinline__ void load_run(const double* __restrict__ h, uint64_t i0,
                                         uint64_t nbins, double* v) {
  if (i0 + kPerLane <= nbins) {
    const dvec2* p = reinterpret_cast<const dvec2*>(h + i0);
#pragma unroll
    for (int q = 0; q < kPerLane / 2; ++q) {
      const dvec2 x = __builtin_nontemporal_load(p + q);
      v[2 * q] = x.x;
      v[2 * q + 1] = x.y;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kPerLane; ++q) v[q] = i0 + q < nbins ? h[i0 + q] : 0.0;
  }
}

template <bool W2>
__global__ void __launch_bounds__(kBlock)
reduce_hist_qe(const float* __restrict__ geo, QEMap M,
               const double* __restrict__ hist, const double* __restrict__ hw2, uint64_t nbins,
               uint64_t tiles_per_block, double* __restrict__ iqe, double* __restrict__ iqe_w2) {
  __shared__ double cv[kCache];
  __shared__ double cw[W2 ? kCache : 1];
  __shared__ int ct[kCache];
  const int tid = threadIdx.x;
  for (int i = tid; i < kCache; i += kBlock) {
    cv[i] = 0.0;
    if (W2) cw[i] = 0.0;
    ct[i] = -1;
  }
  __syncthreads();
  const uint64_t ntof = (uint64_t)M.ntof;
  const double inv_ntof = 1.0 / (double)ntof;
  const uint64_t ntiles = (nbins + kTile - 1) / kTile;
  const uint64_t t0 = (uint64_t)blockIdx.x * tiles_per_block;
  const uint64_t t1 = t0 + tiles_per_block < ntiles ? t0 + tiles_per_block : ntiles;
  double nv[kPerLane], nw[kPerLane];
  uint64_t i0 = t0 * kTile + (uint64_t)tid * kPerLane;
  if (t0 < t1) {
    load_run(hist, i0, nbins, nv);
    if (W2) load_run(hw2, i0, nbins, nw);
  }
  for (uint64_t tile = t0; tile < t1; ++tile, i0 += kTile) {
    double v[kPerLane], w[kPerLane];
#pragma unroll
    for (int q = 0; q < kPerLane; ++q) {
      v[q] = nv[q];
      if (W2) w[q] = nw[q];
    }
    if (tile + 1 < t1) {  // the next run's loads overlap this run's binning
      load_run(hist, i0 + kTile, nbins, nv);
      if (W2) load_run(hw2, i0 + kTile, nbins, nw);
    }
    // runs of equal (Q, E) cells along this lane's bins: the middle ones are
    // put at once; the first (if the lane has more than one) and the last
    // wait, because a cell often spans the boundary between neighbouring
    // lanes (about 2.6 time bins per energy bin at the powder's grid): a lane
    // whose first cell is its left neighbour's last cell hands its first
    // partial sum to that lane, which puts both with one update
    int first_cell = -1, last_cell = -1, ncell = 0;
    double fa = 0.0, fa2 = 0.0, acc = 0.0, acc2 = 0.0;
    bool any = false;
    if (i0 < nbins) {
#pragma unroll
      for (int q = 0; q < kPerLane; ++q) any = any || v[q] != 0.0 || (W2 && w[q] != 0.0);
    }
    if (any) {
      uint32_t pid, tb;
      pixel_of(i0, ntof, inv_ntof, pid, tb);
      float L2, c2t;
      pixel_geom(geo, pid, L2, c2t);
      const int nk = nbins - i0 < (uint64_t)kPerLane ? (int)(nbins - i0) : kPerLane;
#pragma unroll
      for (int k = 0; k < kPerLane; ++k) {
        if (k >= nk) break;
        const double x = v[k];
        const double x2 = W2 ? w[k] : 0.0;
        if (x != 0.0 || x2 != 0.0) {
          const int dst = qe_bin(M, L2, c2t, M.tof_lo + ((float)tb + 0.5f) * M.dt);
          if (dst != last_cell) {
            if (ncell == 1) {
              first_cell = last_cell;
              fa = acc;
              fa2 = acc2;
            } else if (ncell > 1 && last_cell >= 0) {
              put<W2>(cv, cw, ct, iqe, iqe_w2, last_cell, acc, acc2);
            }
            last_cell = dst;
            acc = 0.0;
            acc2 = 0.0;
            ++ncell;
          }
          acc += x;
          if (W2) acc2 += x2;
        }
        if (++tb == (uint32_t)ntof) {
          tb = 0;
          ++pid;
          if (k + 1 < nk) pixel_geom(geo, pid, L2, c2t);
        }
      }
    }
    // whole wave: hand-over between neighbouring lanes (a wave of fewer
    // lanes, as in a host build, hands nothing over)
    const int nl = __popcll(__ballot(1));
    const int lane = (int)__lane_id();
    const int left_last = __shfl_up(last_cell, 1);
    const bool give = ncell > 1 && lane > 0 && first_cell >= 0 && left_last == first_cell;
    const int right_gives = __shfl_down(give ? 1 : 0, 1);
    const double got = __shfl_down(give ? fa : 0.0, 1);
    const double got2 = W2 ? __shfl_down(give ? fa2 : 0.0, 1) : 0.0;
    if (lane + 1 < nl && right_gives) {
      acc += got;
      if (W2) acc2 += got2;
    }
    if (ncell > 1 && !give && first_cell >= 0) put<W2>(cv, cw, ct, iqe, iqe_w2, first_cell, fa, fa2);
    if (last_cell >= 0) put<W2>(cv, cw, ct, iqe, iqe_w2, last_cell, acc, acc2);
  }
  __syncthreads();
  for (int i = tid; i < kCache; i += kBlock) {
    const int b = ct[i];
    if (b >= 0) {
      unsafeAtomicAdd(iqe + b, cv[i]);
      if (W2) unsafeAtomicAdd(iqe_w2 + b, cw[i]);
    }
  }
}

template <bool W2>
__global__ void __launch_bounds__(kBlock)
reduce_events_qe(const float* __restrict__ geo, QEMap M,
                 const DevEvent* __restrict__ ev, const unsigned long long* __restrict__ n_dev,
                 uint64_t cap, double* __restrict__ iqe, double* __restrict__ iqe_w2) {
  const uint64_t n = *n_dev < cap ? *n_dev : cap;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const DevEvent e = ev[i];
    if (e.pixel >= M.npixels) continue;
    float L2, c2t;
    pixel_geom(geo, e.pixel, L2, c2t);
    const int dst = qe_bin(M, L2, c2t, e.tof);
    if (dst >= 0) {
      unsafeAtomicAdd(iqe + dst, (double)e.value);
      if (W2) unsafeAtomicAdd(iqe_w2 + dst, (double)e.value * (double)e.value);
    }
  }
}

}  // namespace red

hipError_t launch_reduce_hist(const float* geo, const QEMap& M,
                              const double* hist, const double* hist_w2, uint64_t nbins,
                              double* iqe, double* iqe_w2, int grid, int cus,
                              hipStream_t stream) {
  // one round of resident workgroups, each with a contiguous range
  int per_cu = 0;
  const hipError_t oe =
      hist_w2 && iqe_w2
          ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, red::reduce_hist_qe<true>,
                                                         red::kBlock, 0)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, red::reduce_hist_qe<false>,
                                                         red::kBlock, 0);
  if (oe == hipSuccess && per_cu > 0) grid = cus * per_cu;
  const uint64_t ntiles = (nbins + red::kTile - 1) / red::kTile;
  const uint64_t per = (ntiles + grid - 1) / grid;
  grid = (int)((ntiles + per - 1) / per);
  if (hist_w2 && iqe_w2)
    hipLaunchKernelGGL(red::reduce_hist_qe<true>, dim3(grid), dim3(red::kBlock), 0, stream, geo,
                       M, hist, hist_w2, nbins, per, iqe, iqe_w2);
  else
    hipLaunchKernelGGL(red::reduce_hist_qe<false>, dim3(grid), dim3(red::kBlock), 0, stream,
                       geo, M, hist, nullptr, nbins, per, iqe, nullptr);
  return hipGetLastError();
}

hipError_t launch_reduce_events(const float* geo, const QEMap& M,
                                const DevEvent* ev, const unsigned long long* n_dev, uint64_t cap,
                                double* iqe, double* iqe_w2, int grid, hipStream_t stream) {
  if (iqe_w2)
    hipLaunchKernelGGL(red::reduce_events_qe<true>, dim3(grid), dim3(red::kBlock), 0, stream,
                       geo, M, ev, n_dev, cap, iqe, iqe_w2);
  else
    hipLaunchKernelGGL(red::reduce_events_qe<false>, dim3(grid), dim3(red::kBlock), 0, stream,
                       geo, M, ev, n_dev, cap, iqe, nullptr);
  return hipGetLastError();
}

int reduce_tile_bins() { return red::kTile; }

}  // namespace mcv
