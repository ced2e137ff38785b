// mcv_reduce.hip -- powder reduction of detector data to I(Q, E) on gfx950.
//
// The reduction step of the simulation workflow (Sec. 3): intensities per
// (pixel, time-of-flight) bin, or detector events, are rebinned into
// momentum transfer |Q| and energy transfer E for a direct-geometry powder
// measurement, with the scattering taken at the sample position.  For a
// pixel centre r_p and a time t: v_f = |r_p| / t, E = E_i - m v_f^2 / 2,
// Q^2 = k_i^2 + k_f^2 - 2 k_i k_f cos(2theta), cos(2theta) = z_p / |r_p|.
//
// Histogram mode streams the histogram once (HBM bound): a workgroup loads
// a tile of 2048 bins with coalesced 16-byte non-temporal loads into LDS,
// then every lane walks 8 consecutive bins of the tile.  Consecutive time
// bins of one pixel fall into the same (Q, E) bin for several steps, so a
// lane sums runs of equal destination bins and issues one binary64 atomic
// per run (zero bins are skipped).  Pixel geometry (two integer divisions,
// a square root) is evaluated once per lane and pixel.
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
constexpr int kPerLane = 8;                  // consecutive bins per lane
constexpr int kTile = kBlock * kPerLane;     // bins per workgroup tile
constexpr int kPadded = kTile + kTile / 8;   // one pad word per 8 bins

// LDS position of bin j of a tile: a pad double after every 8 bins keeps
// the lanes' 8-bin runs on distinct banks
__device__ __forceinline__ int lds_pos(int j) { return j + (j >> 3); }

// centre of pixel `pid`: distance from the sample and cos(2theta)
__device__ __forceinline__ void pixel_geom(const DevDet& D, const float* __restrict__ tab,
                                           uint32_t pid, float& L2, float& c2t) {
  if (D.type == DET_SPHERE) {
    L2 = D.R;
    c2t = cosf(((float)pid + 0.5f) / D.ring_scale);
  } else {
    const uint32_t tube = pid / (uint32_t)D.npix;
    const uint32_t j = pid - tube * (uint32_t)D.npix;
    const uint32_t r = tube / (uint32_t)D.ncols;
    const uint32_t c = tube - r * (uint32_t)D.ncols;
    const float x = tab[D.t_cols + 2 * c];
    const float z = tab[D.t_cols + 2 * c + 1];
    const float y = D.row_y[r] - D.half_len + ((float)j + 0.5f) / D.pix_scale;
    L2 = sqrtf(x * x + y * y + z * z);
    c2t = z / L2;
  }
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

template <bool W2>
__global__ void __launch_bounds__(kBlock)
reduce_hist_qe(const DevPlan* __restrict__ plan, const float* __restrict__ tab, QEMap M,
               const double* __restrict__ hist, const double* __restrict__ hw2, uint64_t nbins,
               double* __restrict__ iqe, double* __restrict__ iqe_w2) {
  __shared__ double sv[kPadded];
  __shared__ double sw[W2 ? kPadded : 1];
  const DevDet& D = plan->det;
  const int tid = threadIdx.x;
  const uint64_t ntof = (uint64_t)M.ntof;
  const bool narrow = nbins <= 0xFFFFFFFFull;
  const uint64_t ntiles = (nbins + kTile - 1) / kTile;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint64_t base = tile * kTile;
#pragma unroll
    for (int k = 0; k < kPerLane / 2; ++k) {
      const int j = 2 * (k * kBlock + tid);
      double a = 0.0, b = 0.0, a2 = 0.0, b2 = 0.0;
      if (base + j + 1 < nbins) {
        const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(hist + base + j));
        a = v.x;
        b = v.y;
        if (W2) {
          const dvec2 w = __builtin_nontemporal_load(reinterpret_cast<const dvec2*>(hw2 + base + j));
          a2 = w.x;
          b2 = w.y;
        }
      } else if (base + j < nbins) {
        a = hist[base + j];
        if (W2) a2 = hw2[base + j];
      }
      sv[lds_pos(j)] = a;
      sv[lds_pos(j) + 1] = b;
      if (W2) {
        sw[lds_pos(j)] = a2;
        sw[lds_pos(j) + 1] = b2;
      }
    }
    __syncthreads();
    const uint64_t i0 = base + (uint64_t)tid * kPerLane;
    if (i0 < nbins) {
      uint32_t pid = narrow ? (uint32_t)i0 / (uint32_t)ntof : (uint32_t)(i0 / ntof);
      uint32_t tb = (uint32_t)(i0 - (uint64_t)pid * ntof);
      float L2, c2t;
      pixel_geom(D, tab, pid, L2, c2t);
      int cur = -1;
      double acc = 0.0, acc2 = 0.0;
      const int nk = nbins - i0 < (uint64_t)kPerLane ? (int)(nbins - i0) : kPerLane;
      for (int k = 0; k < nk; ++k) {
        const double v = sv[lds_pos(tid * kPerLane + k)];
        const double v2 = W2 ? sw[lds_pos(tid * kPerLane + k)] : 0.0;
        if (v != 0.0 || v2 != 0.0) {
          const int dst = qe_bin(M, L2, c2t, M.tof_lo + ((float)tb + 0.5f) * M.dt);
          if (dst != cur) {
            if (cur >= 0) {
              unsafeAtomicAdd(iqe + cur, acc);
              if (W2) unsafeAtomicAdd(iqe_w2 + cur, acc2);
            }
            cur = dst;
            acc = 0.0;
            acc2 = 0.0;
          }
          acc += v;
          if (W2) acc2 += v2;
        }
        if (++tb == (uint32_t)ntof) {
          tb = 0;
          ++pid;
          if (k + 1 < nk) pixel_geom(D, tab, pid, L2, c2t);
        }
      }
      if (cur >= 0) {
        unsafeAtomicAdd(iqe + cur, acc);
        if (W2) unsafeAtomicAdd(iqe_w2 + cur, acc2);
      }
    }
    __syncthreads();
  }
}

template <bool W2>
__global__ void __launch_bounds__(kBlock)
reduce_events_qe(const DevPlan* __restrict__ plan, const float* __restrict__ tab, QEMap M,
                 const DevEvent* __restrict__ ev, const unsigned long long* __restrict__ n_dev,
                 uint64_t cap, double* __restrict__ iqe, double* __restrict__ iqe_w2) {
  const DevDet& D = plan->det;
  const uint64_t n = *n_dev < cap ? *n_dev : cap;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const DevEvent e = ev[i];
    if (e.pixel >= M.npixels) continue;
    float L2, c2t;
    pixel_geom(D, tab, e.pixel, L2, c2t);
    const int dst = qe_bin(M, L2, c2t, e.tof);
    if (dst >= 0) {
      unsafeAtomicAdd(iqe + dst, (double)e.value);
      if (W2) unsafeAtomicAdd(iqe_w2 + dst, (double)e.value * (double)e.value);
    }
  }
}

}  // namespace red

hipError_t launch_reduce_hist(const DevPlan* plan, const float* tables, const QEMap& M,
                              const double* hist, const double* hist_w2, uint64_t nbins,
                              double* iqe, double* iqe_w2, int grid, hipStream_t stream) {
  if (hist_w2 && iqe_w2)
    hipLaunchKernelGGL(red::reduce_hist_qe<true>, dim3(grid), dim3(red::kBlock), 0, stream, plan,
                       tables, M, hist, hist_w2, nbins, iqe, iqe_w2);
  else
    hipLaunchKernelGGL(red::reduce_hist_qe<false>, dim3(grid), dim3(red::kBlock), 0, stream,
                       plan, tables, M, hist, nullptr, nbins, iqe, nullptr);
  return hipGetLastError();
}

hipError_t launch_reduce_events(const DevPlan* plan, const float* tables, const QEMap& M,
                                const DevEvent* ev, const unsigned long long* n_dev, uint64_t cap,
                                double* iqe, double* iqe_w2, int grid, hipStream_t stream) {
  if (iqe_w2)
    hipLaunchKernelGGL(red::reduce_events_qe<true>, dim3(grid), dim3(red::kBlock), 0, stream,
                       plan, tables, M, ev, n_dev, cap, iqe, iqe_w2);
  else
    hipLaunchKernelGGL(red::reduce_events_qe<false>, dim3(grid), dim3(red::kBlock), 0, stream,
                       plan, tables, M, ev, n_dev, cap, iqe, nullptr);
  return hipGetLastError();
}

int reduce_tile_bins() { return red::kTile; }

}  // namespace mcv
