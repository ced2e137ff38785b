// Cost probe for the transport library's device primitives on gfx950.
//
// Each probe kernel runs one primitive of the hot path (a Philox block, a
// shape's interval test, the attenuation terms of one interval, the split of
// a child, one kernel draw, one detector test, the source) many times per
// lane at full occupancy with every lane converged, on packets made from a
// cheap integer hash.  The time of a probe minus the time of the null probe
// (the same packet construction, no primitive), times the VALU issue rate,
// per call, is the primitive's cost in lane-operation slots.  With the
// primitive counts per history of the algorithm these give the arithmetic
// work per history that the transport roofline is priced against.
//
// Built as its own shared library together with the library's sources (the
// probes call the very device functions the transport kernels inline, and
// take plans made by the same plan builder).  Measurement infrastructure,
// not part of the transport path.

#include "mcv_transport.hip"
#include "mcv_reduce.hip"
#include "mcv_adjoint.hip"
#include "mcv_determ.hip"
#include "mcv_api.cpp"

namespace mcv {
namespace probe {

using namespace dev;

enum {
  PR_NULL = 0,
  PR_RNG = 1,
  PR_SOURCE = 2,
  PR_SHAPE = 3,
  PR_SEGMENT = 4,
  PR_SPLIT = 5,
  PR_KERNEL = 6,
  PR_DETECT = 7,
  PR_DETECT_COL = 8,  // tube detectors: the first steps only (tube_column)
  PR_DETECT_HIT = 9   // tube detectors: the whole test on rays aimed at a tube
};

// 32-bit integer mix (the "lowbias32" constants of C. Wellons' hash search)
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

constexpr int kNU = 8;

// a packet near the sample (within +-3 cm of the origin), isotropic
// direction, speed sp0 (1 +- 10 %), and kNU uniforms for the primitive
__device__ __forceinline__ void make_input(uint32_t& h, float sp0, Pk& P, float* u) {
  float v[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    h = mix32(h + 0x9e3779b9u);
    v[i] = unif(h);
  }
#pragma unroll
  for (int i = 0; i < kNU; ++i) {
    h = mix32(h + 0x9e3779b9u);
    u[i] = unif(h);
  }
  P.px = 0.06f * (v[0] - 0.5f);
  P.py = 0.06f * (v[1] - 0.5f);
  P.pz = 0.06f * (v[2] - 0.5f);
  iso_dir(v[3], v[4], P.dx, P.dy, P.dz);
  P.sp = sp0 * (0.9f + 0.2f * v[5]);
  P.t = 1e-4f * v[0];
  P.w = 1.0f;
  P.lin = 9u;
}

__device__ __forceinline__ int entry_code_of(const DevScat& S) {
  return S.shape == SHAPE_BOX ? ENTRY_BOX_X + 2 : ENTRY_OUTER;
}

template <int PR>
__global__ void __launch_bounds__(256)
probe_kernel(const DevPlan* __restrict__ gplan, const float* __restrict__ gtab, DevBeam beam,
             uint64_t seed, int arg, uint32_t iters, float sp0, float* __restrict__ sink,
             uint32_t* __restrict__ hits) {
  __shared__ DevPlan PL;
  extern __shared__ __align__(16) float dyn[];
  const int tid = threadIdx.x;
  stage_plan(PL, dyn, gplan, gtab, blockDim.x, tid);
  __syncthreads();
  const uint32_t gid = blockIdx.x * blockDim.x + tid;
  uint32_t h = mix32(gid * 0x2545f491u + 0x1234567u);
  float acc = 0.0f;
  uint32_t nh = 0;
  for (uint32_t it = 0; it < iters; ++it) {
    Pk P;
    float u[kNU];
    make_input(h, sp0, P, u);
    acc += P.px + P.py + P.pz + P.dx + P.dy + P.dz + P.sp + u[0] + u[1] + u[2] + u[3] + u[4] +
           u[5] + u[6] + u[7];
    if (PR == PR_RNG) {
      float r[4];
      draw4((uint64_t)gid * iters + it, STREAM_SCATTER, h, 0u, seed, r);
      acc += r[0] + r[1] + r[2] + r[3];
    } else if (PR == PR_SOURCE) {
      const Pk S = source(beam, (uint64_t)gid * iters + it + h, seed);
      acc += S.px + S.py + S.pz + S.sp + S.t + S.w;
    } else if (PR == PR_SHAPE) {
      Iv a, b;
      a.lo = a.hi = a.len = b.lo = b.hi = b.len = 0.0f;
      const int n = shape_iv(PL.s[arg], P, a, b);
      acc += a.lo + a.hi + a.len + b.lo + b.len + (float)(n + a.entry + b.entry);
    } else if (PR == PR_SEGMENT) {
      Mu mu;
      float att, pint;
      segment_terms(PL.s[arg], dyn, P.sp, 0.02f * u[0], mu, att, pint);
      acc += att + pint + mu.scat;
    } else if (PR == PR_SPLIT) {
      const DevScat& S = PL.s[arg];
      Mu mu;
      mu.scat = 0.0f;
#pragma unroll
      for (int q = 0; q < kMaxKern; ++q) {
        mu.k[q] = q < S.nk ? 0.1f + u[2 + q] : 0.0f;
        mu.scat += mu.k[q];
      }
      mu.total = mu.scat + 0.5f;
      Pk C;
      float x;
      const int k = split_child(S, mu, 0.5f * u[5], P, P.px, P.py, P.pz, P.t, 0.01f * u[6],
                                (gid & 1u) ? entry_code_of(S) : ENTRY_NONE, u, 73u, C, x);
      acc += C.px + C.py + C.pz + C.t + C.w + x + (float)k;
    } else if (PR == PR_KERNEL) {
      const DevScat& S = PL.s[arg >> 2];
      const Out o = kernel_eval<true, true>(S.k[arg & 3], S, dyn, P, u,
                                            (uint64_t)gid * iters + it, h, seed);
      acc += o.dx + o.dy + o.dz + o.sp + o.f + o.dwq2 + (float)o.bin;
    } else if (PR == PR_DETECT) {
      const Hit hh = PL.det.type == DET_SPHERE
                         ? detect_sphere(PL.det, P)
                         : detect_tubes(PL.det, dyn, P, (uint64_t)gid * iters + it, seed);
      acc += hh.value + hh.tof + (float)hh.bin;
      if (PL.det.type != DET_SPHERE && hh.tube >= 0) ++nh;
    } else if (PR == PR_DETECT_COL) {
      float a;
      uint32_t rows;
      int col;
      const bool pass = tube_column(PL.det, P, a, rows, col);
      acc += a + (float)rows + (float)col;
      nh += pass ? 1u : 0u;
    } else if (PR == PR_DETECT_HIT) {
      // every lane's ray aimed at a point on the axis of a random tube, so
      // that the whole wave runs the candidate tests and the absorption
      const DevDet& D = PL.det;
      const int cc = min((int)(u[0] * (float)D.ncols), D.ncols - 1);
      const int rr = min((int)(u[1] * (float)D.nrows), D.nrows - 1);
      const float ex = dyn[D.t_cols + 2 * cc] - P.px;
      const float ey = D.row_y[rr] + 1.8f * (u[2] - 0.5f) * D.half_len - P.py;
      const float ez = dyn[D.t_cols + 2 * cc + 1] - P.pz;
      const float inv = 1.0f / sqrtf(ex * ex + ey * ey + ez * ez);
      P.dx = ex * inv;
      P.dy = ey * inv;
      P.dz = ez * inv;
      const Hit hh = detect_tubes(D, dyn, P, (uint64_t)gid * iters + it, seed);
      acc += hh.value + hh.tof + (float)hh.bin;
      if (hh.tube >= 0) ++nh;
    }
  }
  sink[gid] = acc;
  hits[gid] = nh;
}

// Binary64 atomic add rate: every lane adds 1.0 `iters` times into a
// histogram of nbins (< 2^32) doubles, at bins from a hash of (lane,
// iteration), uniform over the histogram, except that hot_permille of the
// updates go to bin 0 (the direct beam's one pixel and time bin).  The
// global atomics execute at the memory side.
__global__ void __launch_bounds__(256)
atomic_probe(double* __restrict__ hist, uint32_t nbins, uint32_t iters, uint32_t hot_permille,
             uint32_t seed) {
  const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t h = mix32(gid ^ seed);
  for (uint32_t it = 0; it < iters; ++it) {
    h = mix32(h + 0x9e3779b9u);
    const uint32_t g = mix32(h ^ 0x85ebca6bu);
    uint32_t b = (uint32_t)(((uint64_t)h * nbins) >> 32);  // < nbins
    if (g % 1000u < hot_permille) b = 0u;
    unsafeAtomicAdd(hist + b, 1.0);
  }
}

template <int PR>
hipError_t launch_probe(mcv_plan p, const DevBeam& B, uint64_t seed, int arg, uint32_t iters,
                        float sp0, int grid, float* sink, uint32_t* hits, hipStream_t s) {
  const size_t lds = sizeof(float) * (size_t)((p->host.n_tables + 3) & ~3);
  hipLaunchKernelGGL((probe_kernel<PR>), dim3(grid), dim3(256), lds, s, p->d_plan, p->d_tables, B,
                     seed, arg, iters, sp0, sink, hits);
  return hipGetLastError();
}

}  // namespace probe
}  // namespace mcv

extern "C" {

// Runs probe `kind` (PR_*) with argument `arg` (scatterer index; for
// kernels scatterer * 4 + kernel) on `grid` workgroups of 256 lanes,
// `iters` calls per lane, `reps` timed repetitions after one warm-up.
// Writes the best time in ms and, for the detector probes, the fraction of
// calls that hit a tube (PR_DETECT, PR_DETECT_HIT: one Philox block each) or
// pass tube_column (PR_DETECT_COL).
// Returns MCV_OK or an error status (bad kind, argument or launch).
mcv_status mcv_probe_time(mcv_plan p, const mcv_beam* beam, uint64_t seed, int32_t kind,
                          int32_t arg, uint32_t iters, int32_t grid, int32_t reps,
                          double* ms_out, double* draws_per_call) {
  using namespace mcv::probe;
  if (!p || !ms_out || !draws_per_call) return fail(MCV_EINVAL, "null argument");
  if (grid <= 0 || grid > 65536 || iters == 0 || reps <= 0) return fail(MCV_EINVAL, "bad size");
  if ((kind == PR_SHAPE || kind == PR_SEGMENT || kind == PR_SPLIT) &&
      (arg < 0 || arg >= p->host.nscat))
    return fail(MCV_EINVAL, "scatterer index out of range");
  if (kind == PR_KERNEL &&
      (arg < 0 || (arg >> 2) >= p->host.nscat || (arg & 3) >= p->host.s[arg >> 2].nk))
    return fail(MCV_EINVAL, "kernel index out of range");
  if (kind < PR_NULL || kind > PR_DETECT_HIT) return fail(MCV_EINVAL, "unknown probe");
  if ((kind == PR_DETECT_COL || kind == PR_DETECT_HIT) && p->host.det.type != DET_TUBES)
    return fail(MCV_EINVAL, "tube-detector probe on a plan without tubes");
  DevBeam B;
  mcv_status st = make_beam(p, beam, &B);
  if (st != MCV_OK) return st;
  (void)hipSetDevice(p->device);
  if (set_transport_lds_limit(160 * 1024) != hipSuccess) return fail(MCV_EHIP, "lds limit");
  const size_t lanes = (size_t)grid * 256;
  float* sink = nullptr;
  uint32_t* hits = nullptr;
  hipError_t e = hipMalloc(&sink, lanes * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&hits, lanes * sizeof(uint32_t));
  if (e != hipSuccess) {
    (void)hipFree(sink);
    return hipfail(e, "probe buffers");
  }
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  const float sp0 = std::sqrt((float)beam->E / 5.22703759e-6f);
  double best = 1e30;
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {
    (void)hipEventRecord(a, nullptr);
    switch (kind) {
#define MCV_PROBE_CASE(K)                                                              \
  case K:                                                                              \
    e = launch_probe<K>(p, B, seed, arg, iters, sp0, grid, sink, hits, nullptr); \
    break;
      MCV_PROBE_CASE(PR_NULL)
      MCV_PROBE_CASE(PR_RNG)
      MCV_PROBE_CASE(PR_SOURCE)
      MCV_PROBE_CASE(PR_SHAPE)
      MCV_PROBE_CASE(PR_SEGMENT)
      MCV_PROBE_CASE(PR_SPLIT)
      MCV_PROBE_CASE(PR_KERNEL)
      MCV_PROBE_CASE(PR_DETECT)
      MCV_PROBE_CASE(PR_DETECT_COL)
      MCV_PROBE_CASE(PR_DETECT_HIT)
#undef MCV_PROBE_CASE
    }
    (void)hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (r > 0 && ms < best) best = ms;
  }
  std::vector<uint32_t> hh(lanes);
  if (e == hipSuccess) e = hipMemcpy(hh.data(), hits, lanes * sizeof(uint32_t), hipMemcpyDeviceToHost);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(sink);
  (void)hipFree(hits);
  if (e != hipSuccess) return hipfail(e, "probe run");
  double tot = 0.0;
  for (uint32_t v : hh) tot += v;
  *ms_out = best;
  *draws_per_call = tot / ((double)lanes * iters);
  return MCV_OK;
}

// Times the binary64 atomic probe: grid workgroups of 256 lanes, iters
// adds per lane into hist[nbins] (device, zeroed by the call), best of reps
// after one warm-up; *ms_out is the best time, *total the sum of the
// histogram after the last repetition (grid 256 iters when every add landed).
mcv_status mcv_probe_atomics(double* hist, uint64_t nbins, uint32_t iters, uint32_t hot_permille,
                             int32_t grid, int32_t reps, double* ms_out, double* total) {
  using namespace mcv::probe;
  if (!hist || !ms_out || !total) return fail(MCV_EINVAL, "null argument");
  if (nbins == 0 || nbins >= ((uint64_t)1 << 32) || grid <= 0 || grid > 65536 || iters == 0 ||
      reps <= 0 || hot_permille > 1000)
    return fail(MCV_EINVAL, "bad size");
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  hipError_t e = hipSuccess;
  double best = 1e30;
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {
    e = hipMemset(hist, 0, nbins * sizeof(double));
    if (e != hipSuccess) break;
    (void)hipEventRecord(a, nullptr);
    hipLaunchKernelGGL(atomic_probe, dim3(grid), dim3(256), 0, nullptr, hist, (uint32_t)nbins,
                       iters, hot_permille, 0x1234567u + (uint32_t)r);
    e = hipGetLastError();
    (void)hipEventRecord(b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (r > 0 && ms < best) best = ms;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return hipfail(e, "atomic probe");
  // the sum of the histogram: every add landed
  std::vector<double> h(nbins < 4096 ? nbins : 0);
  double t = 0.0;
  if (!h.empty()) {
    if ((e = hipMemcpy(h.data(), hist, nbins * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess)
      return hipfail(e, "atomic probe copy");
    for (double v : h) t += v;
  } else {
    t = -1.0;  // not summed for large histograms
  }
  *ms_out = best;
  *total = t;
  return MCV_OK;
}

}  // extern "C"
