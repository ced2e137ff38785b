// mcv_determ.hip -- deterministic summation of recorded probabilities.
//
// The intensity of a (pixel, tof) bin is the sum of the probabilities of
// the packets recorded in it (Sec. 3).  Binary64 atomics add them in arrival
// order, so two runs agree only up to rounding order.  In deterministic mode
// a chunk of histories is traced with one (key, value) entry per recorded
// packet, key = bin | history id | lineage (most significant first); the
// entries are sorted by key (hipCUB radix sort) and each run of one bin is
// summed by one thread in key order, then added to the bin.  The order of
// every addition is then fixed by the keys alone, and the chunks are added
// in order on the stream.

#include <hip/hip_runtime.h>
#include <hipcub/device/device_radix_sort.hpp>

#include <cstdint>

namespace mcv {
namespace dev {

__global__ void det_zero_counter(unsigned long long* n) {
  if (threadIdx.x == 0) *n = 0ull;
}

// one thread per entry; the first entry of each bin's run sums the run
// (values in key order, binary64) and adds it (and the sum of squares) to
// the bin, which no other thread of the chunk touches
__global__ void __launch_bounds__(256)
det_run_sums(const uint64_t* __restrict__ keys, const float* __restrict__ vals, uint64_t count,
             int bin_shift, double* __restrict__ hist, double* __restrict__ hist_w2) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t b = keys[i] >> bin_shift;
  if (i > 0 && (keys[i - 1] >> bin_shift) == b) return;
  double s = 0.0, s2 = 0.0;
  for (uint64_t j = i; j < count && (keys[j] >> bin_shift) == b; ++j) {
    const double v = (double)vals[j];
    s += v;
    s2 += v * v;
  }
  if (hist) hist[b] += s;
  if (hist_w2) hist_w2[b] += s2;
}

}  // namespace dev

hipError_t det_zero(unsigned long long* n, hipStream_t stream) {
  hipLaunchKernelGGL(dev::det_zero_counter, dim3(1), dim3(64), 0, stream, n);
  return hipGetLastError();
}

// temp == nullptr: *temp_bytes receives the workspace size for `count` items
hipError_t det_sort(void* temp, size_t* temp_bytes, const uint64_t* kin, uint64_t* kout,
                    const float* vin, float* vout, uint64_t count, int end_bit,
                    hipStream_t stream) {
  return hipcub::DeviceRadixSort::SortPairs(temp, *temp_bytes, kin, kout, vin, vout,
                                            (int)count, 0, end_bit, stream);
}

hipError_t det_sums(const uint64_t* keys, const float* vals, uint64_t count, int bin_shift,
                    double* hist, double* hist_w2, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(dev::det_run_sums, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     stream, keys, vals, count, bin_shift, hist, hist_w2);
  return hipGetLastError();
}

}  // namespace mcv
