// mcv_adjoint.hip -- binary64 tables and the dense terms of the adjoint.
//
// The adjoint differentiates the Monte Carlo estimate of I with every random
// choice held fixed (an extension of the paper's method).  A packet's weight
// is its path density at theta over the density it was drawn from at the
// plan's values theta0.  For the raw DOS values theta_b of a one-phonon
// kernel (Supplement S4: Z = theta / S, S = sum theta de, the Debye-Waller
// exponent 2W = (hbar^2/2M) gamma0 Q^2 with gamma0 = sum_b c_b theta_b / S,
// c_b = coth(e_b/2kT) de / e_b) the derivative of log(weight) splits into
//   sparse terms 1/theta_b for every DOS draw from bin b,
//   dnorm = -de/S per DOS draw (the normalisation S),
//   dense_a[b] = -(hbar^2/2M)(c_b - gamma0 de)/S per unit of sum Q^2 over
//     the packet's Debye-Waller factors (gamma0 through 2W);
// for the cells S_c of a tabulated S(Q,E) grid (Sec. 2.4.2) a draw that reads
// cell c contributes 1/S_c.  The transport kernel gathers dL/dI at each
// recorded packet and accumulates g = dL/dI value per table entry and the two
// scalars sum(g A), sum(g n_draws); this file prepares the 1/theta and dense
// tables on the device from the plan's raw binary64 tables, applies the
// dense terms at the end, and holds the pass that accumulates the same
// partials from a tape written by a forward run instead of a re-trace.
//
// Workspace layout (binary64): [0] sum g A, [1] sum g n_draws, [2] dnorm,
// [3] unused, [4, 4 + nt) 1/table value (nt = nb + nc: DOS bins then grid
// cells; 0 for a zero entry), [4 + nt, 4 + nt + nb) dense_a.

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "mcv_internal.h"

namespace mcv {
namespace dev {

constexpr int kPrepThreads = 256;

// One workgroup: S and sum c_b theta_b by a fixed-order reduction (the same
// result on every call), then the tables.
__global__ void __launch_bounds__(kPrepThreads)
adjoint_prepare(const double* __restrict__ theta, int nb, double de, double kT, double h2m,
                const double* __restrict__ cells, int nc, double* __restrict__ ws) {
  __shared__ double red_s[kPrepThreads], red_g[kPrepThreads];
  const int tid = threadIdx.x;
  double ps = 0.0, pg = 0.0;
  for (int b = tid; b < nb; b += kPrepThreads) {
    const double e = (b + 0.5) * de;
    ps += theta[b] * de;
    pg += theta[b] * de / (e * tanh(e / (2.0 * kT)));
  }
  red_s[tid] = ps;
  red_g[tid] = pg;
  __syncthreads();
  for (int o = kPrepThreads / 2; o > 0; o >>= 1) {
    if (tid < o) {
      red_s[tid] += red_s[tid + o];
      red_g[tid] += red_g[tid + o];
    }
    __syncthreads();
  }
  const double S = red_s[0];
  const double g0 = nb > 0 && S > 0.0 ? red_g[0] / S : 0.0;
  const int nt = nb + nc;
  if (tid == 0) {
    ws[0] = 0.0;
    ws[1] = 0.0;
    ws[2] = nb > 0 && S > 0.0 ? -de / S : 0.0;
    ws[3] = 0.0;
  }
  for (int b = tid; b < nb; b += kPrepThreads) {
    const double e = (b + 0.5) * de;
    const double c = de / (e * tanh(e / (2.0 * kT)));
    ws[4 + b] = theta[b] > 0.0 ? 1.0 / theta[b] : 0.0;
    ws[4 + nt + b] = S > 0.0 ? -h2m * (c - g0 * de) / S : 0.0;
  }
  for (int i = tid; i < nc; i += kPrepThreads) ws[4 + nb + i] = cells[i] != 0.0 ? 1.0 / cells[i] : 0.0;
}

// grad[b] += dense_a[b] sum(g A) + dnorm sum(g n_draws) for the DOS bins:
// the terms of the normalisation and of gamma0, which touch every bin
__global__ void adjoint_finalize(double* __restrict__ grad, const double* __restrict__ ws, int nb,
                                 int nc) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < nb) grad[b] += ws[4 + nb + nc + b] * ws[0] + ws[2] * ws[1];
}

constexpr int kTapeThreads = 256;

// The backward pass over an adjoint tape (one entry per packet a forward run
// recorded, with its carry): per entry g = dL/dI[bin] * value, and the same
// partials as the re-trace accumulates at a detection: g times the carried
// d log w / d sigma_abs and d sigma, g A and g n_draws (wave sums into LDS),
// and g per carried table index (LDS partials when the table fits, scaled
// by 1/table at the flush; global atomics otherwise).  The entries are read
// field by field ([field][entry], coalesced).  A tape whose counter exceeds
// its capacity is incomplete: the gradient entries become NaN.
// WL2: the loss is the weighted least squares L = sum_b w_b (I_b - T_b)^2 of
// the tape run's own histogram I against a target T: dL/dI_b = 2 w_b (I_b -
// T_b) is formed at each entry from I, T and w at its bin (no dL/dI array),
// and since I_b is the sum of the values v of its entries, L = sum_b w_b T_b^2
// + sum over entries of v w_b (I_b - 2 T_b); the second sum is added to
// *loss.
template <bool LDS, bool WL2>
__global__ void __launch_bounds__(kTapeThreads)
tape_adjoint(const uint32_t* __restrict__ tape, uint64_t cap,
             const unsigned long long* __restrict__ n_tape, const double* __restrict__ dLdI,
             const double* __restrict__ I, const double* __restrict__ T,
             const double* __restrict__ w, double* __restrict__ loss, int nb, int nc,
             double* __restrict__ grad, double* __restrict__ ws) {
  extern __shared__ double acc[];  // [table partials (LDS) | 5 scalars]
  const int ntab = LDS ? nb + nc : 0;
  const int np = nb + nc;
  const int tid = threadIdx.x;
  for (int i = tid; i < ntab + 5; i += kTapeThreads) acc[i] = 0.0;
  __syncthreads();
  const unsigned long long count = *n_tape;
  if (count > cap) {
    if (blockIdx.x == 0) {
      for (int i = tid; i < np + 2; i += kTapeThreads) grad[i] = __builtin_nan("");
      if (WL2 && tid == 0) *loss = __builtin_nan("");
    }
    return;
  }
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * kTapeThreads;
  for (uint64_t i = (uint64_t)blockIdx.x * kTapeThreads + tid; i < count; i += stride) {
    const uint32_t bin = tape[i];
    const double v = (double)__uint_as_float(tape[cap + i]);
    double g;
    if (WL2) {
      const double ib = I[bin], tb = T[bin], wb = w[bin];
      g = 2.0 * wb * (ib - tb);
      s4 += v * wb * (ib - 2.0 * tb);
    } else {
      g = dLdI[bin];
    }
    const double gv = g * v;
    if (gv == 0.0) continue;
    s0 += gv * (double)__uint_as_float(tape[2 * cap + i]);
    s1 += gv * (double)__uint_as_float(tape[3 * cap + i]);
    s2 += gv * (double)__uint_as_float(tape[4 * cap + i]);
    const uint32_t cnt = tape[5 * cap + i];
    s3 += gv * (double)(cnt & 0xFFFFu);
    const uint32_t ns = cnt >> 16;
    uint32_t word = 0u;
    for (uint32_t k = 0; k < ns; ++k) {
      if ((k & 1u) == 0u) word = tape[(6 + (k >> 1)) * cap + i];
      const uint32_t idx = (word >> (16u * (k & 1u))) & 0xFFFFu;
      if (LDS) atomicAdd(&acc[idx], gv);
      else unsafeAtomicAdd(&grad[idx], gv * ws[4 + idx]);
    }
  }
  const double sv[5] = {s0, s1, s2, s3, s4};
#pragma unroll
  for (int k = 0; k < (WL2 ? 5 : 4); ++k) {
    double v = sv[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((tid & 63) == 0 && v != 0.0) atomicAdd(&acc[ntab + k], v);
  }
  __syncthreads();
  for (int i = tid; i < ntab; i += kTapeThreads)
    if (acc[i] != 0.0) unsafeAtomicAdd(&grad[i], acc[i] * ws[4 + i]);
  if (tid == 0) {
    if (acc[ntab] != 0.0) unsafeAtomicAdd(&grad[np], acc[ntab]);
    if (acc[ntab + 1] != 0.0) unsafeAtomicAdd(&grad[np + 1], acc[ntab + 1]);
    if (acc[ntab + 2] != 0.0) unsafeAtomicAdd(&ws[0], acc[ntab + 2]);
    if (acc[ntab + 3] != 0.0) unsafeAtomicAdd(&ws[1], acc[ntab + 3]);
    if (WL2 && acc[ntab + 4] != 0.0) unsafeAtomicAdd(loss, acc[ntab + 4]);
  }
}

}  // namespace dev

// LDS of the tape pass's table partials: at most this many entries
constexpr int kTapeLdsTable = 8000;

// dLdI given: the general pass; dLdI null: the weighted least squares form
// with I, T, w and loss
hipError_t launch_tape_adjoint(const uint32_t* tape, uint64_t cap, const unsigned long long* n,
                               const double* dLdI, const double* I, const double* T,
                               const double* w, double* loss, int nb, int nc, double* grad,
                               double* ws, int grid, hipStream_t stream) {
  const bool lds = nb + nc <= kTapeLdsTable;
  const bool wl2 = dLdI == nullptr;
  const size_t bytes = sizeof(double) * (size_t)((lds ? nb + nc : 0) + 5);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(grid), dim3(dev::kTapeThreads), bytes, stream, tape, cap, n,
                       dLdI, I, T, w, loss, nb, nc, grad, ws);
  };
  if (lds) {
    if (wl2) go(dev::tape_adjoint<true, true>);
    else go(dev::tape_adjoint<true, false>);
  } else {
    if (wl2) go(dev::tape_adjoint<false, true>);
    else go(dev::tape_adjoint<false, false>);
  }
  return hipGetLastError();
}

// The workspace of mcv_adjoint_noalloc, for callers that cannot allocate:
// one copy per device, held until the process ends; every such call on a
// device uses it (concurrent calls on one device race).  In host code the
// name `scratch` stands for the host-side shadow, not the device address:
// the address of each device's copy is taken once with hipGetSymbolAddress
// and only that pointer is handed to kernels.
static __device__ __align__(256) double scratch[kNoAllocWorkDoubles];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;  // per device, null until set up
}  // namespace

// Set-up, with `device` current (called by plan creation): records the
// address of that device's copy of the workspace.
hipError_t adjoint_scratch_setup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0) return hipErrorInvalidDevice;
  if (g_scratch_ptr.size() <= (size_t)device) g_scratch_ptr.resize((size_t)device + 1, nullptr);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<double*>(ptr);
  return hipSuccess;
}

// the device address of the workspace on `device`, or null before set-up
double* adjoint_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || (size_t)device >= g_scratch_ptr.size()) return nullptr;
  return g_scratch_ptr[device];
}

hipError_t launch_adjoint_prepare(const double* theta, int nb, double de, double kT, double h2m,
                                  const double* cells, int nc, double* ws, hipStream_t stream) {
  hipLaunchKernelGGL(dev::adjoint_prepare, dim3(1), dim3(dev::kPrepThreads), 0, stream, theta, nb,
                     de, kT, h2m, cells, nc, ws);
  return hipGetLastError();
}

hipError_t launch_adjoint_finalize(double* grad, const double* ws, int nb, int nc,
                                   hipStream_t stream) {
  if (nb <= 0) return hipSuccess;
  hipLaunchKernelGGL(dev::adjoint_finalize, dim3((nb + 255) / 256), dim3(256), 0, stream, grad, ws,
                     nb, nc);
  return hipGetLastError();
}

}  // namespace mcv
