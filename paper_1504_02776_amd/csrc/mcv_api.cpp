// mcv_api.cpp -- host side of the C ABI declared in include/mcv.h.
//
// Builds sample assemblies and detectors, validates them, prepares the
// binary32 device tables in binary64 (sorted d-spacings and prefix sums of
// the Debye-Scherrer cross sections, the normalised cumulative phonon DOS,
// the Debye-Waller coefficient from the DOS, tube column positions), uploads
// a plan, and launches the transport kernels.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/mcv.h"
#include "mcv_internal.h"

namespace mcv {
hipError_t launch_transport(const DevPlan* plan, const DevPlan& host_plan, const float* tables,
                            const DevBeam& beam, uint64_t seed, uint64_t first, uint64_t n,
                            int grid, int block, uint64_t per_wave, double* hist, double* hist_w2,
                            DevRecord* rec, uint64_t cap, unsigned long long* n_out,
                            DevEvent* ev, uint64_t ev_cap, unsigned long long* n_ev,
                            const AdjArgs* adj, float* gstack, const DetArgs* det,
                            const TapeArgs* tape, hipStream_t stream);
hipError_t det_zero(unsigned long long* n, hipStream_t stream);
hipError_t det_sort(void* temp, size_t* temp_bytes, const uint64_t* kin, uint64_t* kout,
                    const float* vin, float* vout, uint64_t count, int end_bit,
                    hipStream_t stream);
hipError_t det_sums(const uint64_t* keys, const float* vals, uint64_t count, int bin_shift,
                    double* hist, double* hist_w2, hipStream_t stream);
hipError_t launch_adjoint_prepare(const double* theta, int nb, double de, double kT, double h2m,
                                  const double* cells, int nc, double* ws, hipStream_t stream);
hipError_t launch_adjoint_finalize(double* grad, const double* ws, int nb, int nc,
                                   hipStream_t stream);
hipError_t launch_tape_adjoint(const uint32_t* tape, uint64_t cap, const unsigned long long* n,
                               const double* dLdI, const double* I, const double* T,
                               const double* w, double* loss, int nb, int nc, double* grad,
                               double* ws, int grid, hipStream_t stream);
hipError_t adjoint_scratch_setup(int device);
double* adjoint_scratch(int device);
hipError_t launch_loss_grad(const double* I, const double* T, const double* w, int64_t n,
                            double* dLdI, double* loss, int grid, hipStream_t stream);
hipError_t launch_fill_zero(double* p, uint64_t n, int grid, hipStream_t stream);
size_t transport_lds_bytes(int n_tables, int stack_cap, int block, int adj_ntab, int hot_n);
int transport_dq_entries(const DevPlan& P);
int batch_dq_entries(const DevPlan& P);
size_t transport_dq_bytes(int block, int entries, bool adjoint);
size_t transport_static_lds();
int transport_waves_per_eu(int nscat, int smax);
int batch_waves_per_eu();
hipError_t set_transport_lds_limit(size_t bytes);
hipError_t launch_reduce_hist(const float* geo, const QEMap& M,
                              const double* hist, const double* hist_w2, uint64_t nbins,
                              double* iqe, double* iqe_w2, int grid, int cus,
                              hipStream_t stream);
hipError_t launch_reduce_events(const float* geo, const QEMap& M,
                                const DevEvent* ev, const unsigned long long* n_dev, uint64_t cap,
                                double* iqe, double* iqe_w2, int grid, hipStream_t stream);
int reduce_tile_bins();
}  // namespace mcv

using namespace mcv;

namespace {

thread_local std::string g_err;

mcv_status fail(mcv_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

mcv_status hipfail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return MCV_EHIP;
}

// CODATA 2018 values used by the host-side table preparation
const double kHbar2over2mn = 2.0721249;  // meV A^2
const double kBoltzmann = 0.08617333;    // meV / K
const double kNeutronMassAmu = 1.00866491595;
const double kPi = 3.14159265358979323846;
const double kHe3SigmaAbs = 5333.0;      // barn at 2200 m/s
const double kEperV2 = 5.22703759e-6;    // meV per (m/s)^2, m_n / 2

struct KernelCopy {
  mcv_kernel k;
  std::vector<double> d, F2, dos, sqe, modes;
};

struct Scatterer {
  mcv_shape shape;
  mcv_material mat;
  std::vector<KernelCopy> kernels;
};

bool finite_all(const double* x, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

// Slots of the LDS histogram bin cache: the most (kHotMin..kHotMax, a power
// of two) that fit beside `base` bytes of LDS per workgroup when the
// Default grid depth (waves_per_simd of mcv_opts: waves per SIMD the grid
// is sized for, two rounds of them), the shallowest one used, and the
// fewest histories per wave a launch spreads to beyond two rounds of the
// shallowest.
constexpr int kGridDepth = 16;
constexpr int kGridDepthMin = 4;
constexpr uint64_t kMinPerWave = 512;

// workgroups of `waves_per_simd` resident waves share a CU's 160 KiB.
int hot_slots(size_t base, int block, int waves_per_simd) {
  const int wgs = std::max(1, waves_per_simd * 4 * 64 / block);
  const size_t budget = (size_t)160 * 1024 / (size_t)wgs;
  int n = kHotMax;
  while (n > kHotMin && base + 4 * (size_t)hot_words(n) > budget) n /= 2;
  return n;
}

// Azimuthal pitch of neighbouring tubes within a pack, and the azimuth of
// column c: phi_lo + floor(c / P) gap + (c + 1/2) pitch (P = 0: no packs).
double tube_pitch(const mcv_tube_layout& L) {
  const int P = L.tubes_per_pack;
  const int npack = P > 0 ? L.ncols / P : 1;
  return (L.phi_hi - L.phi_lo - (P > 0 ? (npack - 1) * L.pack_gap : 0.0)) / L.ncols;
}
double column_azimuth(const mcv_tube_layout& L, int c) {
  const int P = L.tubes_per_pack;
  return L.phi_lo + (P > 0 ? (c / P) * L.pack_gap : 0.0) + (c + 0.5) * tube_pitch(L);
}

int intervals_of(const mcv_shape& s) { return s.type == MCV_SHAPE_ANNULUS ? 2 : 1; }

// lab-frame corners of the bounding box of a shape
std::vector<std::array<double, 3>> corners(const mcv_shape& s) {
  double hx, hy, hz;
  if (s.type == MCV_SHAPE_BOX) {
    hx = 0.5 * s.dims[0];
    hy = 0.5 * s.dims[1];
    hz = 0.5 * s.dims[2];
  } else if (s.type == MCV_SHAPE_CYLINDER) {
    hx = hz = s.dims[0];
    hy = 0.5 * s.dims[1];
  } else {
    hx = hz = s.dims[1];
    hy = 0.5 * s.dims[2];
  }
  std::vector<std::array<double, 3>> out;
  for (int i = 0; i < 8; ++i) {
    double l[3] = {(i & 1) ? hx : -hx, (i & 2) ? hy : -hy, (i & 4) ? hz : -hz};
    std::array<double, 3> p;
    for (int r = 0; r < 3; ++r)
      p[r] = s.pos[r] + s.rot[3 * r] * l[0] + s.rot[3 * r + 1] * l[1] + s.rot[3 * r + 2] * l[2];
    out.push_back(p);
  }
  return out;
}

void aabb(const mcv_shape& s, double lo[3], double hi[3]) {
  auto c = corners(s);
  for (int r = 0; r < 3; ++r) {
    lo[r] = 1e300;
    hi[r] = -1e300;
    for (auto& p : c) {
      lo[r] = std::min(lo[r], p[r]);
      hi[r] = std::max(hi[r], p[r]);
    }
  }
}

// every bounding-box corner of `inner` lies inside the hole of annulus `ann`
bool inside_hole(const mcv_shape& inner, const mcv_shape& ann) {
  if (ann.type != MCV_SHAPE_ANNULUS) return false;
  for (auto& p : corners(inner)) {
    double r[3] = {p[0] - ann.pos[0], p[1] - ann.pos[1], p[2] - ann.pos[2]};
    double x = ann.rot[0] * r[0] + ann.rot[3] * r[1] + ann.rot[6] * r[2];
    double z = ann.rot[2] * r[0] + ann.rot[5] * r[1] + ann.rot[8] * r[2];
    if (x * x + z * z >= ann.dims[0] * ann.dims[0]) return false;
  }
  return true;
}

bool disjoint(const mcv_shape& a, const mcv_shape& b) {
  double la[3], ha[3], lb[3], hb[3];
  aabb(a, la, ha);
  aabb(b, lb, hb);
  for (int r = 0; r < 3; ++r)
    if (ha[r] <= lb[r] || hb[r] <= la[r]) return true;
  return inside_hole(a, b) || inside_hole(b, a);
}

double bounding_radius(const mcv_shape& s) {
  double m = 0.0;
  for (auto& p : corners(s)) m = std::max(m, std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]));
  return m;
}

mcv_status check_shape(const mcv_shape& s) {
  if (s.type < MCV_SHAPE_BOX || s.type > MCV_SHAPE_ANNULUS) return fail(MCV_EINVAL, "unknown shape type");
  if (!finite_all(s.dims, 3) || !finite_all(s.pos, 3) || !finite_all(s.rot, 9))
    return fail(MCV_EINVAL, "non-finite shape parameter");
  int nd = s.type == MCV_SHAPE_ANNULUS ? 3 : (s.type == MCV_SHAPE_BOX ? 3 : 2);
  for (int i = 0; i < nd; ++i)
    if (!(s.dims[i] > 0.0)) return fail(MCV_EINVAL, "shape dimensions must be > 0");
  if (s.type == MCV_SHAPE_ANNULUS && !(s.dims[0] < s.dims[1]))
    return fail(MCV_EINVAL, "annulus needs inner radius < outer radius");
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double d = 0.0;
      for (int k = 0; k < 3; ++k) d += s.rot[3 * i + k] * s.rot[3 * j + k];
      if (std::fabs(d - (i == j ? 1.0 : 0.0)) > 1e-6)
        return fail(MCV_EINVAL, "rotation is not orthonormal");
    }
  return MCV_OK;
}

mcv_status check_kernel(const mcv_kernel& k) {
  if (k.dw != 0 && k.dw != 1) return fail(MCV_EINVAL, "dw must be 0 or 1");
  switch (k.type) {
    case MCV_K_ISO_EL:
      if (!(k.sigma_b >= 0.0)) return fail(MCV_EINVAL, "sigma must be >= 0");
      return MCV_OK;
    case MCV_K_POWDER:
      if (!(k.v0 > 0.0) || k.nrefl < 1 || k.nrefl > 4096 || !k.d || !k.F2)
        return fail(MCV_EINVAL, "powder kernel needs v0 > 0 and 1..4096 reflections");
      for (int i = 0; i < k.nrefl; ++i)
        if (!(k.d[i] > 0.0) || !(k.F2[i] >= 0.0) || !std::isfinite(k.d[i]) || !std::isfinite(k.F2[i]))
          return fail(MCV_EINVAL, "powder reflections need d > 0 and F2 >= 0");
      return MCV_OK;
    case MCV_K_PHONON: {
      if (!(k.sigma_b >= 0.0) || !(k.M_amu > 0.0) || !(k.T_K > 0.0) || !(k.emax > 0.0) ||
          k.nbins < 1 || k.nbins > 8192 || !k.dos)
        return fail(MCV_EINVAL, "phonon kernel needs M > 0, T > 0, emax > 0, 1..8192 bins");
      double s = 0.0;
      for (int i = 0; i < k.nbins; ++i) {
        if (!(k.dos[i] >= 0.0) || !std::isfinite(k.dos[i])) return fail(MCV_EINVAL, "DOS values must be >= 0");
        s += k.dos[i];
      }
      if (!(s > 0.0)) return fail(MCV_EINVAL, "DOS must have positive area");
      return MCV_OK;
    }
    case MCV_K_MULTIPHONON: {
      if (!(k.sigma_b >= 0.0) || !(k.M_amu > 0.0) || !(k.T_K > 0.0) || !(k.emax > 0.0) ||
          k.nbins < 1 || k.nbins > 4096 || !k.dos || k.max_phonons < 2 || k.max_phonons > 8)
        return fail(MCV_EINVAL,
                    "multi-phonon kernel needs M > 0, T > 0, emax > 0, 1..4096 bins, N in 2..8");
      if (k.dw) return fail(MCV_EUNSUPPORTED, "the multi-phonon kernel carries its own Debye-Waller factor");
      double s = 0.0;
      for (int i = 0; i < k.nbins; ++i) {
        if (!(k.dos[i] >= 0.0) || !std::isfinite(k.dos[i])) return fail(MCV_EINVAL, "DOS values must be >= 0");
        s += k.dos[i];
      }
      if (!(s > 0.0)) return fail(MCV_EINVAL, "DOS must have positive area");
      return MCV_OK;
    }
    case MCV_K_DISPERSION:
      if (!(k.sigma_b >= 0.0) || !(k.a > 0.0) || !std::isfinite(k.J) || !std::isfinite(k.S) ||
          !(k.J * k.S >= 0.0) || !finite_all(k.crot, 9))
        return fail(MCV_EINVAL, "dispersion kernel needs a > 0 and J S >= 0");
      if (k.dw) return fail(MCV_EUNSUPPORTED, "Debye-Waller factor not supported for the dispersion kernel");
      return MCV_OK;
    case MCV_K_SPINWAVE:
      if (!(k.sigma_b >= 0.0) || !(k.gamma > 0.0) || !(k.a > 0.0) || !finite_all(k.crot, 9))
        return fail(MCV_EINVAL, "spin-wave kernel needs gamma > 0 and a > 0");
      if (k.dw) return fail(MCV_EUNSUPPORTED, "Debye-Waller factor not supported for the spin-wave kernel");
      return MCV_OK;
    case MCV_K_SQE:
      if (!(k.sigma_b >= 0.0) || k.nQ < 1 || k.nE < 1 || (int64_t)k.nQ * k.nE > 65536 ||
          !(k.Qmax > 0.0) || !(k.Emax > k.Emin) || !k.sqe)
        return fail(MCV_EINVAL, "S(Q,E) kernel needs a grid of 1..65536 cells, Qmax > 0, Emax > Emin");
      for (int i = 0; i < k.nQ * k.nE; ++i)
        if (!(k.sqe[i] >= 0.0) || !std::isfinite(k.sqe[i])) return fail(MCV_EINVAL, "S(Q,E) values must be >= 0");
      if (k.dw) return fail(MCV_EUNSUPPORTED, "Debye-Waller factor not supported for the S(Q,E) kernel");
      return MCV_OK;
    case MCV_K_COH_PHONON: {
      if (!(k.sigma_b >= 0.0) || !(k.M_amu > 0.0) || !(k.T_K > 0.0) || k.grid_n < 2 ||
          k.grid_n > 128 || !k.modes || !finite_all(k.cell, 9))
        return fail(MCV_EINVAL, "coherent phonon kernel needs M > 0, T > 0, 2..128 grid points per axis");
      const double* c = k.cell;
      const double det = c[0] * (c[4] * c[8] - c[5] * c[7]) - c[1] * (c[3] * c[8] - c[5] * c[6]) +
                         c[2] * (c[3] * c[7] - c[4] * c[6]);
      if (!(std::fabs(det) > 1e-6)) return fail(MCV_EINVAL, "cell vectors are degenerate");
      const int64_t np = (int64_t)k.grid_n * k.grid_n * k.grid_n;
      double emax = 0.0;
      for (int64_t i = 0; i < np; ++i) {
        const double* m = k.modes + 12 * i;
        for (int b = 0; b < 3; ++b) {
          if (!(m[b] >= 0.0) || !std::isfinite(m[b])) return fail(MCV_EINVAL, "mode energies must be >= 0");
          emax = std::max(emax, m[b]);
          const double* e = m + 3 + 3 * b;
          const double nn = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
          if (!(std::fabs(nn - 1.0) < 1e-3)) return fail(MCV_EINVAL, "polarization vectors must be unit vectors");
        }
      }
      if (!(emax > 0.0)) return fail(MCV_EINVAL, "all mode energies are zero");
      return MCV_OK;
    }
    default:
      return fail(MCV_EINVAL, "unknown kernel type");
  }
}

}  // namespace

struct mcv_assembly_s {
  std::vector<Scatterer> scat;
};

struct mcv_detector_s {
  int type = 0;
  double R = 0, tof_lo = 0, tof_hi = 0;
  int n2t = 0, ntof = 0, npix = 0;
  mcv_tube_layout tubes;
};

// The adjoint's plan-owned binary64 workspace (see mcv_adjoint.hip for its
// layout), grown on demand.
struct AdjointWork {
  double* ws = nullptr;
  size_t cap = 0;  // doubles
};

struct mcv_plan_s {
  int device = 0;
  DevPlan host;
  std::vector<Scatterer> scat;  // host copy (adjoint tables)
  AdjointWork adj;
  std::vector<float> tables;
  // binary64 copies of the adjoint's table parameters (one-phonon DOS, S(Q,E)
  // grids) in device memory, at raw_off[s][k] (-1: none)
  double* d_raw = nullptr;
  int64_t raw_off[kMaxScat][kMaxKern];
  // per-lane packet stacks of the transport launches in device memory
  float* d_stack = nullptr;
  size_t stack_floats = 0;
  // deterministic summation: chunk of histories, entry capacity, key layout
  // and the (key, value) buffers, sort workspace and entry counter
  uint64_t det_chunk = 0, det_cap = 0;
  int det_lin_bits = 0, det_id_bits = 0;
  uint64_t* d_keys[2] = {nullptr, nullptr};
  float* d_vals[2] = {nullptr, nullptr};
  void* d_sort_tmp = nullptr;
  size_t sort_tmp_bytes = 0;
  unsigned long long* d_det_n = nullptr;
  DevPlan* d_plan = nullptr;
  float* d_tables = nullptr;
  float* d_pixgeo = nullptr;     // per pixel id: |r_p|, cos(2theta) (reduction)
  std::vector<float*> d_grids;   // mode tables of coherent phonon kernels
  int block = 256;
  int cus = 256;
  int waves_per_simd = kGridDepth;
  int64_t max_waves = 0;  // 0: fill the device
  int deterministic = 0;
  int64_t nbins = 0;
  double R = 0;
  double tof_lo = 0, tof_hi = 0;  // detector time window (binary64)
};

extern "C" {

int32_t mcv_abi_version(void) { return 1; }

const char* mcv_last_error(void) { return g_err.c_str(); }

mcv_status mcv_assembly_create(mcv_assembly* out) {
  if (!out) return fail(MCV_EINVAL, "null output handle");
  *out = new (std::nothrow) mcv_assembly_s();
  return *out ? MCV_OK : fail(MCV_ENOMEM, "host allocation failed");
}

mcv_status mcv_assembly_destroy(mcv_assembly a) {
  delete a;
  return MCV_OK;
}

mcv_status mcv_assembly_add(mcv_assembly a, const mcv_shape* shape, const mcv_material* mat,
                            const mcv_kernel* kernels, int32_t nk, int32_t* idx) {
  if (!a || !shape || !mat || (nk > 0 && !kernels)) return fail(MCV_EINVAL, "null argument");
  if (nk < 0) return fail(MCV_EINVAL, "negative kernel count");
  if (a->scat.size() >= (size_t)kMaxScat) return fail(MCV_EUNSUPPORTED, "at most 4 scatterers");
  if (nk > kMaxKern) return fail(MCV_EUNSUPPORTED, "at most 3 kernels per scatterer");
  mcv_status st = check_shape(*shape);
  if (st != MCV_OK) return st;
  if (!(mat->n_per_A3 >= 0.0) || !(mat->sigma_abs_b >= 0.0) || !std::isfinite(mat->n_per_A3) ||
      !std::isfinite(mat->sigma_abs_b))
    return fail(MCV_EINVAL, "material needs n >= 0 and sigma_abs >= 0");
  bool has_phonon = false, wants_dw = false;
  for (int j = 0; j < nk; ++j) {
    if ((st = check_kernel(kernels[j])) != MCV_OK) return st;
    has_phonon |= kernels[j].type == MCV_K_PHONON;
    wants_dw |= kernels[j].dw == 1;
  }
  if (wants_dw && !has_phonon)
    return fail(MCV_EINVAL, "a Debye-Waller factor needs a phonon kernel in the same scatterer");
  int nphon = 0;
  for (int j = 0; j < nk; ++j) nphon += kernels[j].type == MCV_K_PHONON;
  if (nphon > 1) return fail(MCV_EUNSUPPORTED, "at most one phonon kernel per scatterer");
  int slots = intervals_of(*shape);
  for (auto& s : a->scat) slots += intervals_of(s.shape);
  if (slots > 7) return fail(MCV_EUNSUPPORTED, "more than 7 material intervals per ray");
  for (auto& s : a->scat)
    if (!disjoint(s.shape, *shape))
      return fail(MCV_EOVERLAP, "scatterer volume may overlap an existing scatterer");
  Scatterer sc;
  sc.shape = *shape;
  sc.mat = *mat;
  for (int j = 0; j < nk; ++j) {
    KernelCopy kc;
    kc.k = kernels[j];
    const mcv_kernel& k = kernels[j];
    if (k.type == MCV_K_POWDER) {
      kc.d.assign(k.d, k.d + k.nrefl);
      kc.F2.assign(k.F2, k.F2 + k.nrefl);
    } else if (k.type == MCV_K_PHONON || k.type == MCV_K_MULTIPHONON) {
      kc.dos.assign(k.dos, k.dos + k.nbins);
    } else if (k.type == MCV_K_SQE) {
      kc.sqe.assign(k.sqe, k.sqe + (size_t)k.nQ * k.nE);
    } else if (k.type == MCV_K_COH_PHONON) {
      kc.modes.assign(k.modes, k.modes + (size_t)12 * k.grid_n * k.grid_n * k.grid_n);
    }
    kc.k.d = kc.k.F2 = kc.k.dos = kc.k.sqe = kc.k.modes = nullptr;
    sc.kernels.push_back(std::move(kc));
  }
  a->scat.push_back(std::move(sc));
  if (idx) *idx = (int32_t)a->scat.size() - 1;
  return MCV_OK;
}

mcv_status mcv_detector_sphere(mcv_detector* out, double R, int32_t n_2theta, int32_t n_tof,
                               double tof_lo, double tof_hi) {
  if (!out) return fail(MCV_EINVAL, "null output handle");
  if (!(R > 0.0) || n_2theta < 1 || n_tof < 1 || !(tof_hi > tof_lo) || !std::isfinite(tof_lo) ||
      !std::isfinite(tof_hi))
    return fail(MCV_EINVAL, "sphere detector needs R > 0, bins >= 1, tof_hi > tof_lo");
  if ((int64_t)n_2theta * n_tof >= kMaxBins)
    return fail(MCV_EUNSUPPORTED, "histogram too large: n_2theta * n_tof must stay below 2^31");
  auto* d = new (std::nothrow) mcv_detector_s();
  if (!d) return fail(MCV_ENOMEM, "host allocation failed");
  d->type = DET_SPHERE;
  d->R = R;
  d->n2t = n_2theta;
  d->ntof = n_tof;
  d->tof_lo = tof_lo;
  d->tof_hi = tof_hi;
  *out = d;
  return MCV_OK;
}

mcv_status mcv_detector_tubes(mcv_detector* out, const mcv_tube_layout* L, int32_t n_pix,
                              int32_t n_tof, double tof_lo, double tof_hi) {
  if (!out || !L) return fail(MCV_EINVAL, "null argument");
  if (L->nrows < 1 || L->nrows > kMaxRows || L->ncols < 1 || n_pix < 1 || n_tof < 1)
    return fail(MCV_EINVAL, "tube layout needs 1..8 rows, >= 1 column, pixel and tof bins");
  if (!(L->R > 0.0) || !(L->radius > 0.0) || !(L->length > 0.0) || !(L->n_he >= 0.0) ||
      !(L->phi_hi > L->phi_lo) || !(tof_hi > tof_lo))
    return fail(MCV_EINVAL, "tube layout needs R, radius, length > 0, phi_hi > phi_lo");
  if (L->R < 10.0 * L->radius) return fail(MCV_EUNSUPPORTED, "tube circle radius must be >= 10 tube radii");
  if (L->tubes_per_pack < 0 || (L->tubes_per_pack > 0 && L->ncols % L->tubes_per_pack != 0) ||
      (L->tubes_per_pack > 0 && !(L->pack_gap >= 0.0)))
    return fail(MCV_EINVAL, "tubes per pack must divide the columns, with a gap >= 0");
  const double dphi = tube_pitch(*L);
  if (!(dphi > 0.0)) return fail(MCV_EINVAL, "pack gaps leave no room for the tubes");
  if (L->ncols > 1 && 2.0 * L->R * std::sin(0.5 * dphi) < 2.0 * L->radius)
    return fail(MCV_EINVAL, "neighbouring tubes overlap");
  if (L->phi_hi - L->phi_lo > 2.0 * kPi) return fail(MCV_EINVAL, "tube columns span more than 2 pi");
  for (int r = 1; r < L->nrows; ++r)
    if (!(L->row_y[r] - L->row_y[r - 1] >= L->length))
      return fail(MCV_EINVAL, "rows must be ascending and must not overlap");
  // bins are 32-bit indices on the device (histogram updates, bin cache
  // tags, event pixels)
  if ((int64_t)L->nrows * L->ncols * n_pix * n_tof >= kMaxBins)
    return fail(MCV_EUNSUPPORTED, "histogram too large: nrows * ncols * n_pix * n_tof must stay below 2^31");
  auto* d = new (std::nothrow) mcv_detector_s();
  if (!d) return fail(MCV_ENOMEM, "host allocation failed");
  d->type = DET_TUBES;
  d->R = L->R;
  d->npix = n_pix;
  d->ntof = n_tof;
  d->tof_lo = tof_lo;
  d->tof_hi = tof_hi;
  d->tubes = *L;
  *out = d;
  return MCV_OK;
}

int64_t mcv_detector_nbins(mcv_detector d) {
  if (!d) return -1;
  if (d->type == DET_SPHERE) return (int64_t)d->n2t * d->ntof;
  return (int64_t)d->tubes.nrows * d->tubes.ncols * d->npix * d->ntof;
}

mcv_status mcv_detector_destroy(mcv_detector d) {
  delete d;
  return MCV_OK;
}

mcv_status mcv_plan_create(mcv_plan* out, mcv_assembly a, mcv_detector d, const mcv_opts* opts,
                           int32_t device) {
  if (!out || !a || !d) return fail(MCV_EINVAL, "null argument");
  *out = nullptr;
  mcv_opts o = {};
  o.max_orders = 1;
  if (opts) o = *opts;
  if (o.max_orders < 0 || o.max_orders > kMaxOrders) return fail(MCV_EUNSUPPORTED, "max_orders must be 0..7");
  if (!(o.min_prob >= 0.0)) return fail(MCV_EINVAL, "min_prob must be >= 0");
  if (o.max_waves < 0) return fail(MCV_EINVAL, "max_waves must be >= 0");
  if (o.deterministic != 0 && o.deterministic != 1) return fail(MCV_EINVAL, "deterministic must be 0 or 1");
  int block = o.block_size ? o.block_size : 256;
  if (block < 64 || block > 256 || block % 64) return fail(MCV_EINVAL, "block_size must be 64, 128, 192 or 256");

  auto p = new (std::nothrow) mcv_plan_s();
  if (!p) return fail(MCV_ENOMEM, "host allocation failed");
  std::memset(&p->host, 0, sizeof(DevPlan));
  DevPlan& P = p->host;
  std::vector<float>& T = p->tables;
  // mode tables of coherent phonon kernels, uploaded to device memory below
  std::vector<std::pair<DevKernel*, std::vector<float>>> grids;
  P.nscat = (int)a->scat.size();
  P.K = o.max_orders;
  P.min_prob = (float)o.min_prob;
  int smax = 0;
  double brad = 0.0;
  for (int s = 0; s < P.nscat; ++s) {
    const Scatterer& sc = a->scat[s];
    DevScat& S = P.s[s];
    smax += intervals_of(sc.shape);
    brad = std::max(brad, bounding_radius(sc.shape));
    S.shape = sc.shape.type;
    S.nk = (int)sc.kernels.size();
    if (sc.shape.type == MCV_SHAPE_BOX) {
      for (int i = 0; i < 3; ++i) S.h[i] = (float)(0.5 * sc.shape.dims[i]);
    } else if (sc.shape.type == MCV_SHAPE_CYLINDER) {
      S.h[0] = (float)sc.shape.dims[0];
      S.h[1] = (float)(0.5 * sc.shape.dims[1]);
    } else {
      S.h[0] = (float)sc.shape.dims[0];
      S.h[1] = (float)sc.shape.dims[1];
      S.h[2] = (float)(0.5 * sc.shape.dims[2]);
    }
    for (int i = 0; i < 3; ++i) S.pos[i] = (float)sc.shape.pos[i];
    for (int i = 0; i < 9; ++i) S.rot[i] = (float)sc.shape.rot[i];
    S.ident = 1;
    for (int i = 0; i < 9; ++i) S.ident &= S.rot[i] == (i % 4 == 0 ? 1.0f : 0.0f);
    S.mu_abs2200 = (float)(100.0 * sc.mat.n_per_A3 * sc.mat.sigma_abs_b * 2200.0);
    S.n100 = (float)(100.0 * sc.mat.n_per_A3);
    // Debye-Waller coefficient from the scatterer's phonon DOS:
    // 2W/Q^2 = hbar^2/2M * gamma_0, gamma_0 = int coth(E/2kT) Z(E)/E dE
    double dw = 0.0;
    for (const KernelCopy& kc : sc.kernels) {
      if (kc.k.type != MCV_K_PHONON) continue;
      const int nb = kc.k.nbins;
      const double de = kc.k.emax / nb;
      double area = 0.0;
      for (double v : kc.dos) area += v * de;
      double g0 = 0.0;
      for (int b = 0; b < nb; ++b) {
        const double e = (b + 0.5) * de;
        g0 += kc.dos[b] / area / e * de / std::tanh(e / (2.0 * kBoltzmann * kc.k.T_K));
      }
      dw = kHbar2over2mn * kNeutronMassAmu / kc.k.M_amu * g0;
    }
    S.dw_coef = (float)dw;
    for (int j = 0; j < S.nk; ++j) {
      const KernelCopy& kc = sc.kernels[j];
      const mcv_kernel& k = kc.k;
      DevKernel& K = S.k[j];
      K.type = k.type;
      K.dw = k.dw;
      K.mu = (float)(100.0 * sc.mat.n_per_A3 * k.sigma_b);
      if (k.type == MCV_K_POWDER) {
        std::vector<int> idx(k.nrefl);
        std::iota(idx.begin(), idx.end(), 0);
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return kc.d[x] > kc.d[y]; });
        K.nrefl = k.nrefl;
        K.t_d = (int)T.size();
        for (int i : idx) T.push_back((float)kc.d[i]);
        K.t_pref = (int)T.size();
        double acc = 0.0;
        for (int i : idx) {
          acc += kc.d[i] * kc.F2[i];
          T.push_back((float)acc);
        }
        K.bragg_coef = (float)(100.0 / (2.0 * k.v0 * k.v0));
      } else if (k.type == MCV_K_PHONON) {
        K.nbins = k.nbins;
        K.t_cdf = (int)T.size();
        double tot = 0.0;
        for (double v : kc.dos) tot += v;
        double acc = 0.0;
        for (int b = 0; b < k.nbins; ++b) {
          acc += kc.dos[b];
          T.push_back(b == k.nbins - 1 ? 1.0f : (float)(acc / tot));
        }
        K.de = (float)(k.emax / k.nbins);
        K.kT = (float)(kBoltzmann * k.T_K);
        K.h2m = (float)(kHbar2over2mn * kNeutronMassAmu / k.M_amu);
      } else if (k.type == MCV_K_MULTIPHONON) {
        // One-phonon spectrum A_1 on 2 nbins bins over [-emax, emax] of the
        // energy the neutron loses (bin nbins + b: loss in [b de, (b+1) de];
        // bin nbins - 1 - b: the same gain), midpoint rule on the DOS bins:
        // Z_b de / (e_b gamma_0) times n(e_b) + 1 for a loss and n(e_b) for
        // a gain, n the Bose occupation; the masses sum to 1 because
        // 2n + 1 = coth(e/2kT).  Stored as a cumulative table.
        const int nb = k.nbins;
        const double de = k.emax / nb, kT = kBoltzmann * k.T_K;
        double area = 0.0;
        for (double v : kc.dos) area += v * de;
        double g0 = 0.0;
        for (int b = 0; b < nb; ++b) {
          const double e = (b + 0.5) * de;
          g0 += kc.dos[b] / area / e * de / std::tanh(e / (2.0 * kT));
        }
        std::vector<double> mass(2 * (size_t)nb);
        for (int b = 0; b < nb; ++b) {
          const double e = (b + 0.5) * de;
          const double occ = 1.0 / std::expm1(e / kT);
          const double base = kc.dos[b] / area * de / (e * g0);
          mass[nb + b] = base * (occ + 1.0);
          mass[nb - 1 - b] = base * occ;
        }
        double tot = 0.0;
        for (double v : mass) tot += v;
        K.t_cdf = (int)T.size();
        double acc = 0.0;
        for (int j = 0; j < 2 * nb; ++j) {
          acc += mass[j];
          T.push_back(j == 2 * nb - 1 ? 1.0f : (float)(acc / tot));
        }
        K.nbins = nb;
        K.de = (float)de;
        K.kT = (float)kT;
        K.h2m = (float)(kHbar2over2mn * kNeutronMassAmu / k.M_amu);
        K.dw_self = (float)(kHbar2over2mn * kNeutronMassAmu / k.M_amu * g0);
        K.nmax = k.max_phonons;
      } else if (k.type == MCV_K_SPINWAVE || k.type == MCV_K_DISPERSION) {
        K.j4s = (float)(4.0 * k.J * k.S);
        K.wmax = (float)(24.0 * k.J * k.S);
        K.a = (float)k.a;
        K.gamma = (float)k.gamma;
        for (int i = 0; i < 9; ++i) K.crot[i] = (float)k.crot[i];
      } else if (k.type == MCV_K_COH_PHONON) {
        const int n = k.grid_n;
        K.nbins = n;
        K.kT = (float)(kBoltzmann * k.T_K);
        K.h2m = (float)(kHbar2over2mn * kNeutronMassAmu / k.M_amu);
        double emax = 0.0;
        std::vector<float> g(kc.modes.size());
        for (size_t i = 0; i < kc.modes.size(); ++i) {
          g[i] = (float)kc.modes[i];
          if (i % 12 < 3) emax = std::max(emax, kc.modes[i]);
        }
        K.wmax = (float)emax;
        for (int i = 0; i < 9; ++i) K.crot[i] = (float)(k.cell[i] * n / (2.0 * kPi));
        grids.push_back({&K, std::move(g)});
      } else if (k.type == MCV_K_SQE) {
        K.t_s = (int)T.size();
        for (double v : kc.sqe) T.push_back((float)v);
        K.nQ = k.nQ;
        K.nE = k.nE;
        K.Qmax = (float)k.Qmax;
        K.Emin = (float)k.Emin;
        K.Emax = (float)k.Emax;
        K.q_scale = (float)(k.nQ / k.Qmax);
        K.e_scale = (float)(k.nE / (k.Emax - k.Emin));
      }
    }
  }
  P.smax = smax;
  P.stack_cap = smax > 1 ? (smax - 1) * P.K : 0;

  DevDet& D = P.det;
  D.type = d->type;
  D.ntof = d->ntof;
  D.tof_lo = (float)d->tof_lo;
  D.inv_dt = (float)(d->ntof / (d->tof_hi - d->tof_lo));
  D.R = (float)d->R;
  if (d->type == DET_SPHERE) {
    if (brad > 0.5 * d->R) {
      delete p;
      return fail(MCV_EUNSUPPORTED, "sample must lie within half the sphere radius");
    }
    D.n2t = d->n2t;
    D.ring_scale = (float)(d->n2t / kPi);
  } else {
    const mcv_tube_layout& L = d->tubes;
    if (brad > 0.05 * L.R) {
      delete p;
      return fail(MCV_EUNSUPPORTED, "sample must lie within 5% of the tube circle radius");
    }
    D.nrows = L.nrows;
    D.ncols = L.ncols;
    D.npix = d->npix;
    D.phi_lo = (float)L.phi_lo;
    D.inv_dphi = (float)(L.ncols / (L.phi_hi - L.phi_lo));
    D.tpp = L.tubes_per_pack;
    D.pack_pitch = (float)(L.tubes_per_pack * tube_pitch(L) + L.pack_gap);
    D.inv_pack_pitch = (float)(1.0 / (L.tubes_per_pack * tube_pitch(L) + L.pack_gap));
    D.inv_tube_pitch = (float)(1.0 / tube_pitch(L));
    for (int r = 0; r < L.nrows; ++r) D.row_y[r] = (float)L.row_y[r];
    D.half_len = (float)(0.5 * L.length);
    D.radius = (float)L.radius;
    D.mu_he2200 = (float)(100.0 * L.n_he * kHe3SigmaAbs * 2200.0);
    D.pix_scale = (float)(d->npix / L.length);
    D.t_cols = (int)T.size();
    for (int c = 0; c < L.ncols; ++c) {
      const double phi = column_azimuth(L, c);
      T.push_back((float)(L.R * std::sin(phi)));
      T.push_back((float)(L.R * std::cos(phi)));
    }
  }
  P.n_tables = (int)T.size();
  if (T.empty()) T.push_back(0.0f);
  // pixel centres for the (Q, E) reduction, in binary64: tube pixels on the
  // tube axis at the pixel's mid height, sphere rings at their centre angle
  std::vector<float> G;
  if (d->type == DET_SPHERE) {
    for (int i = 0; i < d->n2t; ++i) {
      G.push_back((float)d->R);
      G.push_back((float)std::cos((i + 0.5) * kPi / d->n2t));
    }
  } else {
    const mcv_tube_layout& L = d->tubes;
    for (int r = 0; r < L.nrows; ++r)
      for (int c = 0; c < L.ncols; ++c) {
        const double phi = column_azimuth(L, c);
        const double x = L.R * std::sin(phi), z = L.R * std::cos(phi);
        for (int j = 0; j < d->npix; ++j) {
          const double y = L.row_y[r] - 0.5 * L.length + (j + 0.5) * L.length / d->npix;
          const double L2 = std::sqrt(x * x + y * y + z * z);
          G.push_back((float)L2);
          G.push_back((float)(z / L2));
        }
      }
  }
  p->nbins = mcv_detector_nbins(d);
  p->R = d->R;
  p->tof_lo = d->tof_lo;
  p->tof_hi = d->tof_hi;

  // LDS: plan + tables + bin cache + per-lane stack + detection queues
  const int dq_n = transport_dq_entries(P);
  const int stack_lds = 0;  // transport launches keep their packet stacks in device memory
  size_t lds_dyn = transport_lds_bytes(P.n_tables, stack_lds, block, kLdsNoAdjoint, kHotMin) +
                   transport_dq_bytes(block, dq_n, false);
  while (lds_dyn + transport_static_lds() > 160 * 1024 && block > 64) {
    block -= 64;
    lds_dyn = transport_lds_bytes(P.n_tables, stack_lds, block, kLdsNoAdjoint, kHotMin) +
              transport_dq_bytes(block, dq_n, false);
  }
  if (lds_dyn + transport_static_lds() > 160 * 1024) {
    delete p;
    return fail(MCV_EUNSUPPORTED, "tables and packet stack exceed the 160 KiB of LDS");
  }
  P.hot_n = hot_slots(transport_static_lds() +
                          transport_lds_bytes(P.n_tables, stack_lds, block, kLdsNoAdjoint, 0) +
                          transport_dq_bytes(block, dq_n, false),
                      block, transport_waves_per_eu(P.nscat, P.smax));
  P.hot_all = mcv_detector_nbins(d) <= kHotAllBins ? 1 : 0;
  P.heavy = 0;
  for (int si = 0; si < P.nscat; ++si)
    for (int j = 0; j < P.s[si].nk; ++j)
      P.heavy |= P.s[si].k[j].type == K_DISPERSION || P.s[si].k[j].type == K_COH_PHONON;
  p->block = block;
  p->device = device;
  p->scat = a->scat;
  p->waves_per_simd = o.waves_per_simd > 0 ? o.waves_per_simd : kGridDepth;
  p->max_waves = o.max_waves;
  p->deterministic = o.deterministic;

  hipError_t e;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if ((e = hipSetDevice(device)) != hipSuccess) {
    delete p;
    return hipfail(e, "hipSetDevice");
  }
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  p->cus = cus > 0 ? cus : 256;
  if ((e = set_transport_lds_limit(160 * 1024)) != hipSuccess) {
    (void)hipSetDevice(cur);
    delete p;
    return hipfail(e, "hipFuncSetAttribute");
  }
  // the static workspace of mcv_adjoint_noalloc on this device
  if ((e = adjoint_scratch_setup(device)) != hipSuccess) {
    (void)hipSetDevice(cur);
    delete p;
    return hipfail(e, "hipGetSymbolAddress");
  }
  if ((e = hipMalloc(&p->d_plan, sizeof(DevPlan))) != hipSuccess ||
      (e = hipMalloc(&p->d_tables, T.size() * sizeof(float))) != hipSuccess ||
      (e = hipMalloc(&p->d_pixgeo, G.size() * sizeof(float))) != hipSuccess) {
    if (p->d_plan) (void)hipFree(p->d_plan);
    if (p->d_tables) (void)hipFree(p->d_tables);
    (void)hipSetDevice(cur);
    delete p;
    return fail(MCV_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  for (auto& gk : grids) {
    float* dg = nullptr;
    if ((e = hipMalloc(&dg, gk.second.size() * sizeof(float))) == hipSuccess) p->d_grids.push_back(dg);
    if (e != hipSuccess || (e = hipMemcpy(dg, gk.second.data(), gk.second.size() * sizeof(float),
                                          hipMemcpyHostToDevice)) != hipSuccess) {
      for (float* x : p->d_grids) (void)hipFree(x);
      (void)hipFree(p->d_plan);
      (void)hipFree(p->d_tables);
      (void)hipFree(p->d_pixgeo);
      (void)hipSetDevice(cur);
      delete p;
      return hipfail(e, "mode table upload");
    }
    gk.first->grid_lo = (uint32_t)(uintptr_t)dg;
    gk.first->grid_hi = (uint32_t)((uintptr_t)dg >> 32);
  }
  if ((e = hipMemcpy(p->d_plan, &P, sizeof(DevPlan), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->d_tables, T.data(), T.size() * sizeof(float), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(p->d_pixgeo, G.data(), G.size() * sizeof(float), hipMemcpyHostToDevice)) !=
          hipSuccess) {
    for (float* x : p->d_grids) (void)hipFree(x);
    (void)hipFree(p->d_plan);
    (void)hipFree(p->d_tables);
    (void)hipFree(p->d_pixgeo);
    (void)hipSetDevice(cur);
    delete p;
    return hipfail(e, "hipMemcpy");
  }
  // binary64 table parameters of the adjoint (one-phonon DOS, S(Q,E) grids)
  {
    std::vector<double> raw;
    for (int si = 0; si < kMaxScat; ++si)
      for (int j = 0; j < kMaxKern; ++j) p->raw_off[si][j] = -1;
    for (size_t si = 0; si < p->scat.size(); ++si)
      for (size_t j = 0; j < p->scat[si].kernels.size(); ++j) {
        const KernelCopy& kc = p->scat[si].kernels[j];
        const std::vector<double>* v = kc.k.type == MCV_K_PHONON ? &kc.dos
                                       : kc.k.type == MCV_K_SQE  ? &kc.sqe
                                                                 : nullptr;
        if (!v) continue;
        p->raw_off[si][j] = (int64_t)raw.size();
        raw.insert(raw.end(), v->begin(), v->end());
      }
    if (!raw.empty()) {
      if ((e = hipMalloc(&p->d_raw, raw.size() * sizeof(double))) != hipSuccess ||
          (e = hipMemcpy(p->d_raw, raw.data(), raw.size() * sizeof(double),
                         hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipSetDevice(cur);
        mcv_plan_destroy(p);
        return hipfail(e, "adjoint table upload");
      }
    }
  }
  if (p->deterministic) {
    // key = bin (31 bits) | id - chunk first | lineage (3K + 1 bits: a child
    // of lineage L is 8 L + g + 1, g < 7); entries <= histories x packets
    // per history <= chunk x sum_{j <= K} smax^j
    p->det_lin_bits = 3 * P.K + 1;
    p->det_id_bits = 64 - 31 - p->det_lin_bits;
    uint64_t maxpk = 0, pw = 1;
    for (int j = 0; j <= P.K; ++j, pw *= (uint64_t)std::max(1, P.smax)) maxpk += pw;
    uint64_t chunk = (uint64_t)1 << 16;
    chunk = std::min<uint64_t>(chunk, (uint64_t)1 << p->det_id_bits);
    chunk = std::max<uint64_t>(1, std::min<uint64_t>(chunk, ((uint64_t)1 << 22) / maxpk));
    p->det_chunk = chunk;
    p->det_cap = chunk * maxpk;
    size_t tb = 0;
    e = det_sort(nullptr, &tb, nullptr, nullptr, nullptr, nullptr, p->det_cap, 64, nullptr);
    p->sort_tmp_bytes = tb;
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
      e = hipMalloc(&p->d_keys[i], p->det_cap * sizeof(uint64_t));
      if (e == hipSuccess) e = hipMalloc(&p->d_vals[i], p->det_cap * sizeof(float));
    }
    if (e == hipSuccess) e = hipMalloc(&p->d_sort_tmp, std::max<size_t>(tb, 16));
    if (e == hipSuccess) e = hipMalloc(&p->d_det_n, sizeof(unsigned long long));
    if (e != hipSuccess) {
      (void)hipSetDevice(cur);
      mcv_plan_destroy(p);
      return hipfail(e, "deterministic summation workspace");
    }
  }
  if (P.stack_cap > 0) {
    // stacks of every wave of the largest grid (grid_shape: cus x 4 x
    // waves_per_simd x 2 waves), adjoint fields included; with the default
    // depth, a shallower grid for plans whose stacks would pass 2 GiB
    auto stack_bytes = [&](int depth) {
      return ((size_t)p->cus * 4 * depth * 2 + (size_t)block / 64) * 64 * (size_t)P.stack_cap *
             stack_words(true) * sizeof(float);
    };
    if (o.waves_per_simd <= 0)
      while (p->waves_per_simd > kGridDepthMin && stack_bytes(p->waves_per_simd) > ((size_t)2 << 30))
        p->waves_per_simd /= 2;
    const size_t waves = (size_t)p->cus * 4 * p->waves_per_simd * 2 + (size_t)block / 64;
    p->stack_floats = waves * 64 * (size_t)P.stack_cap * stack_words(true);
    if ((e = hipMalloc(&p->d_stack, p->stack_floats * sizeof(float))) != hipSuccess) {
      (void)hipSetDevice(cur);
      mcv_plan_destroy(p);
      return hipfail(e, "packet stack allocation");
    }
  }
  (void)hipSetDevice(cur);
  *out = p;
  return MCV_OK;
}

mcv_status mcv_plan_destroy(mcv_plan p) {
  if (!p) return MCV_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(p->device);
  (void)hipFree(p->d_plan);
  (void)hipFree(p->d_tables);
  (void)hipFree(p->d_pixgeo);
  for (float* x : p->d_grids) (void)hipFree(x);
  if (p->adj.ws) (void)hipFree(p->adj.ws);
  if (p->d_raw) (void)hipFree(p->d_raw);
  if (p->d_stack) (void)hipFree(p->d_stack);
  for (int i = 0; i < 2; ++i) {
    if (p->d_keys[i]) (void)hipFree(p->d_keys[i]);
    if (p->d_vals[i]) (void)hipFree(p->d_vals[i]);
  }
  if (p->d_sort_tmp) (void)hipFree(p->d_sort_tmp);
  if (p->d_det_n) (void)hipFree(p->d_det_n);
  (void)hipSetDevice(cur);
  delete p;
  return MCV_OK;
}

int64_t mcv_plan_nbins(mcv_plan p) { return p ? p->nbins : -1; }

}  // extern "C"

namespace {

mcv_status make_beam(const mcv_plan_s* p, const mcv_beam* b, DevBeam* out) {
  if (!b) return fail(MCV_EINVAL, "null beam");
  if (b->type == MCV_BEAM_SAVED) {
    if (!b->saved || b->n_saved == 0) return fail(MCV_EINVAL, "saved beam needs rows and n_saved > 0");
    *out = DevBeam{};
    out->type = b->type;
    out->saved = b->saved;
    out->n_saved = b->n_saved;
    return MCV_OK;
  }
  if (b->type != MCV_BEAM_MONO && b->type != MCV_BEAM_GAUSS) return fail(MCV_EINVAL, "unknown beam type");
  if (!(b->E > 0.0) || !std::isfinite(b->E)) return fail(MCV_EINVAL, "beam energy must be > 0");
  if (!(b->W >= 0.0) || !(b->H >= 0.0) || !std::isfinite(b->W) || !std::isfinite(b->H))
    return fail(MCV_EINVAL, "beam size must be >= 0");
  if (!(b->z0 < 0.0) || std::fabs(b->z0) > 0.05 * p->R)
    return fail(MCV_EINVAL, "beam start z0 must be negative and within 5% of the detector radius");
  if (std::hypot(0.5 * b->W, 0.5 * b->H) > 0.05 * p->R) return fail(MCV_EINVAL, "beam too wide for the detector");
  if (b->type == MCV_BEAM_GAUSS && !(b->sigma_rel >= 0.0 && b->sigma_rel <= 0.2))
    return fail(MCV_EINVAL, "sigma_rel must be in [0, 0.2]");
  *out = DevBeam{};
  out->type = b->type;
  out->E = (float)b->E;
  out->sigma_rel = (float)b->sigma_rel;
  out->W = (float)b->W;
  out->H = (float)b->H;
  out->z0 = (float)b->z0;
  return MCV_OK;
}

// history ids [first, first + n) against the limits of the beam
mcv_status check_ids(const DevBeam& B, uint64_t first, uint64_t n) {
  if (n > ((uint64_t)1 << 62) || first > ((uint64_t)1 << 62) - n)
    return fail(MCV_EINVAL, "history ids must stay below 2^62");
  if (B.type == MCV_BEAM_SAVED && (first > B.n_saved || n > B.n_saved - first))
    return fail(MCV_EINVAL, "history ids must stay below the number of saved neutrons");
  return MCV_OK;
}

// Waves of a launch: each takes a contiguous id range.  At least two rounds
// of the 4 resident waves per SIMD (when there are 64 histories per wave),
// then up to cus x 4 x waves_per_simd x 2 waves, in whole rounds, while
// each keeps at least kMinPerWave histories: shorter ranges shorten the tail
// where the last waves run alone, and each workgroup pays to stage the plan
// and flush its bin cache.  Measured (ms; depth 4 / 8 / 16 / 24, i.e. 2 to 12 rounds):
// crystal in its can 1e8 79.1 / 75.7 / 73.5 / 73.0, powder 1e7 1.33 / 1.23
// / 1.20 / 1.41, exact-delta crystal 1e7 24.6 / 23.6 / 24.0 / 24.6, plate
// 1e9 31.8 / 30.1 / 28.9 / 28.5.  shallow: at most two rounds (event
// launches: every wave's last, partial stage of events is one more atomic
// on the single event counter; powder 1e7 events 1.63 ms at the default
// depth, 1.52 ms at 4).
void grid_shape(const mcv_plan_s* p, uint64_t n, int block, uint64_t* grid, uint64_t* per_wave,
                bool shallow = false) {
  const uint64_t waves_per_block = (uint64_t)block / 64;
  // one round: the waves resident at once at 4 per SIMD
  const uint64_t round = (uint64_t)p->cus * 4 * kGridDepthMin;
  uint64_t target = (uint64_t)p->cus * 4 * (shallow ? std::min(p->waves_per_simd, kGridDepthMin)
                                                    : p->waves_per_simd) * 2;
  // whole rounds only: a partial last round is a tail of its own (exact-delta
  // crystal 1e7: 24.5 ms on 4.77 rounds, 23.6 ms on 4)
  const uint64_t by_work = n / kMinPerWave / round * round;
  if (target > 2 * round) target = std::max(2 * round, std::min(target, by_work));
  if (p->max_waves > 0 && (uint64_t)p->max_waves < target) target = (uint64_t)p->max_waves;
  uint64_t waves = (n + 63) / 64;
  if (waves > target) waves = target;
  *per_wave = (n + waves - 1) / waves;
  waves = (n + *per_wave - 1) / *per_wave;
  *grid = (waves + waves_per_block - 1) / waves_per_block;
}

mcv_status launch(mcv_plan p, const mcv_beam* beam, uint64_t seed, uint64_t first, uint64_t n,
                  double* hist, double* hist_w2, DevRecord* rec, uint64_t cap,
                  unsigned long long* n_out, void* stream, DevEvent* ev = nullptr,
                  uint64_t ev_cap = 0, unsigned long long* n_ev = nullptr) {
  DevBeam B;
  mcv_status st = make_beam(p, beam, &B);
  if (st != MCV_OK) return st;
  if ((st = check_ids(B, first, n)) != MCV_OK) return st;
  if (n == 0) return MCV_OK;
  uint64_t grid, per_wave;
  grid_shape(p, n, p->block, &grid, &per_wave, ev != nullptr);
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != p->device) (void)hipSetDevice(p->device);
  if (p->d_stack && grid * p->block * (size_t)p->host.stack_cap * stack_words(false) > p->stack_floats)
    return fail(MCV_EUNSUPPORTED, "packet stacks exceed their buffer");
  hipError_t e = launch_transport(p->d_plan, p->host, p->d_tables, B,
                                  seed, first, n, (int)grid, p->block, per_wave, hist, hist_w2,
                                  rec, cap, n_out, ev, ev_cap, n_ev, nullptr, p->d_stack, nullptr,
                                  nullptr, (hipStream_t)stream);
  if (cur != p->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return hipfail(e, "transport launch");
  return MCV_OK;
}

}  // namespace

extern "C" {

// Deterministic summation (plan option): chunks of det_chunk histories in id
// order; per chunk the transport writes (key, value) entries, the host reads
// their number (the stream is synchronised once per chunk), the entries are
// sorted by key and every bin's run is summed in key order and added.
static mcv_status run_deterministic(mcv_plan p, const mcv_beam* beam, uint64_t seed,
                                    uint64_t first,
                                    uint64_t n, double* hist, double* hist_w2,
                                    hipStream_t stream) {
  DevBeam B;
  mcv_status st = make_beam(p, beam, &B);
  if (st != MCV_OK) return st;
  if ((st = check_ids(B, first, n)) != MCV_OK) return st;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != p->device) (void)hipSetDevice(p->device);
  const int shift = p->det_id_bits + p->det_lin_bits;
  for (uint64_t cf = first; cf < first + n && st == MCV_OK; cf += p->det_chunk) {
    const uint64_t m = std::min<uint64_t>(p->det_chunk, first + n - cf);
    uint64_t grid, per_wave;
    grid_shape(p, m, p->block, &grid, &per_wave);
    if (p->d_stack && grid * p->block * (size_t)p->host.stack_cap * stack_words(false) > p->stack_floats) {
      st = fail(MCV_EUNSUPPORTED, "packet stacks exceed their buffer");
      break;
    }
    DetArgs D = {p->d_keys[0], p->d_vals[0], p->det_cap, p->d_det_n, cf, p->det_lin_bits,
                 p->det_id_bits};
    hipError_t e = det_zero(p->d_det_n, stream);
    if (e == hipSuccess)
      e = launch_transport(p->d_plan, p->host, p->d_tables, B, seed, cf, m, (int)grid, p->block,
                           per_wave, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0, nullptr,
                           nullptr, p->d_stack, &D, nullptr, stream);
    unsigned long long count = 0;
    if (e == hipSuccess)
      e = hipMemcpyAsync(&count, p->d_det_n, sizeof(count), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      st = hipfail(e, "deterministic transport");
      break;
    }
    if (count > p->det_cap) {
      st = fail(MCV_ECAPACITY, "deterministic entries exceed their bound");
      break;
    }
    size_t tb = p->sort_tmp_bytes;
    e = det_sort(p->d_sort_tmp, &tb, p->d_keys[0], p->d_keys[1], p->d_vals[0], p->d_vals[1], count,
                 31 + shift, stream);
    if (e == hipSuccess) e = det_sums(p->d_keys[1], p->d_vals[1], count, shift, hist, hist_w2, stream);
    if (e != hipSuccess) st = hipfail(e, "deterministic summation");
  }
  if (cur != p->device) (void)hipSetDevice(cur);
  return st;
}

mcv_status mcv_run(mcv_plan p, const mcv_beam* beam, uint64_t seed, uint64_t first, uint64_t n,
                   double* hist, double* hist_w2, void* stream) {
  if (!p) return fail(MCV_EINVAL, "null plan");
  if (!hist) return fail(MCV_EINVAL, "null histogram");
  if (p->deterministic)
    return run_deterministic(p, beam, seed, first, n, hist, hist_w2, (hipStream_t)stream);
  return launch(p, beam, seed, first, n, hist, hist_w2, nullptr, 0, nullptr, stream);
}

mcv_status mcv_trace(mcv_plan p, const mcv_beam* beam, uint64_t seed, uint64_t first, uint64_t n,
                     double* hist, mcv_packet_record* records, uint64_t capacity,
                     uint64_t* n_out_dev, void* stream) {
  static_assert(sizeof(mcv_packet_record) == sizeof(DevRecord), "record layout");
  if (!p) return fail(MCV_EINVAL, "null plan");
  if (!records || !n_out_dev) return fail(MCV_EINVAL, "null record buffer or counter");
  return launch(p, beam, seed, first, n, hist, nullptr, reinterpret_cast<DevRecord*>(records),
                capacity, reinterpret_cast<unsigned long long*>(n_out_dev), stream);
}

mcv_status mcv_run_events(mcv_plan p, const mcv_beam* beam, uint64_t seed, uint64_t first,
                          uint64_t n, double* hist, double* hist_w2, mcv_event* events,
                          uint64_t capacity, uint64_t* n_events_dev, void* stream) {
  static_assert(sizeof(mcv_event) == sizeof(DevEvent), "event layout");
  if (!p) return fail(MCV_EINVAL, "null plan");
  if (!events || !n_events_dev) return fail(MCV_EINVAL, "null event buffer or counter");
  if (p->nbins > (int64_t)0xFFFFFFFF)
    return fail(MCV_EUNSUPPORTED, "event mode needs fewer than 2^32 detector bins");
  return launch(p, beam, seed, first, n, hist, hist_w2, nullptr, 0, nullptr, stream,
                reinterpret_cast<DevEvent*>(events), capacity,
                reinterpret_cast<unsigned long long*>(n_events_dev));
}

}  // extern "C"

namespace {

mcv_status make_qe_map(const mcv_plan_s* p, const mcv_qe_grid* g, QEMap* M) {
  if (!g) return fail(MCV_EINVAL, "null grid");
  if (!(g->Ei > 0.0) || !std::isfinite(g->Ei)) return fail(MCV_EINVAL, "reduction needs Ei > 0");
  if (g->nq < 1 || g->ne < 1 || (int64_t)g->nq * g->ne > ((int64_t)1 << 31) - 1)
    return fail(MCV_EINVAL, "grid needs nq, ne >= 1 and fewer than 2^31 bins");
  if (!(g->q_hi > g->q_lo) || !(g->e_hi > g->e_lo) || !std::isfinite(g->q_lo) ||
      !std::isfinite(g->q_hi) || !std::isfinite(g->e_lo) || !std::isfinite(g->e_hi))
    return fail(MCV_EINVAL, "grid needs finite q_lo < q_hi, e_lo < e_hi");
  const DevDet& D = p->host.det;
  const double ki = std::sqrt(g->Ei / kHbar2over2mn);
  M->Ei = (float)g->Ei;
  M->ki2 = (float)(ki * ki);
  M->two_ki = (float)(2.0 * ki);
  M->e_per_v2 = (float)kEperV2;
  M->k_per_v = (float)std::sqrt(kEperV2 / kHbar2over2mn);
  M->q_lo = (float)g->q_lo;
  M->q_scale = (float)(g->nq / (g->q_hi - g->q_lo));
  M->e_lo = (float)g->e_lo;
  M->e_scale = (float)(g->ne / (g->e_hi - g->e_lo));
  M->nq = g->nq;
  M->ne = g->ne;
  M->ntof = D.ntof;
  M->tof_lo = (float)p->tof_lo;
  M->dt = (float)((p->tof_hi - p->tof_lo) / D.ntof);
  M->npixels = (uint32_t)(p->nbins / D.ntof);
  M->pad = 0;
  return MCV_OK;
}

int reduce_grid(const mcv_plan_s* p, uint64_t work_items, uint64_t per_block) {
  const uint64_t blocks = (work_items + per_block - 1) / per_block;
  const uint64_t cap = (uint64_t)p->cus * 8;
  return (int)(blocks < 1 ? 1 : blocks < cap ? blocks : cap);
}

}  // namespace

extern "C" {

mcv_status mcv_reduce_qe(mcv_plan p, const mcv_qe_grid* grid, const double* hist,
                         const double* hist_w2, double* iqe, double* iqe_w2, void* stream) {
  if (!p || !hist || !iqe) return fail(MCV_EINVAL, "null plan, histogram or output");
  if (p->nbins / p->host.det.ntof > (int64_t)0xFFFFFFFF)
    return fail(MCV_EUNSUPPORTED, "reduction needs fewer than 2^32 pixels");
  if (((uintptr_t)hist & 15u) != 0 || ((uintptr_t)hist_w2 & 15u) != 0)
    return fail(MCV_EINVAL, "histograms must be 16-byte aligned");
  QEMap M;
  mcv_status st = make_qe_map(p, grid, &M);
  if (st != MCV_OK) return st;
  const int g = reduce_grid(p, (uint64_t)p->nbins, (uint64_t)reduce_tile_bins());
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != p->device) (void)hipSetDevice(p->device);
  hipError_t e = launch_reduce_hist(p->d_pixgeo, M, hist, hist_w2, (uint64_t)p->nbins,
                                    iqe, iqe_w2, g, p->cus, (hipStream_t)stream);
  if (cur != p->device) (void)hipSetDevice(cur);
  return e == hipSuccess ? MCV_OK : hipfail(e, "reduction launch");
}

mcv_status mcv_reduce_events_qe(mcv_plan p, const mcv_qe_grid* grid, const mcv_event* events,
                                const uint64_t* n_events_dev, uint64_t capacity, double* iqe,
                                double* iqe_w2, void* stream) {
  if (!p || !events || !n_events_dev || !iqe)
    return fail(MCV_EINVAL, "null plan, events, counter or output");
  if (p->nbins / p->host.det.ntof > (int64_t)0xFFFFFFFF)
    return fail(MCV_EUNSUPPORTED, "reduction needs fewer than 2^32 pixels");
  QEMap M;
  mcv_status st = make_qe_map(p, grid, &M);
  if (st != MCV_OK) return st;
  if (capacity == 0) return MCV_OK;
  const int g = reduce_grid(p, capacity, 256);
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != p->device) (void)hipSetDevice(p->device);
  hipError_t e = launch_reduce_events(
      p->d_pixgeo, M, reinterpret_cast<const DevEvent*>(events),
      reinterpret_cast<const unsigned long long*>(n_events_dev), capacity, iqe, iqe_w2, g,
      (hipStream_t)stream);
  if (cur != p->device) (void)hipSetDevice(cur);
  return e == hipSuccess ? MCV_OK : hipfail(e, "reduction launch");
}

mcv_status mcv_sync(void* stream) {
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hipfail(e, "hipStreamSynchronize");
  e = hipGetLastError();
  if (e != hipSuccess) return hipfail(e, "pending device error");
  return MCV_OK;
}

}  // extern "C"

namespace {

const double kBoltzmannA = 0.08617333;

// The parameter map resolved against a plan: table sizes, the scalars of the
// DOS kernel for the device-side table preparation, and the LDS layout.
struct AdjSetup {
  int nb = 0, nc = 0;
  double de = 1.0, kT = 1.0, h2m = 0.0;
  const double* theta = nullptr;  // device
  const double* cells = nullptr;  // device
  int block = 0;
  int sparse_lds = 1;
};

mcv_status check_param_map(mcv_plan p, const mcv_param_map* pm, AdjSetup* out) {
  if (!pm) return fail(MCV_EINVAL, "null parameter map");
  const int ns = (int)p->scat.size();
  auto kernel_of = [&](int si, int k) -> const KernelCopy* {
    if (si < 0 || si >= ns || k < 0 || k >= (int)p->scat[si].kernels.size()) return nullptr;
    return &p->scat[si].kernels[k];
  };
  AdjSetup A;
  int per_event = 0;  // most table indices one kernel draw adds to a packet
  if (pm->dos_scatterer != -1) {
    const KernelCopy* kd = kernel_of(pm->dos_scatterer, pm->dos_kernel);
    if (!kd || kd->k.type != MCV_K_PHONON)
      return fail(MCV_EINVAL, "dos_scatterer/dos_kernel must name a one-phonon kernel (or -1)");
    A.nb = kd->k.nbins;
    A.de = kd->k.emax / kd->k.nbins;
    A.kT = kBoltzmannA * kd->k.T_K;
    A.h2m = kHbar2over2mn * kNeutronMassAmu / kd->k.M_amu;
    A.theta = p->d_raw + p->raw_off[pm->dos_scatterer][pm->dos_kernel];
    per_event = 1;
    if (pm->multiphonon_kernel != -1) {
      const KernelCopy* km = kernel_of(pm->dos_scatterer, pm->multiphonon_kernel);
      if (!km || km->k.type != MCV_K_MULTIPHONON)
        return fail(MCV_EINVAL, "multiphonon_kernel must name a multi-phonon kernel of dos_scatterer");
      if (km->k.nbins != kd->k.nbins || km->k.emax != kd->k.emax || km->k.T_K != kd->k.T_K ||
          km->k.M_amu != kd->k.M_amu || km->dos != kd->dos)
        return fail(MCV_EINVAL,
                    "a tied multi-phonon kernel needs the DOS values, emax, M and T of the one-phonon kernel");
      per_event = std::max(per_event, km->k.max_phonons);
    }
  } else if (pm->multiphonon_kernel != -1) {
    return fail(MCV_EINVAL, "multiphonon_kernel needs dos_scatterer/dos_kernel");
  }
  if (pm->sqe_scatterer != -1) {
    const KernelCopy* kq = kernel_of(pm->sqe_scatterer, pm->sqe_kernel);
    if (!kq || kq->k.type != MCV_K_SQE)
      return fail(MCV_EINVAL, "sqe_scatterer/sqe_kernel must name an S(Q,E) kernel (or -1)");
    A.nc = kq->k.nQ * kq->k.nE;
    A.cells = p->d_raw + p->raw_off[pm->sqe_scatterer][pm->sqe_kernel];
    per_event = std::max(per_event, 1);
  }
  if (A.nb + A.nc > kAdjMaxTable)
    return fail(MCV_EUNSUPPORTED, "adjoint supports up to 65535 table parameters (DOS bins + S(Q,E) cells)");
  if (pm->abs_scatterer < -1 || pm->abs_scatterer >= ns)
    return fail(MCV_EINVAL, "abs_scatterer out of range");
  if (pm->sigma_scatterer < -1 || pm->sigma_scatterer >= ns)
    return fail(MCV_EINVAL, "sigma_scatterer out of range");
  if (pm->sigma_scatterer >= 0) {
    const KernelCopy* ks = kernel_of(pm->sigma_scatterer, pm->sigma_kernel);
    if (!ks || ks->k.type == MCV_K_POWDER || !(ks->k.sigma_b > 0.0))
      return fail(MCV_EINVAL, "sigma_kernel must name a non-powder kernel with sigma > 0");
  }
  if ((int64_t)p->host.K * per_event > kAdjMaxSparse)
    return fail(MCV_EUNSUPPORTED,
                "a packet would carry more than 12 table indices (max_orders x phonons per draw)");
  // LDS: table partials when they fit beside tables and packet stacks with a
  // workgroup of at least 128 lanes, otherwise global atomics per entry
  const size_t lim = (size_t)160 * 1024 - transport_static_lds();
  const int dq_n = transport_dq_entries(p->host);
  auto lds = [&](int block, int ntab) {
    return transport_lds_bytes(p->host.n_tables, 0, block, ntab, 0) +
           transport_dq_bytes(block, dq_n, true);
  };
  int block = p->block;
  while (block > 128 && lds(block, A.nb + A.nc) > lim) block -= 64;
  if (lds(block, A.nb + A.nc) > lim) {
    A.sparse_lds = 0;
    block = p->block;
    while (block > 64 && lds(block, 0) > lim) block -= 64;
    if (lds(block, 0) > lim) return fail(MCV_EUNSUPPORTED, "adjoint packet stacks do not fit in LDS");
  }
  A.block = block;
  if (out) *out = A;
  return MCV_OK;
}

// the kernels' view of a checked parameter map
AdjArgs adj_args(const mcv_param_map* pm, const AdjSetup& A, const double* dL_dI, double* grad,
                 double* ws) {
  AdjArgs AA = {};
  AA.dos_s = A.nb > 0 ? pm->dos_scatterer : -1;
  AA.dos_k = pm->dos_kernel;
  AA.mp_k = A.nb > 0 ? pm->multiphonon_kernel : -1;
  AA.sqe_s = A.nc > 0 ? pm->sqe_scatterer : -1;
  AA.sqe_k = pm->sqe_kernel;
  AA.abs_s = pm->abs_scatterer;
  AA.sig_s = pm->sigma_scatterer;
  AA.sig_k = pm->sigma_kernel;
  AA.nb = A.nb;
  AA.nc = A.nc;
  AA.sparse_lds = A.sparse_lds;
  AA.dLdI = dL_dI;
  AA.grad = grad;
  AA.ws = ws;
  return AA;
}

// the plan-owned binary64 workspace of the adjoint (allocated on first use,
// grown when a map needs more); device of the plan current
mcv_status adjoint_workspace(mcv_plan p, const AdjSetup& A) {
  const size_t need = 4 + 2 * (size_t)A.nb + (size_t)A.nc;
  if (p->adj.cap >= need) return MCV_OK;
  if (p->adj.ws) (void)hipFree(p->adj.ws);
  p->adj.ws = nullptr;
  p->adj.cap = 0;
  if (hipMalloc(&p->adj.ws, need * sizeof(double)) != hipSuccess)
    return fail(MCV_ENOMEM, "hipMalloc adjoint workspace");
  p->adj.cap = need;
  return MCV_OK;
}

// the workspace the adjoint kernels use: prepare -> transport -> finalize
mcv_status adjoint_launch(mcv_plan p, const mcv_param_map* pm, const AdjSetup& A,
                          const DevBeam& B, uint64_t seed, uint64_t first, uint64_t n,
                          const double* dL_dI, double* grad, double* ws, hipStream_t stream) {
  hipError_t e = launch_adjoint_prepare(A.theta, A.nb, A.de, A.kT, A.h2m, A.cells, A.nc, ws, stream);
  if (e == hipSuccess && n > 0) {
    const AdjArgs AA = adj_args(pm, A, dL_dI, grad, ws);
    uint64_t grid, per_wave;
    grid_shape(p, n, A.block, &grid, &per_wave);
    if (p->d_stack &&
        grid * A.block * (size_t)p->host.stack_cap * stack_words(true) > p->stack_floats)
      return fail(MCV_EUNSUPPORTED, "packet stacks exceed their buffer");
    e = launch_transport(p->d_plan, p->host, p->d_tables, B, seed, first, n, (int)grid, A.block,
                         per_wave, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0, nullptr, &AA,
                         p->d_stack, nullptr, nullptr, stream);
  }
  if (e == hipSuccess) e = launch_adjoint_finalize(grad, ws, A.nb, A.nc, stream);
  if (e != hipSuccess) return hipfail(e, "adjoint launch");
  return MCV_OK;
}

}  // namespace

extern "C" {

int64_t mcv_adjoint_nparams(mcv_plan p, const mcv_param_map* pm) {
  AdjSetup A;
  if (!p || check_param_map(p, pm, &A) != MCV_OK) return -1;
  return (int64_t)A.nb + A.nc + 2;
}

mcv_status mcv_adjoint(mcv_plan p, const mcv_param_map* pm, const mcv_beam* beam, uint64_t seed,
                       uint64_t first, uint64_t n, const double* dL_dI, double* grad,
                       void* stream) {
  if (!p) return fail(MCV_EINVAL, "null plan");
  AdjSetup A;
  mcv_status st = check_param_map(p, pm, &A);
  if (st != MCV_OK) return st;
  if (!dL_dI || !grad) return fail(MCV_EINVAL, "null dL_dI or grad");
  DevBeam B;
  if ((st = make_beam(p, beam, &B)) != MCV_OK) return st;
  if ((st = check_ids(B, first, n)) != MCV_OK) return st;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != p->device) (void)hipSetDevice(p->device);
  st = adjoint_workspace(p, A);
  if (st == MCV_OK)
    st = adjoint_launch(p, pm, A, B, seed, first, n, dL_dI, grad, p->adj.ws, (hipStream_t)stream);
  if (cur != p->device) (void)hipSetDevice(cur);
  return st;
}

mcv_status mcv_run_tape(mcv_plan p, const mcv_param_map* pm, const mcv_beam* beam, uint64_t seed,
                        uint64_t first, uint64_t n, double* hist, double* hist_w2, uint32_t* tape,
                        uint64_t capacity, uint64_t* n_tape_dev, void* stream) {
  static_assert(MCV_TAPE_FIELDS == kTapeFields, "tape layout");
  if (!p) return fail(MCV_EINVAL, "null plan");
  AdjSetup A;
  mcv_status st = check_param_map(p, pm, &A);
  if (st != MCV_OK) return st;
  if (!tape || !n_tape_dev) return fail(MCV_EINVAL, "null tape or counter");
  if (((uintptr_t)tape & 3u) || ((uintptr_t)n_tape_dev & 7u))
    return fail(MCV_EINVAL, "tape must be 4-byte and its counter 8-byte aligned");
  if (p->nbins > (int64_t)0xFFFFFFFF)
    return fail(MCV_EUNSUPPORTED, "the tape needs fewer than 2^32 detector bins");
  DevBeam B;
  if ((st = make_beam(p, beam, &B)) != MCV_OK) return st;
  if ((st = check_ids(B, first, n)) != MCV_OK) return st;
  if (n == 0) return MCV_OK;
  // LDS: tables, the histogram bin cache and the detection queues with the
  // carry
  const size_t lim = (size_t)160 * 1024 - transport_static_lds();
  const int dq_n = transport_dq_entries(p->host);
  auto lds = [&](int b) {
    return transport_lds_bytes(p->host.n_tables, 0, b, kLdsNoAdjoint, p->host.hot_n) +
           transport_dq_bytes(b, dq_n, true);
  };
  int block = p->block;
  while (block > 64 && lds(block) > lim) block -= 64;
  if (lds(block) > lim) return fail(MCV_EUNSUPPORTED, "tape run does not fit in LDS");
  uint64_t grid, per_wave;
  grid_shape(p, n, block, &grid, &per_wave);
  if (p->d_stack &&
      grid * block * (size_t)p->host.stack_cap * stack_words(true) > p->stack_floats)
    return fail(MCV_EUNSUPPORTED, "packet stacks exceed their buffer");
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != p->device) (void)hipSetDevice(p->device);
  const AdjArgs AA = adj_args(pm, A, nullptr, nullptr, nullptr);
  const TapeArgs T = {tape, capacity, reinterpret_cast<unsigned long long*>(n_tape_dev)};
  const hipError_t e = launch_transport(p->d_plan, p->host, p->d_tables, B, seed, first, n,
                                        (int)grid, block, per_wave, hist, hist_w2, nullptr, 0,
                                        nullptr, nullptr, 0, nullptr, &AA, p->d_stack, nullptr, &T,
                                        (hipStream_t)stream);
  if (cur != p->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return hipfail(e, "tape run launch");
  return MCV_OK;
}

}  // extern "C"

namespace {

// prepare -> pass over the tape -> dense terms; dL_dI null: the weighted
// least squares form (I, T, w, loss)
mcv_status tape_backward(mcv_plan p, const mcv_param_map* pm, const uint32_t* tape,
                         uint64_t capacity, const uint64_t* n_tape_dev, const double* dL_dI,
                         const double* I, const double* T, const double* w, double* loss,
                         double* grad, void* stream) {
  AdjSetup A;
  mcv_status st = check_param_map(p, pm, &A);
  if (st != MCV_OK) return st;
  if (((uintptr_t)tape & 3u) || ((uintptr_t)n_tape_dev & 7u))
    return fail(MCV_EINVAL, "tape must be 4-byte and its counter 8-byte aligned");
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != p->device) (void)hipSetDevice(p->device);
  st = adjoint_workspace(p, A);
  if (st == MCV_OK) {
    double* ws = p->adj.ws;
    const hipStream_t s = (hipStream_t)stream;
    hipError_t e =
        launch_adjoint_prepare(A.theta, A.nb, A.de, A.kT, A.h2m, A.cells, A.nc, ws, s);
    if (e == hipSuccess)
      e = launch_tape_adjoint(tape, capacity,
                              reinterpret_cast<const unsigned long long*>(n_tape_dev), dL_dI, I, T,
                              w, loss, A.nb, A.nc, grad, ws, p->cus * 4, s);
    if (e == hipSuccess) e = launch_adjoint_finalize(grad, ws, A.nb, A.nc, s);
    if (e != hipSuccess) st = hipfail(e, "tape adjoint launch");
  }
  if (cur != p->device) (void)hipSetDevice(cur);
  return st;
}

}  // namespace

extern "C" {

mcv_status mcv_adjoint_tape(mcv_plan p, const mcv_param_map* pm, const uint32_t* tape,
                            uint64_t capacity, const uint64_t* n_tape_dev, const double* dL_dI,
                            double* grad, void* stream) {
  if (!p) return fail(MCV_EINVAL, "null plan");
  if (!tape || !n_tape_dev || !dL_dI || !grad)
    return fail(MCV_EINVAL, "null tape, counter, dL_dI or grad");
  return tape_backward(p, pm, tape, capacity, n_tape_dev, dL_dI, nullptr, nullptr, nullptr,
                       nullptr, grad, stream);
}

mcv_status mcv_adjoint_tape_wl2(mcv_plan p, const mcv_param_map* pm, const uint32_t* tape,
                                uint64_t capacity, const uint64_t* n_tape_dev, const double* I,
                                const double* T, const double* w, double* loss, double* grad,
                                void* stream) {
  if (!p) return fail(MCV_EINVAL, "null plan");
  if (!tape || !n_tape_dev || !I || !T || !w || !loss || !grad)
    return fail(MCV_EINVAL, "null tape, counter, I, T, w, loss or grad");
  return tape_backward(p, pm, tape, capacity, n_tape_dev, nullptr, I, T, w, loss, grad, stream);
}

mcv_status mcv_adjoint_noalloc(mcv_plan p, const mcv_param_map* pm, const mcv_beam* beam,
                               uint64_t seed, uint64_t first, uint64_t n, const double* dL_dI,
                               double* grad, void* stream) {
  if (!p) return fail(MCV_EINVAL, "null plan");
  AdjSetup A;
  mcv_status st = check_param_map(p, pm, &A);
  if (st != MCV_OK) return st;
  if (!dL_dI || !grad) return fail(MCV_EINVAL, "null dL_dI or grad");
  if (4 + 2 * (int64_t)A.nb + A.nc > kNoAllocWorkDoubles)
    return fail(MCV_ECAPACITY, "mcv_adjoint_noalloc: 4 + 2 DOS bins + S(Q,E) cells exceeds the "
                               "32768 values of its static workspace");
  DevBeam B;
  if ((st = make_beam(p, beam, &B)) != MCV_OK) return st;
  if ((st = check_ids(B, first, n)) != MCV_OK) return st;
  double* ws = adjoint_scratch(p->device);
  if (!ws) return fail(MCV_EHIP, "static adjoint workspace not set up on this device");
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != p->device) (void)hipSetDevice(p->device);
  st = adjoint_launch(p, pm, A, B, seed, first, n, dL_dI, grad, ws, (hipStream_t)stream);
  if (cur != p->device) (void)hipSetDevice(cur);
  return st;
}

mcv_status mcv_loss_grad(const double* I, const double* T, const double* w, int64_t n,
                         double* dL_dI, double* loss, void* stream) {
  if (!I || !T || !w || !dL_dI || !loss || n < 0) return fail(MCV_EINVAL, "bad loss arguments");
  if (((uintptr_t)I | (uintptr_t)T | (uintptr_t)w | (uintptr_t)dL_dI) & 15u)
    return fail(MCV_EINVAL, "loss arrays must be 16-byte aligned");
  if (n == 0) return MCV_OK;
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int64_t grid = (n / 2 + 255) / 256;
  if (grid > (int64_t)cus * 64) grid = (int64_t)cus * 64;
  if (grid < 1) grid = 1;
  hipError_t e = launch_loss_grad(I, T, w, n, dL_dI, loss, (int)grid, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(e, "loss launch");
  return MCV_OK;
}

mcv_status mcv_zero(double* p, int64_t n, void* stream) {
  if (n < 0 || (n > 0 && !p)) return fail(MCV_EINVAL, "bad zero arguments");
  if ((uintptr_t)p & 7u) return fail(MCV_EINVAL, "array must be 8-byte aligned");
  if (n == 0) return MCV_OK;
  // one 16-byte store per lane (larger arrays loop)
  int64_t grid = (n / 2 + 255) / 256;
  if (grid > ((int64_t)1 << 30)) grid = (int64_t)1 << 30;
  if (grid < 1) grid = 1;
  hipError_t e = launch_fill_zero(p, (uint64_t)n, (int)grid, (hipStream_t)stream);
  if (e != hipSuccess) return hipfail(e, "zero launch");
  return MCV_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
namespace mcv {
hipError_t launch_batch(const BatchItem* items, const BatchChunk* chunks, uint32_t n_chunks,
                        uint32_t* cursor, double* const* zero_ptrs, const uint64_t* zero_sizes,
                        int n_zero, int grid, int block, size_t lds, int hot_n, int dq_off,
                        float* gstack, int stack_max, bool heavy, hipStream_t stream);
int batch_occupancy(int block, size_t lds, bool heavy);
}  // namespace mcv

struct mcv_batch_s {
  int device = 0;
  BatchItem* d_items = nullptr;
  BatchChunk* d_chunks = nullptr;
  uint32_t* d_cursor = nullptr;
  uint32_t n_chunks = 0;
  int n_zero = 0;
  int grid = 0, block = 0;
  size_t lds = 0;
  int hot_n = kHotMin;
  int dq_off = 0;  // words from the start of dynamic LDS to the detection queues
  float* d_stack = nullptr;  // packet stacks of the resident workgroups (device memory)
  int stack_max = 0;
  bool heavy = false;  // some plan has an exact-delta or coherent-phonon kernel
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void batch_free(mcv_batch_s* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_chunks) (void)hipFree(b->d_chunks);
  if (b->d_cursor) (void)hipFree(b->d_cursor);
  if (b->d_stack) (void)hipFree(b->d_stack);
  delete b;
}

// relative cost of one history of a plan: packets per history grow with the
// order bound and the intervals per ray; the tube detector is dearer
double history_cost(const mcv_plan_s* p) {
  const double packets = 1.0 + p->host.K * std::max(1, p->host.smax);
  return packets * (p->host.det.type == DET_TUBES ? 1.6 : 1.0);
}

}  // namespace

extern "C" {

mcv_status mcv_batch_create(mcv_batch* out, const mcv_batch_item* items, int32_t n,
                            const mcv_tuning* tuning, int32_t device) {
  if (!out || !items || n < 1) return fail(MCV_EINVAL, "batch needs at least one item");
  *out = nullptr;
  mcv_tuning t = {0, 0, 0, 1};
  if (tuning) t = *tuning;
  int block = t.block_size ? t.block_size : 256;
  if (block < 64 || block > 256 || block % 64) return fail(MCV_EINVAL, "block_size must be 64..256, multiple of 64");
  const uint64_t chunk = t.chunk > 0 ? (uint64_t)t.chunk : 4096;
  if (chunk > 0xFFFFFFFFull) return fail(MCV_EINVAL, "chunk too large");
  std::vector<BatchItem> hitems(n);
  std::vector<std::pair<double, BatchChunk>> hchunks;
  std::vector<double*> zp;
  std::vector<uint64_t> zs;
  int n_tables_max = 0, stack_max = 0, dq_max = 0;
  bool heavy = false;
  for (int i = 0; i < n; ++i) {
    const mcv_batch_item& it = items[i];
    if (!it.plan || !it.hist) return fail(MCV_EINVAL, "batch item needs a plan and a histogram");
    if (it.plan->device != device) return fail(MCV_EINVAL, "batch item plan is on another device");
    DevBeam B;
    mcv_status st = make_beam(it.plan, &it.beam, &B);
    if (st != MCV_OK) return st;
    if ((st = check_ids(B, it.first, it.n)) != MCV_OK) return st;
    hitems[i].plan = it.plan->d_plan;
    hitems[i].tables = it.plan->d_tables;
    hitems[i].beam = B;
    hitems[i].seed = it.seed;
    hitems[i].id0 = it.first;
    hitems[i].hist = it.hist;
    n_tables_max = std::max(n_tables_max, it.plan->host.n_tables);
    heavy = heavy || it.plan->host.heavy != 0;
    stack_max = std::max(stack_max, it.plan->host.stack_cap);
    dq_max = std::max(dq_max, batch_dq_entries(it.plan->host));
    const double c = history_cost(it.plan);
    for (uint64_t f = 0; f < it.n; f += chunk) {
      BatchChunk ch;
      ch.item = (uint32_t)i;
      ch.first = f;
      ch.count = (uint32_t)std::min<uint64_t>(chunk, it.n - f);
      hchunks.push_back({c * ch.count, ch});
    }
    if (t.zero_hists) {
      zp.push_back(it.hist);
      zs.push_back((uint64_t)it.plan->nbins);
    }
  }
  if (hchunks.empty()) return fail(MCV_EINVAL, "batch has no histories");
  std::stable_sort(hchunks.begin(), hchunks.end(),
                   [](const auto& a, const auto& b) { return a.first > b.first; });
  std::vector<BatchChunk> cl;
  for (auto& c : hchunks) cl.push_back(c.second);
  // dynamic LDS: bin cache, largest tables, then the waves' detection queues
  // (the largest any item uses); the packet stacks live in device memory
  size_t lds = transport_lds_bytes(n_tables_max, 0, block, kLdsNoAdjoint, kHotMin) +
               transport_dq_bytes(block, dq_max, false);
  while (lds + transport_static_lds() + 64 > 160 * 1024 && block > 64) {
    block -= 64;
    lds = transport_lds_bytes(n_tables_max, 0, block, kLdsNoAdjoint, kHotMin) +
          transport_dq_bytes(block, dq_max, false);
  }
  if (lds + transport_static_lds() + 64 > 160 * 1024)
    return fail(MCV_EUNSUPPORTED, "batch tables exceed LDS");
  const int hot_n = hot_slots(transport_static_lds() + 64 +
                                  transport_lds_bytes(n_tables_max, 0, block, kLdsNoAdjoint, 0) +
                                  transport_dq_bytes(block, dq_max, false),
                              block, batch_waves_per_eu());
  const size_t lds_q = transport_lds_bytes(n_tables_max, 0, block, kLdsNoAdjoint, hot_n);
  lds = lds_q + transport_dq_bytes(block, dq_max, false);

  auto* b = new (std::nothrow) mcv_batch_s();
  if (!b) return fail(MCV_ENOMEM, "host allocation failed");
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(device);
  b->device = device;
  b->block = block;
  b->lds = lds;
  b->hot_n = hot_n;
  b->dq_off = (int)(lds_q / sizeof(float));
  b->n_chunks = (uint32_t)cl.size();
  b->n_zero = (int)zp.size();
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  b->heavy = heavy;
  int occ = batch_occupancy(block, lds, heavy);
  if (occ < 1) occ = 1;
  if (t.wgs_per_cu > 0) occ = std::min(occ, (int)t.wgs_per_cu);
  b->grid = std::max(1, std::min<int>(cus * occ, (int)cl.size()));
  hipError_t e = hipSuccess;
  auto up = [&](void** dst, const void* src, size_t bytes) {
    if (e != hipSuccess) return;
    if ((e = hipMalloc(dst, std::max<size_t>(bytes, 8))) != hipSuccess) return;
    if (bytes) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  b->stack_max = stack_max;
  if (stack_max > 0 && e == hipSuccess)
    e = hipMalloc(&b->d_stack, (size_t)b->grid * block * stack_max * stack_words(false) * sizeof(float));
  up((void**)&b->d_items, hitems.data(), hitems.size() * sizeof(BatchItem));
  up((void**)&b->d_chunks, cl.data(), cl.size() * sizeof(BatchChunk));
  uint32_t zero = 0;
  up((void**)&b->d_cursor, &zero, sizeof(uint32_t));
  if (e != hipSuccess) {
    batch_free(b);
    (void)hipSetDevice(cur);
    return hipfail(e, "batch upload");
  }
  // capture reset + persistent kernel once; runs replay the graph
  if ((e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking)) == hipSuccess &&
      (e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal)) == hipSuccess) {
    hipError_t el = launch_batch(b->d_items, b->d_chunks, b->n_chunks, b->d_cursor, zp.data(),
                                 zs.data(), b->n_zero, b->grid, b->block, b->lds, b->hot_n,
                                 b->dq_off, b->d_stack, b->stack_max, b->heavy, b->capture);
    e = hipStreamEndCapture(b->capture, &b->graph);
    if (e == hipSuccess) e = el;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  }
  (void)hipSetDevice(cur);
  if (e != hipSuccess) {
    batch_free(b);
    return hipfail(e, "batch graph capture");
  }
  *out = b;
  return MCV_OK;
}

mcv_status mcv_batch_run(mcv_batch b, void* stream) {
  if (!b) return fail(MCV_EINVAL, "null batch");
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != b->device) (void)hipSetDevice(b->device);
  hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
  if (cur != b->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return hipfail(e, "hipGraphLaunch");
  return MCV_OK;
}

mcv_status mcv_batch_destroy(mcv_batch b) {
  if (!b) return MCV_OK;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(b->device);
  batch_free(b);
  (void)hipSetDevice(cur);
  return MCV_OK;
}

mcv_status mcv_autotune(const mcv_batch_item* items, int32_t n, int32_t device, int32_t reps,
                        mcv_tuning* best, double* best_ms) {
  if (!items || n < 1 || !best) return fail(MCV_EINVAL, "autotune needs items and an output");
  if (reps < 1) reps = 3;
  const int blocks[] = {64, 128, 192, 256};
  const int chunks[] = {1024, 4096, 16384, 65536};
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(device);
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipSetDevice(cur);
    return hipfail(e, "autotune setup");
  }
  double best_t = 1e300;
  mcv_tuning bt = {256, 4096, 0, 1};
  mcv_status st = MCV_OK;
  for (int bl : blocks) {
    for (int ck : chunks) {
      mcv_tuning t = {bl, ck, 0, 1};
      mcv_batch b = nullptr;
      st = mcv_batch_create(&b, items, n, &t, device);
      if (st != MCV_OK) break;
      (void)mcv_batch_run(b, s);  // warm
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps; ++r) (void)mcv_batch_run(b, s);
      (void)hipEventRecord(e1, s);
      e = hipEventSynchronize(e1);
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      mcv_batch_destroy(b);
      if (e != hipSuccess) {
        st = hipfail(e, "autotune run");
        break;
      }
      const double per = ms / reps;
      if (per < best_t) {
        best_t = per;
        bt = t;
      }
    }
    if (st != MCV_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  (void)hipSetDevice(cur);
  if (st != MCV_OK) return st;
  *best = bt;
  if (best_ms) *best_ms = best_t;
  return MCV_OK;
}

}  // extern "C"
