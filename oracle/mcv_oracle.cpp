// mcv_oracle.cpp -- serial FP64 CPU oracle for weighted neutron-packet transport.
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
// GPU path is checked against.  Only the test-suite, the smoke check and the
// CPU-baseline leg of the benchmark may load it.  It shares no code, header,
// constant or table generator with the GPU library: every constant and every
// formula below is written out here on its own.
//
// What it computes (arXiv:1504.02776, "MCViNE"):
//   * ray tracing through a composite of homogeneous scatterers: intersect the
//     forward ray with every shape, walk the material intervals in order
//     (Sec. 2.4.3 "Ray Tracing");
//   * packet splitting: at every material interval the packet is split into a
//     transmitted part (weight times the attenuation e^{-mu L}) and a scattered
//     part born at a random point of the interval, with a randomly chosen
//     kernel (Sec. 2.4.3 "Multiple Scattering"; Supplement S3, interactM1);
//   * multiple scattering as repeated splitting of scattered packets up to a
//     maximum order, leftovers leaving with attenuation only (Supplement S3,
//     scatterM / interactM_path1);
//   * the scattering kernels of Supplement S4: incoherent elastic, powder
//     Bragg (Debye-Scherrer cones), incoherent one-phonon from a DOS, and a
//     dispersion surface E(Q) with S(Q); plus a tabulated isotropic S(Q,E)
//     (Sec. 2.4.2, kernel "S(Q,omega) histogram");
//   * detection on a sphere or on 3He tubes: chord through the tube, MC
//     absorption point, weight times absorption probability, pixel from the
//     axial position, time of flight (Sec. 2.4.3 "Ray tracing in a detector
//     system");
//   * intensity per (pixel, tof) bin = sum of packet probabilities (Sec. 3,
//     four-step workflow, "Reduction").
//
// Where the paper is silent the readings are the ones listed in the design
// notes (forced-collision point on a segment, implicit capture, 1/v
// absorption, per-packet order count, nearest interceptor, and so on); each is
// restated at the place it is used.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11), keyed by the 64-bit seed, with the
// counter (id_lo, id_hi | stream<<30, lineage, block).  Every random decision
// of a packet is a fixed word of a fixed block, so the traversal order of the
// packet tree does not change any result.
//
// Decision margins: for every discrete decision the oracle records how far
// the continuous quantity was from the decision boundary, divided by a stated
// uncertainty scale.  Packets with a margin below 1 are "near-decision" in the
// parity tests (a single-precision implementation may legitimately take the
// other branch there).
//
// Reading guide: lines and helpers marked [bookkeeping] carry those margins
// and the binary32 conditioning of each packet (the uncertainties the parity
// bars are built from); `tally->` lines count primitives for the work model.
// Neither changes what the method computes: skip both to read the method
// against the paper.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// ---------------------------------------------------------------- constants
// CODATA 2018 values, restated independently of any other source file.
const double kEperV2 = 5.22703759e-6;     // E[meV] = kEperV2 * v[m/s]^2
const double kHbar2over2mn = 2.0721249;   // E[meV] = kHbar2over2mn * k[1/A]^2
const double kBoltzmann = 0.08617333;     // meV / K
const double kNeutronMassAmu = 1.00866491595;
const double kV2200 = 2200.0;             // reference speed for sigma_abs
const double kHe3SigmaAbs = 5333.0;       // barn at 2200 m/s
const double kSurfaceEps = 1e-7;          // m; intervals ending closer are behind
const double kHuge = 1e30;                // stands for an unbounded interval end
const double kPi = 3.14159265358979323846;

// uncertainty scales used to normalise decision margins
const double kTauRel = 2e-5;     // relative, for sums of cross sections etc.
const double kTauGeom = 2e-6;    // m, for geometric distances near a surface
const double kTauCos = 2e-6;     // in cos(2theta), sphere rings
const double kTauTof = 4e-6;     // relative time of flight
const double kTauImpact = 4e-4;  // relative impact parameter in a tube
const double kTauU = 2e-6;       // absolute, for u < p tests on computed p
const double kTauJ = 5e-2;       // |dG/dE_f| of a delta-function root (tangency)
const double kTauDk = 1e-4;      // relative uncertainty of a delta-function root
// Conditioning of a single-precision implementation (reported, not used by
// the method): a position of ~1 cm is known to ~3e-9 m in binary32 (half an
// ulp, 4.7e-10 m, per coordinate from each of the roundings of a birth point
// -- entry point, x d, and their sum -- plus the squared radius of the next
// shape test, whose cancellation near a surface adds about as much), which
// makes a chord L uncertain by 3e-9 m / |cos| at each surface it crosses.
const double kEpsPos = 3e-9;

inline double k_from_speed(double v) { return v * std::sqrt(kEperV2 / kHbar2over2mn); }
inline double speed_from_k(double k) { return k * std::sqrt(kHbar2over2mn / kEperV2); }

// ----------------------------------------------------------------- ABI types
// (mirrored by ctypes in oracle.py)
enum { SHAPE_BOX = 1, SHAPE_CYLINDER = 2, SHAPE_ANNULUS = 3 };
enum { K_ISO_EL = 1, K_POWDER = 2, K_PHONON = 3, K_SPINWAVE = 4, K_SQE = 5, K_MULTIPHONON = 6,
       K_DISPERSION = 7, K_COH_PHONON = 8 };
enum { BEAM_MONO = 1, BEAM_GAUSS = 2, BEAM_SAVED = 3 };
enum { DET_SPHERE = 1, DET_TUBES = 2 };
enum { STREAM_SOURCE = 0, STREAM_SCATTER = 1, STREAM_DETECT = 2 };

}  // namespace

extern "C" {

struct OShape {
  int32_t type;
  int32_t pad;
  double dims[3];  // BOX: full x,y,z; CYLINDER: r,h,-; ANNULUS: r_in,r_out,h
  double pos[3];   // lab position of the shape centre, m
  double rot[9];   // local->lab rotation, row major
};

struct OKernel {
  int32_t type;
  int32_t dw;      // 1: multiply by the Debye-Waller factor of the scatterer
  double sigma;    // nominal cross section, barn (ignored by POWDER)
  // POWDER
  double v0;       // cell volume, A^3
  int32_t nrefl;
  int32_t pad0;
  const double* d;   // d-spacings, A
  const double* F2;  // multiplicity * |F|^2 per cell, barn
  // PHONON and MULTIPHONON
  double M;        // amu
  double T;        // K
  int32_t nbins;
  int32_t nmax;    // MULTIPHONON: highest phonon order N (orders 2..N)
  double emax;     // meV, DOS defined on [0, emax]
  const double* dos;  // raw (unnormalised) DOS values, one per bin
  // SPINWAVE
  double J, S, a, gamma;  // meV, -, A, meV (HWHM)
  double crot[9];         // lab->crystal rotation
  // SQE
  int32_t nQ, nE;
  double Qmax, Emin, Emax;
  const double* sqe;      // nQ x nE, row major (Q slow)
  // COH_PHONON (also M, T)
  int32_t grid_n;         // modes on grid_n^3 points of the reciprocal cell
  int32_t pad1;
  double cell[9];         // direct lattice vectors a_1, a_2, a_3 (rows), A
  const double* modes;    // per point: E_0..E_2 (meV), then e_0, e_1, e_2
};

struct OScatterer {
  OShape shape;
  double n;          // atoms / A^3
  double sigma_abs;  // barn at 2200 m/s
  int32_t nk;
  int32_t pad;
  OKernel k[3];
};

struct OBeam {
  int32_t type;
  int32_t pad;
  double E, sigma_rel, W, H, z0;
  // SAVED: neutrons saved at the sample position by an earlier step (Sec. 3
  // workflow): rows x, y, z (m), vx, vy, vz (m/s), t (s), p, n_saved each
  const double* saved;
  uint64_t n_saved;
};

struct ODetector {
  int32_t type;
  int32_t n2t;      // sphere rings
  int32_t ntof;
  int32_t nrows, ncols, npix;
  double R;
  double tof_lo, tof_hi;
  double phi_lo, phi_hi;  // rad, tube columns
  double row_y[8];
  double length, radius, n_he;
  int32_t tubes_per_pack;  // 0: evenly spaced columns; else packs of this many tubes
  int32_t pad;
  double pack_gap;         // rad, extra azimuth between neighbouring packs
};

// Azimuth of the axis of tube column c.  Columns are grouped in packs of
// tubes_per_pack tubes (the instruments' 8-packs, Sec. 2.1 and 2.4.1) with a gap
// between packs; the tube pitch d fills [phi_lo, phi_hi] with the packs and
// their gaps: phi_c = phi_lo + floor(c / P) gap + (c + 1/2) d.
double column_phi(const ODetector& D, int c) {
  const int P = D.tubes_per_pack;
  if (P <= 0) return D.phi_lo + (c + 0.5) * (D.phi_hi - D.phi_lo) / D.ncols;
  const int npack = D.ncols / P;
  const double d = (D.phi_hi - D.phi_lo - (npack - 1) * D.pack_gap) / D.ncols;
  return D.phi_lo + (c / P) * D.pack_gap + (c + 0.5) * d;
}

struct OSetup {
  OBeam beam;
  int32_t nscat;
  int32_t K;         // maximum scattering order
  OScatterer s[4];
  ODetector det;
  double min_prob;
};

struct ORecord {
  uint64_t id;
  uint32_t lineage;
  int32_t order;
  double pos[3], vel[3], t, w;  // state when leaving the sample assembly
  int64_t bin;                  // -1: not recorded
  double value;                 // contribution to the histogram
  double tof;
  int32_t tube;                 // -1 for the sphere or a miss
  int32_t pixel;
  double margin_anc;            // smallest normalised margin of the ancestors
  double margin_own;            // smallest normalised margin of this packet
  double value_sens;            // allowance on value: its change when the ray is shifted
                                // sideways by its binary32 uncertainty (tubes)
  uint32_t kinds;               // bit t set: a kernel of type t scattered an ancestor
  int32_t pad;
  double cond;                  // amplification of relative state errors (E_i/E_f chain)
  double wsens;                 // relative weight error from position rounding (see kEpsPos)
  double tof_tol;               // allowance on tof from the same sideways shift
  double ddir;                  // binary32 uncertainty of the direction (rad)
  double dpos;                  // binary32 uncertainty of the position (m)
  double dtime;                 // binary32 uncertainty of the time (s)
};

// Parameters of a gradient: the raw DOS values of the one-phonon kernel
// dos_k of scatterer dos_s (one parameter per bin; -1: none), the cells of
// the S(Q,E) grid of kernel sqe_k of scatterer sqe_s (-1: none), sigma_abs
// of scatterer abs_s, and the nominal sigma of kernel sig_k of scatterer
// sig_s.  mp_k: a multi-phonon kernel of scatterer dos_s whose DOS is the
// same parameter vector (its A_1 and S_n follow the DOS; -1: none).
// Gradient layout: [DOS bins..., S(Q,E) cells..., sigma_abs, sigma].
struct OParamMap {
  int32_t dos_s, dos_k, abs_s, sig_s, sig_k;
  int32_t sqe_s, sqe_k, mp_k;
};

struct OTally {
  double w_escaped[8];      // sum of escaping weight per order
  double w_detected[8];     // sum of recorded value per order
  uint64_t n_packets[8];    // packets per order
  uint64_t n_detected, n_missed, n_out_of_window, n_zero_weight;
  uint64_t n_rng_blocks, n_transcend, n_sqrt, n_shape_tests, n_tube_tests,
      n_table_steps, n_hist_updates;
  uint64_t n_segments;      // material intervals crossed
  uint64_t n_splits;        // scattered children drawn
  uint64_t n_kernel[9];     // kernel draws by type
  uint64_t n_detect;        // detector calls (escaping packets)
  double w_start[8];        // sum of weight at the start of each flight, per order
  double w_scat[8];         // weight split off to scattering (before the kernel factor)
  double w_abs[8];          // weight removed by absorption in split segments
  double w_lost[8];         // weight removed in segments that were not split
};

}  // extern "C"

namespace {

// ---------------------------------------------------------------- Philox
// Philox4x32-10 as defined by Salmon et al. (SC'11): ten rounds of
// (hi,lo) = M * x on words 0 and 2, permuted with xor of the key; the key is
// advanced by the Weyl constants between rounds.
struct Block {
  uint32_t w[4];
};

Block philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                    uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = (uint64_t)M0 * c0;
    uint64_t p1 = (uint64_t)M1 * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  Block b = {{c0, c1, c2, c3}};
  return b;
}

// 23 random bits -> an odd multiple of 2^-24 in (0,1); exact in binary32 too.
inline double to_uniform(uint32_t x) {
  return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
}

struct Rng {
  uint64_t seed;
  OTally* tally;
  // Four uniforms of block `block` in stream `stream` for packet (id, lineage).
  void draw(uint64_t id, int stream, uint32_t lineage, uint32_t block, double u[4]) {
    Block b = philox4x32_10((uint32_t)id, (uint32_t)(id >> 32) | ((uint32_t)stream << 30),
                            lineage, block, (uint32_t)seed, (uint32_t)(seed >> 32));
    for (int i = 0; i < 4; ++i) u[i] = to_uniform(b.w[i]);
    tally->n_rng_blocks++;
  }
};

// ------------------------------------------------------------- 3-vectors
struct V3 {
  double x, y, z;
};
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 scale(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline double norm(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// y = M x with M row major
inline V3 matvec(const double* m, V3 v) {
  return {m[0] * v.x + m[1] * v.y + m[2] * v.z, m[3] * v.x + m[4] * v.y + m[5] * v.z,
          m[6] * v.x + m[7] * v.y + m[8] * v.z};
}
// y = M^T x
inline V3 matTvec(const double* m, V3 v) {
  return {m[0] * v.x + m[3] * v.y + m[6] * v.z, m[1] * v.x + m[4] * v.y + m[7] * v.z,
          m[2] * v.x + m[5] * v.y + m[8] * v.z};
}

// ------------------------------------------------------------- packets
struct Packet {
  V3 pos;
  V3 dir;        // unit vector
  double speed;  // m/s
  double t;      // s
  double w;      // probability weight
  uint32_t lineage;
  int order;
  double margin_anc;  // min normalised margin of the decisions that made it
  uint32_t kinds;     // kernel types met in its ancestry (bit = type)
  double cond;        // see ORecord
  double wsens;       // see ORecord
  double ddir;        // see ORecord
  double dpos;        // see ORecord
  double dtime;       // see ORecord
  double dsp = 2e-7;  // relative uncertainty of the speed in binary32 (conditioning)
  std::vector<double> dlogw;  // d log(w) / d(parameters), when gradients are on
};

struct Interval {
  double s_in, s_out;
  int scat;  // scatterer index
  int sub;   // interval index within the scatterer
};

// ------------------------------------------------------------- geometry
// Ray p + s d (d unit).  Each routine returns the parameter interval(s) where
// the ray is inside the shape, with no clipping to s >= 0.  `margin` is
// lowered to the distance from a grazing or tangent decision.

// Slab |p_a + s d_a| <= h along one axis.  Returns false if the ray misses.
bool slab(double p, double d, double h, double* lo, double* hi, double* margin) {
  if (d == 0.0) {
    *margin = std::min(*margin, std::fabs(std::fabs(p) - h) / kTauGeom);
    if (p < -h || p > h) return false;
    *lo = -kHuge;
    *hi = kHuge;
    return true;
  }
  double s1 = (-h - p) / d, s2 = (h - p) / d;
  *lo = std::min(s1, s2);
  *hi = std::max(s1, s2);
  return true;
}

// Infinite circular cylinder of radius r about the local y axis.
bool radial(V3 p, V3 d, double r, double* lo, double* hi, double* margin) {
  double a = d.x * d.x + d.z * d.z;
  double c = p.x * p.x + p.z * p.z - r * r;
  if (a == 0.0) {
    double rho = std::sqrt(p.x * p.x + p.z * p.z);
    *margin = std::min(*margin, std::fabs(rho - r) / kTauGeom);
    if (c > 0.0) return false;
    *lo = -kHuge;
    *hi = kHuge;
    return true;
  }
  // distance of closest approach to the axis in the x-z plane
  double s_c = -(p.x * d.x + p.z * d.z) / a;
  double qx = p.x + s_c * d.x, qz = p.z + s_c * d.z;
  double b2 = qx * qx + qz * qz;
  *margin = std::min(*margin, std::fabs(std::sqrt(b2) - r) / kTauGeom);
  if (b2 >= r * r) return false;
  double half = std::sqrt((r * r - b2) / a);
  *lo = s_c - half;
  *hi = s_c + half;
  return true;
}

bool cylinder_interval(V3 p, V3 d, double r, double h, double* lo, double* hi,
                       double* margin) {
  double a0, a1, b0, b1;
  if (!radial(p, d, r, &a0, &a1, margin)) return false;
  if (!slab(p.y, d.y, 0.5 * h, &b0, &b1, margin)) return false;
  *lo = std::max(a0, b0);
  *hi = std::min(a1, b1);
  if (a0 > -kHuge && b0 > -kHuge)
    *margin = std::min(*margin, std::fabs(a0 - b0) / kTauGeom);
  if (*lo < kHuge && *hi > -kHuge)
    *margin = std::min(*margin, std::fabs(*hi - *lo) / kTauGeom);
  return *hi > *lo;
}

int shape_intervals(const OShape& sh, V3 pl, V3 dl, double lo[2], double hi[2],
                    double* margin) {
  // pl, dl already in the shape frame
  if (sh.type == SHAPE_BOX) {
    double l[3], h[3];
    if (!slab(pl.x, dl.x, 0.5 * sh.dims[0], &l[0], &h[0], margin)) return 0;
    if (!slab(pl.y, dl.y, 0.5 * sh.dims[1], &l[1], &h[1], margin)) return 0;
    if (!slab(pl.z, dl.z, 0.5 * sh.dims[2], &l[2], &h[2], margin)) return 0;
    double L = std::max(l[0], std::max(l[1], l[2]));
    double H = std::min(h[0], std::min(h[1], h[2]));
    if (L < kHuge && H > -kHuge) *margin = std::min(*margin, std::fabs(H - L) / kTauGeom);
    if (H <= L) return 0;
    lo[0] = L;
    hi[0] = H;
    return 1;
  }
  if (sh.type == SHAPE_CYLINDER) {
    if (!cylinder_interval(pl, dl, sh.dims[0], sh.dims[1], &lo[0], &hi[0], margin)) return 0;
    return 1;
  }
  // ANNULUS: outer cylinder minus the inner cylinder of the same height
  double a0, a1, b0, b1;
  if (!cylinder_interval(pl, dl, sh.dims[1], sh.dims[2], &a0, &a1, margin)) return 0;
  double mdummy = kHuge;
  bool inner = cylinder_interval(pl, dl, sh.dims[0], sh.dims[2], &b0, &b1, &mdummy);
  *margin = std::min(*margin, mdummy);
  if (!inner || b1 <= a0 || b0 >= a1) {
    lo[0] = a0;
    hi[0] = a1;
    return 1;
  }
  int n = 0;
  if (b0 > a0) {
    lo[n] = a0;
    hi[n] = b0;
    ++n;
  }
  if (a1 > b1) {
    lo[n] = b1;
    hi[n] = a1;
    ++n;
  }
  return n;
}

// |cos| of the angle between the ray and the normal of the shape surface
// nearest to the local point q (used only for the conditioning estimate)
double surface_cos(const OShape& sh, V3 q, V3 d) {
  if (sh.type == SHAPE_BOX) {
    double best = kHuge, c = 1.0;
    double qa[3] = {q.x, q.y, q.z}, da[3] = {d.x, d.y, d.z};
    for (int a = 0; a < 3; ++a) {
      double dist = std::fabs(std::fabs(qa[a]) - 0.5 * sh.dims[a]);
      if (dist < best) {
        best = dist;
        c = std::fabs(da[a]);
      }
    }
    return c;
  }
  double rho = std::sqrt(q.x * q.x + q.z * q.z);
  double h = sh.type == SHAPE_CYLINDER ? sh.dims[1] : sh.dims[2];
  double r_out = sh.type == SHAPE_CYLINDER ? sh.dims[0] : sh.dims[1];
  double best = std::fabs(std::fabs(q.y) - 0.5 * h), c = std::fabs(d.y);
  double rc = rho > 0.0 ? std::fabs(q.x * d.x + q.z * d.z) / rho : 1.0;
  if (std::fabs(rho - r_out) < best) {
    best = std::fabs(rho - r_out);
    c = rc;
  }
  if (sh.type == SHAPE_ANNULUS && std::fabs(rho - sh.dims[0]) < best) c = rc;
  return c;
}

// ------------------------------------------------------------- materials
struct KernelInfo {
  // host-side derived data for one kernel (FP64)
  std::vector<double> d_sorted, f2_sorted;  // powder, by descending d
  std::vector<double> cdf;                  // phonon: cumulative DOS (normalised);
                                            // multi-phonon: cumulative A_1 masses
  double de = 0.0;                          // phonon bin width
  std::vector<double> a1;                   // multi-phonon: A_1 masses (see a1_masses)
  double a1_sum = 0.0;                      // their sum before normalisation (1 exactly)
  double dw_self = 0.0;                     // multi-phonon: 2W / Q^2 of its own DOS
  double mode_emax = 0.0;                   // coherent one-phonon: largest mode energy
};

struct ScatInfo {
  KernelInfo k[3];
  double dw_coef = 0.0;  // 2W / Q^2 in A^2, from the scatterer's phonon DOS
};

// gamma_0 = integral of coth(E/2kT) Z(E)/E dE over [0, Emax], midpoint rule on
// the DOS bins; Z normalised to unit area (Supplement S4, multi-phonon).
double gamma0(const OKernel& k) {
  double de = k.emax / k.nbins;
  double area = 0.0;
  for (int b = 0; b < k.nbins; ++b) area += k.dos[b] * de;
  double g = 0.0;
  for (int b = 0; b < k.nbins; ++b) {
    double e = (b + 0.5) * de;
    double z = k.dos[b] / area;
    g += (1.0 / std::tanh(e / (2.0 * kBoltzmann * k.T))) * z / e * de;
  }
  return g;
}

double hbar2_over_2M(double M_amu) { return kHbar2over2mn * kNeutronMassAmu / M_amu; }

// Multi-phonon scattering in the incoherent approximation (Supplement S4):
// S(Q,E) = sum_{n=2..N} S_n(Q) A_n(E), S_n = (2W)^n/n! e^{-2W}, A_n = A_1 * A_{n-1}
// (convolution), A_1 from the DOS.  With e the energy the neutron loses,
// A_1(e) = Z(|e|)/(|e| gamma_0) (n(|e|) + 1) for e > 0 (one phonon created)
// and Z(|e|)/(|e| gamma_0) n(|e|) for e < 0 (one absorbed), n the Bose
// occupation: the paper's expression with its E = -e, which obeys detailed
// balance A_1(-e) = exp(-e/kT) A_1(e).  On the DOS bins (midpoint rule, as
// gamma_0) A_1 is a histogram with 2 nbins bins over [-emax, emax]: index j
// < nbins covers e in [-(nbins - j) de, -(nbins - j - 1) de], index nbins + b
// covers [b de, (b+1) de].  mass_j = Z_b de / (e_b gamma_0) x (n_b or n_b+1),
// which sums to 1 (2n + 1 = coth(e/2kT)).
void a1_masses(const OKernel& k, std::vector<double>& m, double* sum) {
  const int nb = k.nbins;
  const double de = k.emax / nb;
  double area = 0.0;
  for (int b = 0; b < nb; ++b) area += k.dos[b] * de;
  const double g0 = gamma0(k);
  const double kT = kBoltzmann * k.T;
  m.assign(2 * nb, 0.0);
  for (int b = 0; b < nb; ++b) {
    const double e = (b + 0.5) * de;
    const double z = k.dos[b] / area;
    const double nbose = 1.0 / std::expm1(e / kT);
    const double base = z * de / (e * g0);
    m[nb + b] = base * (nbose + 1.0);  // neutron loses e
    m[nb - 1 - b] = base * nbose;      // neutron gains e
  }
  double t = 0.0;
  for (double x : m) t += x;
  *sum = t;
}

void prepare(const OSetup& S, std::vector<ScatInfo>& info) {
  info.assign(S.nscat, ScatInfo());
  for (int s = 0; s < S.nscat; ++s) {
    const OScatterer& sc = S.s[s];
    for (int j = 0; j < sc.nk; ++j) {
      const OKernel& k = sc.k[j];
      KernelInfo& ki = info[s].k[j];
      if (k.type == K_POWDER) {
        std::vector<int> idx(k.nrefl);
        for (int i = 0; i < k.nrefl; ++i) idx[i] = i;
        std::stable_sort(idx.begin(), idx.end(),
                         [&](int a, int b) { return k.d[a] > k.d[b]; });
        for (int i : idx) {
          ki.d_sorted.push_back(k.d[i]);
          ki.f2_sorted.push_back(k.F2[i]);
        }
      } else if (k.type == K_PHONON) {
        ki.de = k.emax / k.nbins;
        double area = 0.0;
        for (int b = 0; b < k.nbins; ++b) area += k.dos[b];
        double c = 0.0;
        for (int b = 0; b < k.nbins; ++b) {
          c += k.dos[b] / area;
          ki.cdf.push_back(c);
        }
        info[s].dw_coef = hbar2_over_2M(k.M) * gamma0(k);
      } else if (k.type == K_COH_PHONON) {
        const int64_t np = (int64_t)k.grid_n * k.grid_n * k.grid_n;
        for (int64_t i = 0; i < np; ++i)
          for (int b = 0; b < 3; ++b) ki.mode_emax = std::max(ki.mode_emax, k.modes[12 * i + b]);
      } else if (k.type == K_MULTIPHONON) {
        ki.de = k.emax / k.nbins;
        a1_masses(k, ki.a1, &ki.a1_sum);
        double c = 0.0;
        for (double m : ki.a1) {
          c += m / ki.a1_sum;
          ki.cdf.push_back(c);
        }
        ki.dw_self = hbar2_over_2M(k.M) * gamma0(k);
      }
    }
  }
}

// linear attenuation coefficients, 1/m, of kernel j and of absorption
// mu = 100 * n[1/A^3] * sigma[b]; absorption follows the 1/v law.
struct Mu {
  double k[3];
  double scat, abs, total;
};

Mu attenuation(const OScatterer& sc, const ScatInfo& si, double speed, double* margin) {
  Mu m;
  double kk = k_from_speed(speed);
  double lambda = 2.0 * kPi / kk;
  m.scat = 0.0;
  for (int j = 0; j < sc.nk; ++j) {
    const OKernel& k = sc.k[j];
    if (k.type == K_POWDER) {
      // sum of Debye-Scherrer cone cross sections per unit volume:
      // lambda^2 / (2 v0^2) * sum_{d > lambda/2} d |F|^2 (Supplement S4)
      const KernelInfo& ki = si.k[j];
      double sum = 0.0;
      for (size_t i = 0; i < ki.d_sorted.size(); ++i) {
        *margin = std::min(*margin, std::fabs(ki.d_sorted[i] - 0.5 * lambda) /
                                        (kTauRel * ki.d_sorted[i]));
        if (ki.d_sorted[i] > 0.5 * lambda) sum += ki.d_sorted[i] * ki.f2_sorted[i];
      }
      m.k[j] = 100.0 * lambda * lambda / (2.0 * k.v0 * k.v0) * sum;
    } else {
      m.k[j] = 100.0 * sc.n * k.sigma;
    }
    m.scat += m.k[j];
  }
  m.abs = 100.0 * sc.n * sc.sigma_abs * (kV2200 / speed);
  m.total = m.scat + m.abs;
  return m;
}

// ------------------------------------------------------------- kernels
struct Scatter {
  V3 dir{0.0, 0.0, 0.0};
  double speed = 0.0;
  double factor = 0.0;   // weight multiplier
  double dw_q2 = 0.0;    // Q^2 entering the Debye-Waller factor (0 if none)
  int dos_bin = -1;      // DOS bin of a one-phonon draw (-1 otherwise)
  double dq_sens = 0.0;  // |d log(factor) / dQ| (per 1/A of error in Q), for conditioning
  double wsens_add = 0.0;  // further relative weight uncertainty of binary32 (conditioning)
  double dk_rel = 0.0;     // relative uncertainty of the outgoing wave number (conditioning)
  double ddir_add = -1.0;  // direction uncertainty of a cone kernel (< 0: fresh direction)
  int cell = -1;           // S(Q,E) grid cell of a tabulated draw (-1 otherwise)
  int n_a1 = 0;            // multi-phonon: phonons drawn, their A_1 bins, and Q^2
  int a1_bin[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double q2 = 0.0;
};

V3 isotropic_direction(double u_cos, double u_phi) {
  double c = 2.0 * u_cos - 1.0;
  double s = std::sqrt(std::max(0.0, 1.0 - c * c));
  double phi = 2.0 * kPi * u_phi;
  return {s * std::cos(phi), s * std::sin(phi), c};
}

// Orthonormal basis perpendicular to a unit vector n (Duff et al., "Building
// an Orthonormal Basis, Revisited", JCGT 6(1), 2017).
void perp_basis(V3 n, V3* e1, V3* e2, double* margin) {
  *margin = std::min(*margin, std::fabs(n.z) / 1e-6);
  double sgn = n.z >= 0.0 ? 1.0 : -1.0;
  double a = -1.0 / (sgn + n.z);
  double b = n.x * n.y * a;
  *e1 = {1.0 + sgn * n.x * n.x * a, sgn * b, -sgn * n.x};
  *e2 = {b, sgn + n.y * n.y * a, -n.y};
}

// incoherent elastic: dsigma/dOmega = sigma_inc/4pi N e^{-2W} (Supplement S4)
Scatter k_iso(const OKernel& k, const ScatInfo& si, const Packet& P, const double* u) {
  Scatter r;
  r.dq_sens = 0.0;
  r.dir = isotropic_direction(u[2], u[3]);
  r.speed = P.speed;
  r.factor = 1.0;
  r.dw_q2 = 0.0;
  r.dos_bin = -1;
  if (k.dw) {
    double kk = k_from_speed(P.speed);
    V3 Q = sub(scale(P.dir, kk), scale(r.dir, kk));
    r.dw_q2 = dot(Q, Q);
    r.factor = std::exp(-si.dw_coef * r.dw_q2);
    // the Debye-Waller factor depends on |Q|: d log f / dQ = -2 (2W/Q^2) Q
    r.dq_sens = 2.0 * si.dw_coef * std::sqrt(r.dw_q2);
  }
  return r;
}

// powder Bragg: one Debye-Scherrer cone chosen with probability proportional
// to its cross section; 2theta = 2 asin(lambda / 2d); uniform azimuth
Scatter k_powder(const OKernel& k, const KernelInfo& ki, const ScatInfo& si,
                 const Packet& P, const double* u, double* margin) {
  Scatter r;
  double kk = k_from_speed(P.speed);
  double lambda = 2.0 * kPi / kk;
  double total = 0.0;
  size_t nact = 0;
  for (size_t i = 0; i < ki.d_sorted.size(); ++i)
    if (ki.d_sorted[i] > 0.5 * lambda) {
      total += ki.d_sorted[i] * ki.f2_sorted[i];
      nact = i + 1;
    }
  double target = u[2] * total;
  double cum = 0.0;
  size_t pick = nact - 1;
  for (size_t i = 0; i < nact; ++i) {
    cum += ki.d_sorted[i] * ki.f2_sorted[i];
    *margin = std::min(*margin, std::fabs(target - cum) / (kTauRel * total));
    if (target < cum) {
      pick = i;
      break;
    }
  }
  double d = ki.d_sorted[pick];
  double sin_b = lambda / (2.0 * d);
  double two_theta = 2.0 * std::asin(sin_b);
  double phi = 2.0 * kPi * u[3];
  V3 e1, e2;
  perp_basis(P.dir, &e1, &e2, margin);
  V3 lateral = add(scale(e1, std::cos(phi)), scale(e2, std::sin(phi)));
  r.dir = add(scale(P.dir, std::cos(two_theta)), scale(lateral, std::sin(two_theta)));
  r.speed = P.speed;
  r.factor = 1.0;
  r.dw_q2 = 0.0;
  r.dos_bin = -1;
  if (k.dw) {
    double Q = 2.0 * kPi / d;
    r.dw_q2 = Q * Q;
    r.factor = std::exp(-si.dw_coef * r.dw_q2);
  }
  return r;
}

// incoherent one-phonon (Supplement S4):
//   d2sigma/dOmega dEf = sigma/4pi (kf/ki) N (hbar^2 Q^2/2M) e^{-2W} Z(E)/E
//                        * {coth(E/2kT) +- 1}/2
// Proposal: E from Z, creation (+) with probability (coth+1)/(2 coth),
// isotropic direction.  The ratio of the cross section per unit of sigma to
// this proposal density is (kf/ki)(hbar^2 Q^2/2M) e^{-2W} coth(E/2kT)/E.
Scatter k_phonon(const OKernel& k, const KernelInfo& ki, const ScatInfo& si,
                 const Packet& P, const double* u, double* margin) {
  Scatter r;
  r.dq_sens = 0.0;
  r.dw_q2 = 0.0;
  int b = 0;
  for (; b < k.nbins; ++b)
    if (u[2] < ki.cdf[b]) break;
  if (b == k.nbins) b = k.nbins - 1;
  r.dos_bin = b;
  *margin = std::min(*margin, std::fabs(u[2] - ki.cdf[b]) / kTauU);
  if (b > 0) *margin = std::min(*margin, std::fabs(u[2] - ki.cdf[b - 1]) / kTauU);
  double e = (b + u[3]) * ki.de;
  double kT = kBoltzmann * k.T;
  double nb = 1.0 / std::expm1(e / kT);  // Bose occupation
  double p_create = (nb + 1.0) / (2.0 * nb + 1.0);
  *margin = std::min(*margin, std::fabs(u[4] - p_create) / kTauU);
  bool create = u[4] < p_create;
  double Ei = kEperV2 * P.speed * P.speed;
  double Ef = create ? Ei - e : Ei + e;
  *margin = std::min(*margin, std::fabs(Ef) / (kTauRel * Ei));
  r.dir = isotropic_direction(u[5], u[6]);
  if (Ef <= 0.0) {
    r.speed = P.speed;
    r.factor = 0.0;
    return r;
  }
  double k_i = k_from_speed(P.speed);
  double k_f = std::sqrt(Ef / kHbar2over2mn);
  r.speed = speed_from_k(k_f);
  V3 Q = sub(scale(P.dir, k_i), scale(r.dir, k_f));
  double Q2 = dot(Q, Q);
  double h2m = hbar2_over_2M(k.M);
  double dw = k.dw ? std::exp(-si.dw_coef * Q2) : 1.0;
  r.dw_q2 = k.dw ? Q2 : 0.0;
  double coth = 1.0 / std::tanh(e / (2.0 * kT));
  r.factor = (k_f / k_i) * h2m * Q2 * dw * coth / e;
  // the weight depends on |Q| through Q^2 and the Debye-Waller factor:
  // d log f / dQ = 2/Q - 2 (2W/Q^2) Q
  const double q = std::sqrt(Q2);
  r.dq_sens = q > 0.0 ? std::fabs(2.0 / q - (k.dw ? 2.0 * si.dw_coef * q : 0.0)) : 0.0;
  return r;
}

// dispersion surface S(Q) delta(E - E(Q)) with the delta broadened to a
// Lorentzian of HWHM gamma; E(Q) = 4JS(3 - sum_a cos(Q_a a)); S(Q) = 1.
// Proposal: isotropic direction, energy transfer uniform on [E_lo, E_hi].
Scatter k_spinwave(const OKernel& k, const Packet& P, const double* u) {
  Scatter r;
  r.dq_sens = 0.0;
  r.dw_q2 = 0.0;
  r.dos_bin = -1;
  double Ei = kEperV2 * P.speed * P.speed;
  double wmax = 24.0 * k.J * k.S;
  double lo = -10.0 * k.gamma;
  double hi = std::min(wmax + 10.0 * k.gamma, 0.99 * Ei);
  r.dir = isotropic_direction(u[3], u[4]);
  r.speed = P.speed;
  if (hi <= lo) {
    r.factor = 0.0;
    return r;
  }
  double E = lo + u[2] * (hi - lo);
  double Ef = Ei - E;
  double k_i = k_from_speed(P.speed);
  double k_f = std::sqrt(Ef / kHbar2over2mn);
  r.speed = speed_from_k(k_f);
  V3 Q = sub(scale(P.dir, k_i), scale(r.dir, k_f));
  V3 Qc = matvec(k.crot, Q);
  double w = 4.0 * k.J * k.S *
             (3.0 - std::cos(Qc.x * k.a) - std::cos(Qc.y * k.a) - std::cos(Qc.z * k.a));
  double x = E - w;
  double lor = (k.gamma / kPi) / (x * x + k.gamma * k.gamma);
  r.factor = (k_f / k_i) * lor * (hi - lo);
  // conditioning: |d log L / d omega| * |grad_Q omega| (crystal axes)
  double gw = 4.0 * k.J * k.S * k.a *
              (std::fabs(std::sin(Qc.x * k.a)) + std::fabs(std::sin(Qc.y * k.a)) +
               std::fabs(std::sin(Qc.z * k.a)));
  r.dq_sens = 2.0 * std::fabs(x) / (x * x + k.gamma * k.gamma) * gw;
  return r;
}

// Dispersion surface with an exact delta function (Supplement S4, E_vQ
// kernel): S(Q,E) = S(Q) delta(E - omega(Q)) with S(Q) = 1 and omega the
// spin-wave surface above.  For an isotropic outgoing direction d (u3, u4)
// energy conservation E_i - c k^2 = omega(k_i - k d) (c = hbar^2/2m_n) fixes
// the outgoing wave number: the roots of g(k) = E_i - c k^2 - omega(k_i - k d)
// on [0, k_i] (omega >= 0).  They are bracketed by the sign changes of g
// (g > 0 against g <= 0) at kDispGrid + 1 equally spaced k and refined by
// bisection; root floor(u2 n) of the n found is taken, and the weight
// n (k_f/k_i) / |dG/dE_f| with dG/dE_f = -1 + (grad omega . d) / (2 c k_f)
// carries the integral of the delta function over E_f.  No root: weight 0.
constexpr int kDispGrid = 256;

Scatter k_dispersion(const OKernel& k, const Packet& P, const double* u, double* margin) {
  Scatter r;
  r.dw_q2 = 0.0;
  r.dos_bin = -1;
  r.dir = isotropic_direction(u[3], u[4]);
  r.speed = P.speed;
  r.factor = 0.0;
  const double Ei = kEperV2 * P.speed * P.speed;
  const double k_i = k_from_speed(P.speed);
  const double c = kHbar2over2mn;
  const double wmax = 24.0 * k.J * k.S;
  const V3 q0 = matvec(k.crot, scale(P.dir, k_i));   // crystal frame
  const V3 dc = matvec(k.crot, r.dir);
  auto omega = [&](double kk) {
    const V3 Q = sub(q0, scale(dc, kk));
    return 4.0 * k.J * k.S *
           (3.0 - std::cos(Q.x * k.a) - std::cos(Q.y * k.a) - std::cos(Q.z * k.a));
  };
  auto g = [&](double kk) { return Ei - c * kk * kk - omega(kk); };
  std::vector<int> cells;
  double gprev = g(0.0);
  *margin = std::min(*margin, std::fabs(gprev) / (kTauRel * (Ei + wmax)));
  for (int j = 1; j <= kDispGrid; ++j) {
    const double gj = g(k_i * j / kDispGrid);
    *margin = std::min(*margin, std::fabs(gj) / (kTauRel * (Ei + wmax)));
    if ((gprev > 0.0) != (gj > 0.0)) cells.push_back(j - 1);
    gprev = gj;
  }
  const int n = (int)cells.size();
  if (n == 0) return r;
  const double fu = u[2] * n;
  if (n > 1) *margin = std::min(*margin, std::fabs(fu - std::nearbyint(fu)) / (kTauU * n));
  const int pick = std::min((int)std::floor(fu), n - 1);
  double lo = k_i * cells[pick] / kDispGrid, hi = k_i * (cells[pick] + 1) / kDispGrid;
  const bool slo = g(lo) > 0.0;
  for (int it = 0; it < 200 && hi - lo > 1e-15 * k_i; ++it) {
    const double mid = 0.5 * (lo + hi);
    if ((g(mid) > 0.0) == slo) lo = mid;
    else hi = mid;
  }
  const double k_f = 0.5 * (lo + hi);
  const V3 Q = sub(q0, scale(dc, k_f));
  const double s4 = 4.0 * k.J * k.S * k.a;
  const V3 grad = {s4 * std::sin(Q.x * k.a), s4 * std::sin(Q.y * k.a), s4 * std::sin(Q.z * k.a)};
  const double A = dot(grad, dc) / (2.0 * c * k_f);
  const double J = -1.0 + A;
  *margin = std::min(*margin, std::fabs(J) / kTauJ);
  if (!(k_f > 0.0) || J == 0.0) return r;
  r.speed = speed_from_k(k_f);
  r.factor = n * (k_f / k_i) / std::fabs(J);
  // conditioning: a binary32 evaluation of g is uncertain by ~4e-7 (E_i +
  // wmax), which moves the root by that over |dg/dk| = 2 c k_f |J|, and the
  // phases Q_a a (up to ~40 rad) by ~2.4e-6 rad
  // and the incident direction's own uncertainty moves Q by k_i ddir,
  // omega by |grad omega| times that, and the root accordingly; a root
  // known to worse than kTauDk is a near decision for what follows (the
  // outgoing speed sets cone angles and cross sections downstream)
  const double dq = k_i * (P.ddir + 2e-7 + P.dsp) + k_f * 2e-7 + (k_i + k_f) * 2e-7 * P.cond;
  const double eg = 4e-7 * (Ei + wmax) + norm(grad) * dq;
  r.dk_rel = eg / (2.0 * c * k_f * k_f * std::fabs(J));
  *margin = std::min(*margin, kTauDk / r.dk_rel);
  r.wsens_add = std::fabs(A) * (2.4e-6 + r.dk_rel) / std::fabs(J) + r.dk_rel;
  r.dq_sens = 0.0;
  return r;
}

// coherent inelastic one-phonon scattering from a powder (Supplement S4).
// Averaging the lattice delta function over crystallite orientations turns
// each point K of reciprocal space (crystal frame) and branch s into a cone
// of final states with |Q| = |K| and E_f = E_i -+ E_s(K), whose cross section
// per unit sigma_coh, per unit volume of K space, is
//   (1/4pi)(k_f/k_i) e^{-2W} hbar^2 (K.e_s)^2/(2M E_s) {coth -+ 1}/2 / (2 k_i k_f K)
// (the paper's sigma_Q; the (2pi)^3/v0 of the lattice sum cancels against
// the density of K points).  Proposal: K uniform in the ball of radius
// Q_max = k_i + k_f,max (k_f,max for E_i plus the largest mode energy: no
// larger |Q| is reachable), branch uniform, phonon creation with probability
// (n+1)/(2n+1), azimuth of the cone uniform.  The weight, cross section over
// proposal density, is Q_max^3 coth(E_s/2kT) e^{-2W} hbar^2 (K.e_s)^2 /
// (2M E_s) / (2 k_i^2 K).  Modes come from the grid point nearest to K in
// fractional coordinates K.a_j/2pi (periodic); modes below 1e-3 meV (the
// acoustic branches at the zone centre) scatter with weight 0.
// grid point nearest to K: fractional coordinates g_j = n K.a_j / 2pi rounded
// (floor(g + 1/2)) and taken modulo n; returns ((i0 n + i1) n + i2)
int64_t cohphonon_index(const OKernel& k, const V3& K, double* margin) {
  const int n = k.grid_n;
  const double Km = std::sqrt(dot(K, K));
  int64_t idx[3];
  for (int j = 0; j < 3; ++j) {
    const V3 a = {k.cell[3 * j], k.cell[3 * j + 1], k.cell[3 * j + 2]};
    const double g = dot(K, a) / (2.0 * kPi) * n;
    const double fl = std::floor(g + 0.5);
    // distance to the cell boundary against a binary32 evaluation of g
    const double tau = kTauRel * (Km * std::sqrt(dot(a, a)) / (2.0 * kPi) * n + 1.0);
    *margin = std::min(*margin, (0.5 - std::fabs(g - fl)) / tau);
    idx[j] = (((int64_t)fl % n) + n) % n;
  }
  return (idx[0] * n + idx[1]) * n + idx[2];
}

Scatter k_cohphonon(const OKernel& k, const KernelInfo& ki, const ScatInfo& si,
                    const Packet& P, const double* u, double* margin) {
  Scatter r;
  r.dq_sens = 0.0;
  r.dw_q2 = 0.0;
  r.dos_bin = -1;
  r.dir = P.dir;
  r.speed = P.speed;
  r.factor = 0.0;
  const double k_i = k_from_speed(P.speed);
  const double Ei = kEperV2 * P.speed * P.speed;
  const double Qmax = k_i + std::sqrt((Ei + ki.mode_emax) / kHbar2over2mn);
  const double Km = Qmax * std::cbrt(u[2]);
  const V3 K = scale(isotropic_direction(u[3], u[4]), Km);
  const double* m = k.modes + 12 * cohphonon_index(k, K, margin);
  const int s = (int)std::floor(3.0 * u[5]);  // exact: 3u is exact in binary64
  const double Es = m[s];
  const V3 e = {m[3 + 3 * s], m[4 + 3 * s], m[5 + 3 * s]};
  if (!(Es >= 1e-3)) return r;
  const double kT = kBoltzmann * k.T;
  const double nb = 1.0 / std::expm1(Es / kT);
  const double p_create = (nb + 1.0) / (2.0 * nb + 1.0);
  *margin = std::min(*margin, std::fabs(u[6] - p_create) / kTauU);
  const bool create = u[6] < p_create;
  const double Ef = create ? Ei - Es : Ei + Es;
  *margin = std::min(*margin, std::fabs(Ef) / (kTauRel * Ei));
  if (Ef <= 0.0) return r;
  const double k_f = std::sqrt(Ef / kHbar2over2mn);
  const double scale_c = (k_i * k_i + k_f * k_f + Km * Km) / (2.0 * k_i * k_f);
  const double c = (k_i * k_i + k_f * k_f - Km * Km) / (2.0 * k_i * k_f);
  *margin = std::min(*margin, (1.0 - std::fabs(c)) / (kTauRel * scale_c));
  if (!(std::fabs(c) <= 1.0)) return r;
  const double sn = std::sqrt(std::max(0.0, 1.0 - c * c));
  const double phi = 2.0 * kPi * u[7];
  V3 e1, e2;
  perp_basis(P.dir, &e1, &e2, margin);
  const V3 lateral = add(scale(e1, std::cos(phi)), scale(e2, std::sin(phi)));
  r.dir = add(scale(P.dir, c), scale(lateral, sn));
  r.speed = speed_from_k(k_f);
  const double ke = dot(K, e);
  const double dw = k.dw ? std::exp(-si.dw_coef * Km * Km) : 1.0;
  r.dw_q2 = k.dw ? Km * Km : 0.0;
  const double coth = 1.0 / std::tanh(Es / (2.0 * kT));
  r.factor = Qmax * Qmax * Qmax * coth * dw * hbar2_over_2M(k.M) * ke * ke / Es /
             (2.0 * k_i * k_i * Km);
  // binary32 conditioning: the projection K.e loses digits when K is nearly
  // perpendicular to e; the cone angle acos(c) is steep near c = +-1
  r.wsens_add = 2.0 * 8.0 * 6e-8 * Km / std::max(std::fabs(ke), 1e-30);
  const double dc = scale_c * (8.0 * 6e-8 + 2.0 * P.dsp);
  r.ddir_add = dc / std::max(sn, std::sqrt(dc));
  return r;
}

// tabulated isotropic S(Q,E): value of the grid cell containing (|Q|, E)
Scatter k_sqe(const OKernel& k, const Packet& P, const double* u, double* margin) {
  Scatter r;
  r.dq_sens = 0.0;
  r.dw_q2 = 0.0;
  r.dos_bin = -1;
  double Ei = kEperV2 * P.speed * P.speed;
  double E = k.Emin + u[2] * (k.Emax - k.Emin);
  double Ef = Ei - E;
  r.dir = isotropic_direction(u[3], u[4]);
  r.speed = P.speed;
  *margin = std::min(*margin, std::fabs(Ef) / (kTauRel * Ei));
  if (Ef <= 0.0) {
    r.factor = 0.0;
    return r;
  }
  double k_i = k_from_speed(P.speed);
  double k_f = std::sqrt(Ef / kHbar2over2mn);
  r.speed = speed_from_k(k_f);
  double Q = norm(sub(scale(P.dir, k_i), scale(r.dir, k_f)));
  double fq = Q / k.Qmax * k.nQ;
  double fe = (E - k.Emin) / (k.Emax - k.Emin) * k.nE;
  *margin = std::min(*margin, std::fabs(fq - std::nearbyint(fq)) / (kTauRel * std::max(fq, 1.0)));
  *margin = std::min(*margin, std::fabs(fe - std::nearbyint(fe)) / (kTauRel * std::max(fe, 1.0)));
  int iq = (int)std::floor(fq);
  int ie = (int)std::floor(fe);
  if (ie < 0) ie = 0;
  if (ie > k.nE - 1) ie = k.nE - 1;
  if (iq >= k.nQ) {
    r.factor = 0.0;
    return r;
  }
  r.cell = iq * k.nE + ie;
  r.factor = (k_f / k_i) * k.sqe[r.cell] * (k.Emax - k.Emin);
  return r;
}

// Multi-phonon kernel: order n uniform on 2..N (u2), direction isotropic
// (u3, u4), energy loss e = sum of n independent draws from the A_1
// histogram (bin by inverse CDF, position uniform within the bin), so that e
// follows A_n exactly; weight (k_f/k_i) S_n(Q) (N - 1) against that proposal.
// Phonon i takes words 2(i mod 2), 2(i mod 2)+1 of extra block i/2 (blocks
// 2, 3, ... of the scattering stream).
template <class Extra>
Scatter k_multiphonon(const OKernel& k, const KernelInfo& ki, const Packet& P, const double* u,
                      Extra extra, double* margin) {
  Scatter r;
  r.dq_sens = 0.0;
  r.dw_q2 = 0.0;
  r.dos_bin = -1;
  const int N = k.nmax;
  double fn = u[2] * (N - 1);
  *margin = std::min(*margin, std::fabs(fn - std::nearbyint(fn)) / (kTauU * (N - 1)));
  int n = 2 + std::min((int)std::floor(fn), N - 2);
  r.dir = isotropic_direction(u[3], u[4]);
  const int nb = k.nbins;
  double e = 0.0;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < n; ++i) {
    if ((i & 1) == 0) extra(i / 2, v);
    const double ub = v[2 * (i & 1)], up = v[2 * (i & 1) + 1];
    int j = 0;
    for (; j < 2 * nb; ++j)
      if (ub < ki.cdf[j]) break;
    if (j == 2 * nb) j = 2 * nb - 1;
    *margin = std::min(*margin, std::fabs(ub - ki.cdf[j]) / kTauU);
    if (j > 0) *margin = std::min(*margin, std::fabs(ub - ki.cdf[j - 1]) / kTauU);
    e += (j - nb + up) * ki.de;
    r.a1_bin[i] = j;
  }
  r.n_a1 = n;
  const double Ei = kEperV2 * P.speed * P.speed;
  const double Ef = Ei - e;
  *margin = std::min(*margin, std::fabs(Ef) / (kTauRel * Ei));
  r.speed = P.speed;
  if (Ef <= 0.0) {
    r.factor = 0.0;
    return r;
  }
  const double k_i = k_from_speed(P.speed);
  const double k_f = std::sqrt(Ef / kHbar2over2mn);
  r.speed = speed_from_k(k_f);
  const V3 Q = sub(scale(P.dir, k_i), scale(r.dir, k_f));
  const double Q2 = dot(Q, Q);
  r.q2 = Q2;
  const double w2 = ki.dw_self * Q2;  // 2W
  double sn = std::exp(-w2);
  for (int m = 1; m <= n; ++m) sn *= w2 / m;
  r.factor = (k_f / k_i) * sn * (N - 1);
  const double q = std::sqrt(Q2);
  r.dq_sens = q > 0.0 ? std::fabs(2.0 * n / q - 2.0 * ki.dw_self * q) : 0.0;
  return r;
}

// ------------------------------------------------------------- simulation
// distance (in bins) of a fractional tof bin index to the boundary that
// decides it: a bin edge inside the window, the window edge outside it
double tof_margin(double ft, int ntof) {
  if (ft < 0.0) return -ft;
  if (ft >= ntof) return ft - ntof;
  return std::fabs(ft - std::nearbyint(ft));
}

struct Sim {
  // S: the parameters the weights are evaluated at; Sp: the parameters the
  // random choices are drawn from (the same setup except for a gradient or a
  // re-weighting check, where Sp is frozen at the reference point)
  const OSetup& S;
  const OSetup& Sp;
  std::vector<ScatInfo> info, pinfo;
  // gradient (forward mode): dense tangent of log(w) for every packet
  bool tangent = false;
  OParamMap pm;
  int np = 0;
  int nb = 0;  // DOS parameters (first in the gradient), then nc S(Q,E) cells
  int nc = 0;
  const double* dLdI = nullptr;
  double* grad = nullptr;
  double* gabs = nullptr;   // sum of |dL/dI value d log(w)| per parameter (or null)
  double* gflag = nullptr;  // the same over near-decision packets (or null)
  Rng rng;
  double* hist;
  double* hist_w2;
  ORecord* recs;
  uint64_t rec_cap;
  uint64_t n_rec;
  OTally* tally;

  Sim(const OSetup& s, const OSetup& sp) : S(s), Sp(sp) {}

  // d mu_total / d theta of scatterer s at speed v (only sigma_abs and the
  // nominal sigma are parameters of the attenuation)
  void add_dmu(std::vector<double>& g, int s, double speed, double scale) const {
    const OScatterer& sc = S.s[s];
    if (s == pm.abs_s) g[np - 2] += scale * 100.0 * sc.n * (kV2200 / speed);
    if (s == pm.sig_s) g[np - 1] += scale * 100.0 * sc.n;
  }

  // d log(DW factor) / d theta for a Debye-Waller factor exp(-h2m gamma0 Q^2)
  // of the scatterer that owns the parameter DOS:
  // gamma0 = sum_b c_b theta_b / S, c_b = coth(e_b/2kT) de / e_b, S = sum theta de
  void add_ddw(std::vector<double>& g, double q2) const {
    const OKernel& k = S.s[pm.dos_s].k[pm.dos_k];
    double de = k.emax / k.nbins;
    double Ssum = 0.0;
    for (int b = 0; b < k.nbins; ++b) Ssum += k.dos[b] * de;
    double g0 = gamma0(k);
    double h2m = hbar2_over_2M(k.M);
    for (int b = 0; b < k.nbins; ++b) {
      double e = (b + 0.5) * de;
      double c = de / (e * std::tanh(e / (2.0 * kBoltzmann * k.T)));
      g[b] += -h2m * q2 * (c - g0 * de) / Ssum;
    }
  }

  // d log(weight) / d theta of a multi-phonon draw (kernel k, whose DOS
  // values are the parameters): every phonon i comes from A_1 bin j_i with
  // mass m_j = Z_b de / (e_b gamma0) (n_b or n_b + 1), Z = theta / S, so that
  // d log m_j / d theta = delta_b / theta_b - de / S - d log gamma0 / d theta;
  // S_n(Q) = (2W)^n / n! e^{-2W} with 2W = (hbar^2/2M) gamma0 Q^2 adds
  // (n - 2W) d log gamma0 / d theta; gamma0 = sum_b c_b theta_b / S with
  // c_b = coth(e_b/2kT) de / e_b (Supplement S4, multi-phonon kernel).
  void add_dmultiphonon(std::vector<double>& g, const OKernel& k, const Scatter& r) const {
    const int nbk = k.nbins;
    const double de = k.emax / nbk;
    double Ssum = 0.0;
    for (int b = 0; b < nbk; ++b) Ssum += k.dos[b] * de;
    const double g0 = gamma0(k);
    std::vector<double> dlg0(nbk);
    for (int b = 0; b < nbk; ++b) {
      const double e = (b + 0.5) * de;
      const double c = de / (e * std::tanh(e / (2.0 * kBoltzmann * k.T)));
      dlg0[b] = (c - g0 * de) / (Ssum * g0);
    }
    for (int i = 0; i < r.n_a1; ++i) {
      const int j = r.a1_bin[i];
      const int b = j >= nbk ? j - nbk : nbk - 1 - j;
      g[b] += 1.0 / k.dos[b];
      for (int q = 0; q < nbk; ++q) g[q] += -de / Ssum - dlg0[q];
    }
    const double w2 = hbar2_over_2M(k.M) * g0 * r.q2;
    for (int q = 0; q < nbk; ++q) g[q] += (r.n_a1 - w2) * dlg0[q];
  }

  // d log Z(e) / d theta for a draw from DOS bin b: Z_b = theta_b / S
  void add_dlogz(std::vector<double>& g, int b) const {
    const OKernel& k = S.s[pm.dos_s].k[pm.dos_k];
    double de = k.emax / k.nbins;
    double Ssum = 0.0;
    for (int j = 0; j < k.nbins; ++j) Ssum += k.dos[j] * de;
    for (int j = 0; j < k.nbins; ++j) g[j] -= de / Ssum;
    g[b] += 1.0 / k.dos[b];
  }

  // ----- detector: sphere of radius R about the origin, rings in 2theta
  void detect_sphere(const Packet& P, ORecord& rec, double* margin) {
    const ODetector& D = S.det;
    double b = dot(P.pos, P.dir);
    double c = dot(P.pos, P.pos) - D.R * D.R;
    if (c >= 0.0) return;  // already outside the sphere
    double s = -b + std::sqrt(b * b - c);
    V3 hit = add(P.pos, scale(P.dir, s));
    double cz = std::max(-1.0, std::min(1.0, hit.z / D.R));
    double tt = std::acos(cz);
    double width = kPi / D.n2t;
    int ring = (int)std::floor(tt / width);
    if (ring > D.n2t - 1) ring = D.n2t - 1;
    if (ring < 0) ring = 0;
    // distance in cos(2theta) to the ring edges that bound this ring
    double m_lo = ring > 0 ? std::fabs(cz - std::cos(ring * width)) : kHuge;
    double m_hi = ring < D.n2t - 1 ? std::fabs(cz - std::cos((ring + 1) * width)) : kHuge;
    *margin = std::min(*margin, std::min(m_lo, m_hi) / (kTauCos + 3.0 * (P.ddir + 1e-7)));
    double tof = P.t + s / P.speed;
    rec.tof = tof;
    double dt = (D.tof_hi - D.tof_lo) / D.ntof;
    double ft = (tof - D.tof_lo) / dt;
    int it = (int)std::floor(ft);
    *margin = std::min(*margin, tof_margin(ft, D.ntof) * dt / (kTauTof * std::fabs(tof)));
    if (ft < 0.0 || it >= D.ntof) {
      tally->n_out_of_window++;
      return;
    }
    rec.bin = (int64_t)ring * D.ntof + it;
    rec.value = P.w;
  }

  // ----- detector: vertical 3He tubes on a cylinder of radius R
  // brute force over every tube; the first tube on the ray records
  void detect_tubes(const Packet& P, ORecord& rec, double* margin) {
    const ODetector& D = S.det;
    // lateral uncertainty of the ray at the detector for a binary32
    // implementation, and the geometric decision scale it implies
    const double db = (P.ddir + 1e-7) * D.R + 1e-8;
    const double tauG = kTauGeom + 3.0 * db;
    double best = kHuge, second = kHuge;
    int best_tube = -1;
    double best_out = 0.0, best_b = 0.0, best_dperp = 0.0;
    for (int row = 0; row < D.nrows; ++row) {
      for (int col = 0; col < D.ncols; ++col) {
        tally->n_tube_tests++;
        double phi = column_phi(D, col);
        V3 c = {D.R * std::sin(phi), D.row_y[row], D.R * std::cos(phi)};
        V3 p = sub(P.pos, c);
        double lo, hi, m = kHuge;
        // radial part with the impact parameter kept for the margin
        double a = P.dir.x * P.dir.x + P.dir.z * P.dir.z;
        if (a == 0.0) continue;
        double s_c = -(p.x * P.dir.x + p.z * P.dir.z) / a;
        double qx = p.x + s_c * P.dir.x, qz = p.z + s_c * P.dir.z;
        double bimp = std::sqrt(qx * qx + qz * qz);
        const double tauI = kTauImpact * D.radius + 3.0 * db;
        if (std::fabs(bimp - D.radius) < tauI) *margin = std::min(*margin, std::fabs(bimp - D.radius) / tauI);
        if (!cylinder_interval(p, P.dir, D.radius, D.length, &lo, &hi, &m)) {
          if (bimp < D.radius) *margin = std::min(*margin, m);
          continue;
        }
        if (bimp < D.radius) *margin = std::min(*margin, m);
        if (hi <= 0.0) continue;
        double s_in = std::max(lo, 0.0);
        if (s_in < best) {
          second = best;
          best = s_in;
          best_tube = row * D.ncols + col;
          best_out = hi;
          best_b = bimp;
          best_dperp = std::sqrt(a);
        } else if (s_in < second) {
          second = s_in;
        }
      }
    }
    if (best_tube < 0) {
      tally->n_missed++;
      return;
    }
    if (second < kHuge) *margin = std::min(*margin, (second - best) / tauG);
    double chord = best_out - best;
    double mu = 100.0 * D.n_he * kHe3SigmaAbs * (kV2200 / P.speed);
    double pabs = -std::expm1(-mu * chord);
    double u[4];
    rng.draw(rec.id, STREAM_DETECT, P.lineage, 0, u);
    double s_a = best - std::log1p(-u[0] * pabs) / mu;
    double y_a = P.pos.y + s_a * P.dir.y;
    int row = best_tube / D.ncols;
    double y_bot = D.row_y[row] - 0.5 * D.length;
    double fp = (y_a - y_bot) / D.length * D.npix;
    int pix = (int)std::floor(fp);
    if (pix < 0) pix = 0;
    if (pix > D.npix - 1) pix = D.npix - 1;
    double ym = std::fabs(fp - std::nearbyint(fp)) * D.length / D.npix;
    if (std::nearbyint(fp) > 0 && std::nearbyint(fp) < D.npix) *margin = std::min(*margin, ym / tauG);
    double tof = P.t + s_a / P.speed;
    rec.tof = tof;
    rec.tube = best_tube;
    rec.pixel = pix;
    double dt = (D.tof_hi - D.tof_lo) / D.ntof;
    double ft = (tof - D.tof_lo) / dt;
    int it = (int)std::floor(ft);
    *margin = std::min(*margin, tof_margin(ft, D.ntof) * dt / (kTauTof * std::fabs(tof)));
    // allowance: value and tof of the same tube for the ray shifted sideways
    // by db in two perpendicular directions (chords cut by the caps included)
    {
      (void)best_b;
      (void)best_dperp;
      int brow = best_tube / D.ncols, bcol = best_tube % D.ncols;
      double phi = column_phi(D, bcol);
      V3 c = {D.R * std::sin(phi), D.row_y[brow], D.R * std::cos(phi)};
      V3 e1, e2;
      double mdummy = kHuge;
      perp_basis(P.dir, &e1, &e2, &mdummy);
      double vmax = 0.0, tmax = 0.0;
      for (int k = 0; k < 4; ++k) {
        V3 sh = scale(k < 2 ? e1 : e2, (k & 1) ? -db : db);
        V3 p = sub(add(P.pos, sh), c);
        double lo2, hi2, m2 = kHuge;
        if (!cylinder_interval(p, P.dir, D.radius, D.length, &lo2, &hi2, &m2) || hi2 <= 0.0) {
          vmax = std::max(vmax, P.w * pabs);
          continue;
        }
        double s_in2 = std::max(lo2, 0.0);
        double pabs2 = -std::expm1(-mu * (hi2 - s_in2));
        double s_a2 = s_in2 - std::log1p(-u[0] * pabs2) / mu;
        vmax = std::max(vmax, std::fabs(P.w * pabs2 - P.w * pabs));
        tmax = std::max(tmax, std::fabs(s_a2 - s_a) / P.speed);
      }
      rec.value_sens = vmax;
      rec.tof_tol = tmax;
    }
    if (ft < 0.0 || it >= D.ntof) {
      tally->n_out_of_window++;
      return;
    }
    rec.bin = ((int64_t)best_tube * D.npix + pix) * D.ntof + it;
    rec.value = P.w * pabs;
  }

  void detect(const Packet& P, uint64_t id, double flight_margin) {
    ORecord rec;
    std::memset(&rec, 0, sizeof(rec));
    rec.id = id;
    rec.lineage = P.lineage;
    rec.order = P.order;
    rec.pos[0] = P.pos.x; rec.pos[1] = P.pos.y; rec.pos[2] = P.pos.z;
    rec.vel[0] = P.dir.x * P.speed; rec.vel[1] = P.dir.y * P.speed; rec.vel[2] = P.dir.z * P.speed;
    rec.t = P.t;
    rec.w = P.w;
    rec.bin = -1;
    rec.tube = -1;
    rec.pixel = -1;
    rec.margin_anc = P.margin_anc;
    rec.kinds = P.kinds;
    rec.cond = P.cond;
    rec.wsens = P.wsens;
    rec.ddir = P.ddir;
    rec.dpos = P.dpos;
    rec.dtime = P.dtime;
    double margin = kHuge;
    tally->n_detect++;
    if (S.det.type == DET_SPHERE) detect_sphere(P, rec, &margin);
    else detect_tubes(P, rec, &margin);
    rec.margin_own = std::min(flight_margin, margin);
    tally->w_escaped[P.order] += P.w;
    if (rec.bin >= 0 && tangent) {
      double g = dLdI[rec.bin] * rec.value;
      const bool near = std::min(rec.margin_anc, rec.margin_own) < 1.0;
      for (int j = 0; j < np; ++j) {
        grad[j] += g * P.dlogw[j];
        if (gabs) gabs[j] += std::fabs(g * P.dlogw[j]);
        if (gflag && near) gflag[j] += std::fabs(g * P.dlogw[j]);
      }
    }
    if (rec.bin >= 0 && hist) {
      hist[rec.bin] += rec.value;
      if (hist_w2) hist_w2[rec.bin] += rec.value * rec.value;
      tally->n_detected++;
      tally->n_hist_updates++;
      tally->w_detected[P.order] += rec.value;
    }
    if (recs && n_rec < rec_cap) recs[n_rec] = rec;
    n_rec++;
  }

  // ----- one flight of a packet through the assembly; returns its children
  // Sec. 2.4.3 / Supplement S3: each material interval on the ray splits the
  // packet; the transmitted part keeps flying, the scattered part starts at a
  // point of the interval drawn from the truncated exponential.
  // [bookkeeping] Binary32 conditioning of a child packet -- test
  // bookkeeping beside the method, not part of it: the uncertainties the
  // parity bars are built from (wsens: relative weight sensitivity to
  // position rounding; cond: E_i/E_f amplification; dpos, dtime, dsp, ddir:
  // position, time, speed and direction uncertainties).  P: the parent at
  // the scattering point; birth at s_in + x on a chord of length L whose
  // interaction probability is a = 1 - e^{-mu L}; dL: the chord's
  // uncertainty.
  static void child_conditioning(const Packet& P, const Scatter& r, int ktype, double s_in,
                                 double x, double mu, double L, double a, double dL, Packet& C) {
    // d log(1 - e^{-mu L}) / dL times the chord uncertainty
    C.wsens = P.wsens + mu * std::exp(-mu * L) / a * dL;
    double Ein = kEperV2 * P.speed * P.speed;
    double Eout = kEperV2 * C.speed * C.speed;
    C.cond = P.cond * (Eout > 0.0 ? std::max(1.0, Ein / Eout) : 1.0);
    // the birth point sits x into the interval, with x ~ 1/mu(speed)
    C.dpos = P.dpos + P.ddir * (s_in + x) + kEpsPos + dL + x * P.dsp;
    C.dtime = P.dtime + (dL + kEpsPos) / P.speed + (s_in + x) / P.speed * P.dsp;
    // the child's speed: unchanged by elastic kernels, amplified by
    // E_i/E_f through an energy loss, plus a delta-function root
    C.dsp = Eout == Ein ? P.dsp
                        : P.dsp * (Eout > 0.0 ? std::max(1.0, Ein / Eout) : 1.0) + 2e-7;
    C.dsp += r.dk_rel;
    if (r.dq_sens > 0.0) {
      double kin = k_from_speed(P.speed), kout = k_from_speed(C.speed);
      double dq = kin * (P.ddir + 2e-7) + kout * 2e-7 + (kin + kout) * 2e-7 * P.cond;
      C.wsens += r.dq_sens * dq;
    }
    C.wsens += r.wsens_add;
    C.cond *= 1.0 + r.dk_rel / 1e-5;
    if (ktype == K_POWDER) {
      // the cone angle 2 asin(lambda/2d) from a binary32 wavelength:
      // d(2 theta) = 2 tan(theta) d lambda / lambda
      double c = dot(P.dir, C.dir);
      double th = 0.5 * std::acos(std::max(-1.0, std::min(1.0, c)));
      double tn = std::tan(std::min(th, 0.5 * kPi - 1e-6));
      C.ddir = P.ddir + 2e-7 + 2.0 * tn * std::max(2e-7 * P.cond, P.dsp);
    } else if (r.ddir_add >= 0.0) {
      C.ddir = P.ddir + 2e-7 + r.ddir_add;  // a cone about the incident direction
    } else {
      C.ddir = 2e-7;  // a fresh isotropic direction
    }
  }

  // [bookkeeping] chord uncertainty of a binary32 implementation: lateral
  // uncertainty at the exit (and entry) surface -- position rounding plus
  // the direction's uncertainty over the distance flown -- over the cosine of
  // the surface crossing (sliding the start along the ray does not move the
  // surfaces it meets)
  static void chord_uncertainty(const OShape& sh, const Packet& P, V3 start, double s_in,
                                double s_out, double* dL, double* dL_exit) {
    V3 dl = matTvec(sh.rot, P.dir);
    V3 q_out = matTvec(sh.rot, sub(add(start, scale(P.dir, s_out)),
                                   {sh.pos[0], sh.pos[1], sh.pos[2]}));
    *dL_exit = (kEpsPos + P.ddir * s_out) / std::max(surface_cos(sh, q_out, dl), 1e-9);
    *dL = *dL_exit;
    if (s_in > 0.0) {
      V3 q_in = matTvec(sh.rot, sub(add(start, scale(P.dir, s_in)),
                                    {sh.pos[0], sh.pos[1], sh.pos[2]}));
      *dL += (kEpsPos + P.ddir * s_in) / std::max(surface_cos(sh, q_in, dl), 1e-9);
    }
  }

  void fly(Packet& P, uint64_t id, std::vector<Packet>& children, double* own_margin) {
    std::vector<Interval> segs;
    for (int s = 0; s < S.nscat; ++s) {
      const OShape& sh = S.s[s].shape;
      V3 pl = matTvec(sh.rot, sub(P.pos, {sh.pos[0], sh.pos[1], sh.pos[2]}));
      V3 dl = matTvec(sh.rot, P.dir);
      double lo[2], hi[2];
      tally->n_shape_tests++;
      int n = shape_intervals(sh, pl, dl, lo, hi, own_margin);
      for (int i = 0; i < n; ++i) {
        *own_margin = std::min(*own_margin, std::fabs(hi[i] - kSurfaceEps) / kTauGeom);  // [bookkeeping]
        if (hi[i] <= kSurfaceEps) continue;  // behind or leaving through this surface
        *own_margin = std::min(*own_margin, std::fabs(lo[i]) / kTauGeom);  // [bookkeeping]
        Interval iv = {std::max(lo[i], 0.0), hi[i], s, i};
        segs.push_back(iv);
      }
    }
    std::stable_sort(segs.begin(), segs.end(),
                     [](const Interval& a, const Interval& b) { return a.s_in < b.s_in; });
    V3 start = P.pos;
    double t0 = P.t;
    double last_dL_exit = 0.0;
    for (size_t g = 0; g < segs.size(); ++g) {
      const Interval& iv = segs[g];
      const OScatterer& sc = S.s[iv.scat];
      const ScatInfo& si = info[iv.scat];
      // random choices follow the proposal parameters (identical to S except
      // when re-weighting or differentiating with frozen proposals)
      const OScatterer& scp = Sp.s[iv.scat];
      const ScatInfo& sip = pinfo[iv.scat];
      double L = iv.s_out - iv.s_in;
      double m_mu = kHuge;
      Mu mu = attenuation(sc, si, P.speed, &m_mu);
      Mu mup = attenuation(scp, sip, P.speed, &m_mu);
      *own_margin = std::min(*own_margin, m_mu);  // [bookkeeping]
      tally->n_segments++;
      double dL, dL_exit;  // [bookkeeping]
      chord_uncertainty(sc.shape, P, start, iv.s_in, iv.s_out, &dL, &dL_exit);
      double att = std::exp(-mu.total * L);
      double a = -std::expm1(-mup.total * L);  // probability to interact
      tally->n_transcend += 2;
      if (P.order < S.K && P.w >= S.min_prob && mup.scat > 0.0) {
        uint32_t lin = P.lineage * 8u + (uint32_t)g + 1u;
        double u[8];
        rng.draw(id, STREAM_SCATTER, lin, 0, u);
        rng.draw(id, STREAM_SCATTER, lin, 1, u + 4);
        // forced collision: x ~ mu e^{-mu x} / (1 - e^{-mu L}) on [0, L]
        double x = -std::log1p(-u[0] * a) / mup.total;
        tally->n_transcend++;
        double child_margin = *own_margin;
        Packet C;
        C.pos = add(start, scale(P.dir, iv.s_in + x));
        C.t = t0 + (iv.s_in + x) / P.speed;
        C.dir = P.dir;
        C.speed = P.speed;
        C.w = P.w * (mup.scat / mup.total) * a;
        tally->w_abs[P.order] += P.w * (mup.abs / mup.total) * a;
        tally->w_scat[P.order] += C.w;
        // kernel choice with probability mu_k / mu_s
        double target = u[1] * mup.scat;
        double cum = 0.0;
        int kk = sc.nk - 1;
        for (int j = 0; j < sc.nk; ++j) {
          cum += mup.k[j];
          if (j < sc.nk - 1)  // [bookkeeping]
            child_margin = std::min(child_margin, std::fabs(target - cum) / (kTauRel * mup.scat));
          if (target < cum) {
            kk = j;
            break;
          }
        }
        // true rate over proposal density of the point and the kernel; 1 when
        // the two parameter sets coincide
        C.w *= (mu.k[kk] * std::exp(-mu.total * x)) / (mup.k[kk] * std::exp(-mup.total * x));
        const OKernel& k = sc.k[kk];
        tally->n_splits++;
        tally->n_kernel[k.type]++;
        Scatter r;
        Packet Pin = P;  // state of the incident packet at the scattering point
        const OKernel& kp = scp.k[kk];
        switch (k.type) {
          case K_ISO_EL: r = k_iso(kp, sip, Pin, u); break;
          case K_POWDER: r = k_powder(kp, sip.k[kk], sip, Pin, u, &child_margin); break;
          case K_PHONON: r = k_phonon(kp, sip.k[kk], sip, Pin, u, &child_margin); break;
          case K_SPINWAVE: r = k_spinwave(kp, Pin, u); break;
          case K_MULTIPHONON:
            r = k_multiphonon(
                kp, sip.k[kk], Pin, u,
                [&](int b, double v[4]) { rng.draw(id, STREAM_SCATTER, lin, 2u + b, v); },
                &child_margin);
            break;
          case K_DISPERSION: r = k_dispersion(kp, Pin, u, &child_margin); break;
          case K_COH_PHONON: r = k_cohphonon(kp, sip.k[kk], sip, Pin, u, &child_margin); break;
          default: r = k_sqe(kp, Pin, u, &child_margin); break;
        }
        // evaluation-point Debye-Waller factor and DOS over the proposal's
        if (r.dw_q2 > 0.0) r.factor *= std::exp(-(si.dw_coef - sip.dw_coef) * r.dw_q2);
        if (r.dos_bin >= 0) {
          double ssum = 0.0, psum = 0.0;
          for (int b = 0; b < k.nbins; ++b) {
            ssum += k.dos[b];
            psum += kp.dos[b];
          }
          r.factor *= (k.dos[r.dos_bin] / ssum) / (kp.dos[r.dos_bin] / psum);
        }
        // tabulated S(Q,E): the evaluation grid's cell over the proposal's
        if (r.cell >= 0 && kp.sqe[r.cell] != 0.0) r.factor *= k.sqe[r.cell] / kp.sqe[r.cell];
        // multi-phonon: the A_1 masses of the drawn phonons and S_n at the
        // evaluation DOS over those of the proposal DOS
        if (k.type == K_MULTIPHONON && r.factor > 0.0) {
          const KernelInfo& ke = si.k[kk];
          const KernelInfo& kq = sip.k[kk];
          for (int i = 0; i < r.n_a1; ++i) {
            const int j = r.a1_bin[i];
            r.factor *= (ke.a1[j] / ke.a1_sum) / (kq.a1[j] / kq.a1_sum);
          }
          r.factor *= std::pow(ke.dw_self / kq.dw_self, r.n_a1) *
                      std::exp(-(ke.dw_self - kq.dw_self) * r.q2);
        }
        tally->n_transcend += 4;
        C.dir = r.dir;
        C.speed = r.speed;
        C.w *= r.factor;
        if (tangent) {
          C.dlogw = P.dlogw;
          if (iv.scat == pm.sig_s && kk == pm.sig_k) C.dlogw[np - 1] += 1.0 / k.sigma;
          add_dmu(C.dlogw, iv.scat, P.speed, -x);
          if (r.dw_q2 > 0.0 && iv.scat == pm.dos_s) add_ddw(C.dlogw, r.dw_q2);
          if (r.dos_bin >= 0 && iv.scat == pm.dos_s && kk == pm.dos_k) add_dlogz(C.dlogw, r.dos_bin);
          if (r.cell >= 0 && iv.scat == pm.sqe_s && kk == pm.sqe_k)
            C.dlogw[nb + r.cell] += 1.0 / k.sqe[r.cell];
          if (k.type == K_MULTIPHONON && iv.scat == pm.dos_s && kk == pm.mp_k)
            add_dmultiphonon(C.dlogw, k, r);
        }
        C.lineage = lin;
        C.order = P.order + 1;
        C.kinds = P.kinds | (1u << k.type);
        C.margin_anc = std::min(P.margin_anc, child_margin);  // [bookkeeping]
        child_conditioning(P, r, k.type, iv.s_in, x, mup.total, L, a, dL, C);  // [bookkeeping]
        if (C.w > 0.0) children.push_back(C);
        else tally->n_zero_weight++;
      } else {
        tally->w_lost[P.order] += P.w * a;
      }
      P.w *= att;
      P.wsens += mu.total * dL;  // [bookkeeping]
      last_dL_exit = dL_exit;    // [bookkeeping]
      if (tangent) add_dmu(P.dlogw, iv.scat, P.speed, -L);
    }
    if (!segs.empty()) {
      double s_end = segs.back().s_out;
      P.pos = add(start, scale(P.dir, s_end));
      P.t = t0 + s_end / P.speed;
      P.dpos += P.ddir * s_end + last_dL_exit;                        // [bookkeeping]
      P.dtime += last_dL_exit / P.speed + s_end / P.speed * P.dsp;   // [bookkeeping]
    }
  }

  void process(Packet& P, uint64_t id) {
    tally->n_packets[P.order]++;
    tally->w_start[P.order] += P.w;
    std::vector<Packet> children;
    double own = kHuge;
    fly(P, id, children, &own);
    detect(P, id, own);
    // depth first; the order is immaterial because every random number is
    // addressed by (id, stream, lineage, block)
    for (Packet& C : children) process(C, id);
  }

  void source(uint64_t id, Packet& P) {
    const OBeam& B = S.beam;
    P.lineage = 1u;
    P.order = 0;
    P.margin_anc = kHuge;
    P.kinds = 0u;
    P.cond = 1.0;
    P.wsens = 0.0;
    P.ddir = 0.0;
    P.dpos = 0.0;
    P.dtime = 0.0;
    P.dsp = 2e-7;
    if (tangent) P.dlogw.assign(np, 0.0);
    if (B.type == BEAM_SAVED) {
      // entry `id` of the saved neutrons: position, velocity, time, weight
      const uint64_t n = B.n_saved;
      const double* r = B.saved;
      P.pos = {r[id], r[n + id], r[2 * n + id]};
      const V3 v = {r[3 * n + id], r[4 * n + id], r[5 * n + id]};
      const double sp = std::sqrt(dot(v, v));
      P.t = r[6 * n + id];
      P.w = r[7 * n + id];
      if (!(sp > 0.0) || !std::isfinite(sp) || !(P.w > 0.0) || !std::isfinite(P.w) ||
          !std::isfinite(P.t)) {
        P.dir = {0.0, 0.0, 1.0};
        P.speed = 1.0;
        P.w = 0.0;
        return;
      }
      P.dir = scale(v, 1.0 / sp);
      P.speed = sp;
      // a binary32 normalisation of the velocity: |v| by a square root and
      // three divisions of up to 2.5 ulp each (about 3e-7 per component)
      P.ddir = 5e-7;
      return;
    }
    double u[4];
    double E = B.E;
    uint32_t block = 0;
    rng.draw(id, STREAM_SOURCE, 1u, block, u);
    double x = (u[0] - 0.5) * B.W;
    double y = (u[1] - 0.5) * B.H;
    if (B.type == BEAM_GAUSS) {
      for (;;) {
        // Box-Muller on the last two words of the block
        E = B.E * (1.0 + B.sigma_rel * std::sqrt(-2.0 * std::log(u[2])) * std::cos(2.0 * kPi * u[3]));
        if (E > 0.0) break;
        rng.draw(id, STREAM_SOURCE, 1u, ++block, u);
      }
    }
    P.pos = {x, y, B.z0};
    P.dir = {0.0, 0.0, 1.0};
    P.speed = std::sqrt(E / kEperV2);
    P.t = B.z0 / P.speed;
    P.w = 1.0;
  }
};

}  // namespace

extern "C" {

int oracle_abi_version(void) { return 5; }

// grid index the coherent one-phonon kernel (scatterer s, kernel j) reads for
// a point K of reciprocal space (crystal frame, 1/A); -1 for another kernel
int64_t oracle_cohphonon_index(const OSetup* S, int s, int j, const double K[3]) {
  const OKernel& k = S->s[s].k[j];
  if (k.type != K_COH_PHONON) return -1;
  double m = kHuge;
  return cohphonon_index(k, {K[0], K[1], K[2]}, &m);
}

// A_1 masses of a multi-phonon kernel (2 nbins values, index as in
// a1_masses, before normalisation) and their sum; returns 0, or 2 if the
// kernel is not a multi-phonon kernel.
int oracle_multiphonon_a1(const OSetup* S, int s, int j, double* masses, double* sum) {
  const OKernel& k = S->s[s].k[j];
  if (k.type != K_MULTIPHONON) return 2;
  std::vector<double> m;
  a1_masses(k, m, sum);
  for (size_t i = 0; i < m.size(); ++i) masses[i] = m[i];
  return 0;
}
int oracle_sizeof_setup(void) { return (int)sizeof(OSetup); }
int oracle_sizeof_record(void) { return (int)sizeof(ORecord); }
int oracle_sizeof_tally(void) { return (int)sizeof(OTally); }

void oracle_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                   uint32_t out[4]) {
  Block b = philox4x32_10(c0, c1, c2, c3, k0, k1);
  for (int i = 0; i < 4; ++i) out[i] = b.w[i];
}

double oracle_uniform(uint32_t x) { return to_uniform(x); }

// Intervals of one shape along a ray (lab frame), for geometry pins.
int oracle_shape_intervals(const OShape* sh, const double p[3], const double d[3], double lo[2],
                           double hi[2]) {
  V3 P = {p[0], p[1], p[2]}, D = {d[0], d[1], d[2]};
  V3 pl = matTvec(sh->rot, sub(P, {sh->pos[0], sh->pos[1], sh->pos[2]}));
  V3 dl = matTvec(sh->rot, D);
  double m = kHuge;
  return shape_intervals(*sh, pl, dl, lo, hi, &m);
}

// Attenuation coefficients (1/m) of scatterer s at speed v: out = {mu_k[0..2], mu_s, mu_abs}.
void oracle_attenuation(const OSetup* S, int s, double speed, double out[5]) {
  std::vector<ScatInfo> info;
  prepare(*S, info);
  double m = kHuge;
  Mu mu = attenuation(S->s[s], info[s], speed, &m);
  for (int j = 0; j < 3; ++j) out[j] = j < S->s[s].nk ? mu.k[j] : 0.0;
  out[3] = mu.scat;
  out[4] = mu.abs;
}

// Debye-Waller coefficient 2W/Q^2 (A^2) of scatterer s, and gamma_0 of kernel j.
double oracle_dw_coef(const OSetup* S, int s) {
  std::vector<ScatInfo> info;
  prepare(*S, info);
  return info[s].dw_coef;
}
double oracle_gamma0(const OKernel* k) { return gamma0(*k); }

// One kernel draw for an incident packet with speed v along dir, with the
// eight uniforms u[0..7] (u[2..7] are the kernel's) and, for the
// multi-phonon kernel, the uniforms of its extra blocks (4 per block, up to
// 4 blocks; may be null otherwise).  out = {vx,vy,vz,factor}.
void kernel_sample_prepared(const OSetup* S, const std::vector<ScatInfo>& info, int s, int j,
                            const double dir[3], double speed, const double u[8],
                            const double* extra, double out[4]) {
  Packet P{};
  P.dir = {dir[0], dir[1], dir[2]};
  P.speed = speed;
  double m = kHuge;
  const OKernel& k = S->s[s].k[j];
  Scatter r;
  switch (k.type) {
    case K_ISO_EL: r = k_iso(k, info[s], P, u); break;
    case K_POWDER: r = k_powder(k, info[s].k[j], info[s], P, u, &m); break;
    case K_PHONON: r = k_phonon(k, info[s].k[j], info[s], P, u, &m); break;
    case K_SPINWAVE: r = k_spinwave(k, P, u); break;
    case K_MULTIPHONON:
      r = k_multiphonon(k, info[s].k[j], P, u,
                        [&](int b, double v[4]) {
                          for (int i = 0; i < 4; ++i) v[i] = extra[4 * b + i];
                        },
                        &m);
      break;
    case K_DISPERSION: r = k_dispersion(k, P, u, &m); break;
    case K_COH_PHONON: r = k_cohphonon(k, info[s].k[j], info[s], P, u, &m); break;
    default: r = k_sqe(k, P, u, &m); break;
  }
  out[0] = r.dir.x * r.speed;
  out[1] = r.dir.y * r.speed;
  out[2] = r.dir.z * r.speed;
  out[3] = r.factor;
}

void oracle_kernel_sample(const OSetup* S, int s, int j, const double dir[3], double speed,
                          const double u[8], const double* extra, double out[4]) {
  std::vector<ScatInfo> info;
  prepare(*S, info);
  kernel_sample_prepared(S, info, s, j, dir, speed, u, extra, out);
}

// n draws with the same incident state: u is n x 8, extra n x 16 (or null),
// out n x 4.
void oracle_kernel_sample_many(const OSetup* S, int s, int j, const double dir[3], double speed,
                               int64_t n, const double* u, const double* extra, double* out) {
  std::vector<ScatInfo> info;
  prepare(*S, info);
  for (int64_t i = 0; i < n; ++i)
    kernel_sample_prepared(S, info, s, j, dir, speed, u + 8 * i,
                           extra ? extra + 16 * i : nullptr, out + 4 * i);
}

// Full transport of histories [first, first+n).  hist (and hist_w2 if not
// null) are accumulated into.  Records of every escaping packet go to recs
// (up to rec_cap); *n_rec gets the total count.
// Transport with weights evaluated at S and every random choice drawn from
// the proposal Sp (Sp = S for a plain run).  Sp may differ from S only in
// table values and cross sections, not in structure.
int oracle_run2(const OSetup* S, const OSetup* Sp, uint64_t seed, uint64_t first, uint64_t n,
                double* hist, double* hist_w2, ORecord* recs, uint64_t rec_cap, uint64_t* n_rec,
                OTally* tally) {
  if (S->K < 0 || S->K > 7) return 1;
  std::memset(tally, 0, sizeof(OTally));
  Sim sim(*S, *Sp);
  prepare(*S, sim.info);
  prepare(*Sp, sim.pinfo);
  sim.rng.seed = seed;
  sim.rng.tally = tally;
  sim.hist = hist;
  sim.hist_w2 = hist_w2;
  sim.recs = recs;
  sim.rec_cap = rec_cap;
  sim.n_rec = 0;
  sim.tally = tally;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t id = first + i;
    Packet P;
    sim.source(id, P);
    if (P.w > 0.0) sim.process(P, id);  // invalid saved entries carry no history
  }
  if (n_rec) *n_rec = sim.n_rec;
  return 0;
}

int oracle_run(const OSetup* S, uint64_t seed, uint64_t first, uint64_t n, double* hist,
               double* hist_w2, ORecord* recs, uint64_t rec_cap, uint64_t* n_rec, OTally* tally) {
  return oracle_run2(S, S, seed, first, n, hist, hist_w2, recs, rec_cap, n_rec, tally);
}

// Forward-mode gradient of sum_b dLdI[b] I_b with respect to the parameters
// of `pm`, with every random choice frozen at S (the weights of a path are
// its true density over the proposal density at S).  grad[] is accumulated
// into; its length is nbins(DOS) + cells(S(Q,E)) + 2.  gabs and gflag
// (nullable, same length, accumulated into) receive the sums of the
// absolute per-packet terms over all recorded packets and over the
// near-decision ones.
int oracle_gradient(const OSetup* S, const OParamMap* pm, uint64_t seed, uint64_t first,
                    uint64_t n, const double* dLdI, double* grad, double* gabs, double* gflag,
                    OTally* tally) {
  if (S->K < 0 || S->K > 7) return 1;
  int nb = 0, nc = 0;
  if (pm->dos_s >= 0) {
    const OKernel& kd = S->s[pm->dos_s].k[pm->dos_k];
    if (kd.type != K_PHONON) return 2;
    nb = kd.nbins;
    if (pm->mp_k >= 0) {
      const OKernel& km = S->s[pm->dos_s].k[pm->mp_k];
      if (km.type != K_MULTIPHONON || km.nbins != nb) return 2;
    }
  } else if (pm->mp_k >= 0) {
    return 2;
  }
  if (pm->sqe_s >= 0) {
    const OKernel& kq = S->s[pm->sqe_s].k[pm->sqe_k];
    if (kq.type != K_SQE) return 2;
    nc = kq.nQ * kq.nE;
  }
  std::memset(tally, 0, sizeof(OTally));
  Sim sim(*S, *S);
  prepare(*S, sim.info);
  prepare(*S, sim.pinfo);
  sim.tangent = true;
  sim.pm = *pm;
  sim.nb = nb;
  sim.nc = nc;
  sim.np = nb + nc + 2;
  sim.dLdI = dLdI;
  sim.grad = grad;
  sim.gabs = gabs;
  sim.gflag = gflag;
  sim.rng.seed = seed;
  sim.rng.tally = tally;
  sim.hist = nullptr;
  sim.hist_w2 = nullptr;
  sim.recs = nullptr;
  sim.rec_cap = 0;
  sim.n_rec = 0;
  sim.tally = tally;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t id = first + i;
    Packet P;
    sim.source(id, P);
    if (P.w > 0.0) sim.process(P, id);  // invalid saved entries carry no history
  }
  return 0;
}

}  // extern "C"
