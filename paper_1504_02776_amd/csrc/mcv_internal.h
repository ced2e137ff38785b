// mcv_internal.h -- device-side plan layout shared by the host library and
// the HIP kernels of the transport library (not part of the public ABI).
//
// A plan is a flat POD copied once to device memory and, at the start of
// every workgroup, into LDS together with its binary32 tables, so that
// per-lane (divergent) lookups of scatterer and kernel parameters are LDS
// reads instead of scratch or kernarg traffic.
#ifndef MCV_INTERNAL_H
#define MCV_INTERNAL_H

#include <stdint.h>

namespace mcv {

constexpr int kMaxScat = 4;
constexpr int kMaxKern = 3;
constexpr int kMaxRows = 8;
constexpr int kMaxSlots = 2 * kMaxScat;  // material intervals per flight
constexpr int kMaxOrders = 7;
// words per stacked packet: position, direction, speed, time, weight,
// lineage, code, and for a child not built yet its interval's distance and
// interaction probability
constexpr int kFields = 13;

enum { SHAPE_BOX = 1, SHAPE_CYLINDER = 2, SHAPE_ANNULUS = 3 };
enum { K_ISO_EL = 1, K_POWDER = 2, K_PHONON = 3, K_SPINWAVE = 4, K_SQE = 5, K_MULTIPHONON = 6,
       K_DISPERSION = 7, K_COH_PHONON = 8 };
enum { DET_SPHERE = 1, DET_TUBES = 2 };
enum { STREAM_SOURCE = 0u, STREAM_SCATTER = 1u, STREAM_DETECT = 2u };

struct DevKernel {
  int32_t type;
  int32_t dw;
  float mu;          // 100 n sigma (1/m); POWDER: unused
  // POWDER: mu_B(lambda) = bragg_coef * lambda^2 * prefix[n_active - 1]
  float bragg_coef;  // 100 / (2 v0^2)
  int32_t t_d;       // offset of d-spacings sorted by descending d
  int32_t t_pref;    // offset of prefix sums of d |F|^2 in that order
  int32_t nrefl;
  // PHONON (and MULTIPHONON: t_cdf = cumulative A_1 over 2 nbins bins)
  int32_t t_cdf;     // offset of the normalised cumulative DOS
  int32_t nbins;
  float de;          // bin width, meV
  float kT;          // meV
  float h2m;         // hbar^2 / 2M, meV A^2
  // MULTIPHONON
  float dw_self;     // 2W / Q^2 from the kernel's own DOS, A^2
  int32_t nmax;      // highest order N
  // SPINWAVE and DISPERSION (COH_PHONON: wmax = largest mode energy, crot =
  // rows n a_j / 2 pi giving grid coordinates, nbins = n, kT, h2m)
  float j4s;         // 4 J S
  float a;           // lattice constant
  float gamma;       // HWHM
  float wmax;        // 24 J S
  float crot[9];     // lab -> crystal
  // SQE
  int32_t t_s;
  int32_t nQ, nE;
  float Qmax, Emin, Emax;
  float q_scale;     // nQ / Qmax
  float e_scale;     // nE / (Emax - Emin)
  // COH_PHONON: device address of the mode table (12 floats per grid point)
  uint32_t grid_lo, grid_hi;
};

struct DevScat {
  int32_t shape;
  int32_t nk;
  int32_t ident;     // 1: rot is the identity (the shape frame is the lab frame shifted)
  int32_t pad;
  float h[3];        // BOX: half lengths; CYLINDER: r, h/2, -; ANNULUS: r_in, r_out, h/2
  float pos[3];
  float rot[9];      // local -> lab, row major
  float mu_abs2200;  // 100 n sigma_abs * 2200 (1/m * m/s)
  float n100;        // 100 n: d mu / d sigma (1/m per barn)
  float dw_coef;     // 2W / Q^2 (A^2)
  DevKernel k[kMaxKern];
};

struct DevDet {
  int32_t type;
  int32_t ntof;
  float tof_lo;
  float inv_dt;      // ntof / (tof_hi - tof_lo)
  float R;
  // sphere
  int32_t n2t;
  float ring_scale;  // n2t / pi
  // tubes
  int32_t nrows, ncols, npix;
  float phi_lo, inv_dphi;
  int32_t tpp;          // tubes per pack (0: evenly spaced columns)
  float pack_pitch;     // azimuth of one pack plus its gap
  float inv_pack_pitch;
  float inv_tube_pitch;
  float row_y[kMaxRows];
  float half_len;
  float radius;
  float mu_he2200;   // 100 n_He 5333 * 2200
  float pix_scale;   // npix / length
  int32_t t_cols;    // offset of (x_c, z_c) per column
};

// histogram bins are addressed with 32-bit indices on the device
constexpr int64_t kMaxBins = (int64_t)1 << 31;

// LDS histogram bin cache of a workgroup: slots (a power of two) and size in
// 32-bit words (double v[n], double v2[n], int tag[n])
constexpr int kHotMin = 64;
constexpr int kHotMax = 1024;
constexpr int hot_words(int n) { return 5 * n; }
// histograms up to this many bins send every update through the cache
constexpr int64_t kHotAllBins = 1 << 18;

// 16-byte aligned and sized: the kernels place their dynamic LDS (which holds
// binary64 partial sums in adjoint mode) right after a copy of the plan, and
// binary64 LDS accesses must be 8-byte aligned.
struct alignas(16) DevPlan {
  int32_t nscat;
  int32_t K;
  int32_t smax;       // largest number of material intervals on one ray
  int32_t stack_cap;  // stacked packets per lane = (smax - 1) * K
  float min_prob;
  int32_t n_tables;   // binary32 words in the table blob
  int32_t hot_n;      // slots of the LDS histogram bin cache (power of two)
  int32_t hot_all;    // 1: every histogram update tries the cache (small histograms)
  int32_t heavy;      // 1: an exact-delta dispersion or coherent phonon kernel is present
  int32_t pad0;
  DevScat s[kMaxScat];
  DevDet det;
};
static_assert(sizeof(DevPlan) % 16 == 0, "plan copy must keep the dynamic LDS 16-byte aligned");

// Parameters of an adjoint run and where it accumulates.  The table
// parameters form one vector [DOS values of one one-phonon kernel (nb) |
// cells of one S(Q,E) grid (nc)]; a packet carries the indices into it of the
// table entries its ancestry drew (one per one-phonon or S(Q,E) draw, n per
// n-phonon draw of a multi-phonon kernel tied to the same DOS).
struct AdjArgs {
  int32_t dos_s, dos_k, abs_s, sig_s, sig_k;
  int32_t sqe_s, sqe_k, mp_k;  // -1: none
  int32_t nb, nc;              // DOS bins, S(Q,E) cells
  int32_t sparse_lds;          // 1: table partials in LDS, 0: global atomics
  int32_t pad;
  const double* dLdI;          // per histogram bin
  double* grad;                // [nb + nc + 2]: DOS bins, S(Q,E) cells, sigma_abs, sigma
  // workspace (binary64): [0] sum g A, [1] sum g n_draws (the dense DOS
  // terms), [2] dnorm, [3] unused, [4, 4 + nb + nc) 1 / table value,
  // [4 + nb + nc, 4 + 2 nb + nc) dense_a (per unit of sum Q^2)
  double* ws;
};

constexpr int kAdjFields = 10;     // extra words per stacked packet in adjoint mode
// binary32 words of one stacked packet entry, without or with the adjoint
// carry, padded to a multiple of 4 (moved with 16-byte accesses)
constexpr int stack_words(bool carry) { return (kFields + (carry ? kAdjFields : 0) + 3) & ~3; }
constexpr int kAdjMaxOrders = 4;
constexpr int kAdjMaxSparse = 12;  // table indices a packet carries (16 bits each)
constexpr int kAdjMaxTable = 65535;
// binary64 values of the adjoint workspace that mcv_adjoint_noalloc keeps in
// static device memory (4 + 2 nb + nc must fit): 256 KiB per device
constexpr int kNoAllocWorkDoubles = 32768;
// the adjoint-partials argument of the LDS size computation for launches
// that are not adjoint
constexpr int kLdsNoAdjoint = -1;

// Deterministic summation of one chunk of histories: the transport appends
// (key, value) per recorded packet, key = bin << (id_bits + lin_bits) |
// (id - first) << lin_bits | lineage; sorted, each bin's run is summed in
// key order.
struct DetArgs {
  uint64_t* keys;
  float* vals;
  uint64_t cap;
  unsigned long long* n;  // device counter of entries (zeroed before the chunk)
  uint64_t first;
  int32_t lin_bits, id_bits;
};

// Adjoint tape: one entry per recorded packet (bin >= 0) of a forward run,
// [field][entry] with `cap` entries per field: bin, value (binary32 bits),
// then the packet's adjoint carry (kAdjFields words: d log w / d sigma_abs,
// d log w / d sigma, A, counts, packed table indices).
constexpr int kTapeFields = 2 + kAdjFields;
struct TapeArgs {
  uint32_t* words;
  uint64_t cap;
  unsigned long long* n;  // device counter, advanced by the entries recorded
};

struct DevBeam {
  int32_t type;  // 1 mono, 2 gauss, 3 saved
  float E, sigma_rel, W, H, z0;
  const float* saved;  // SAVED: rows x, y, z, vx, vy, vz, t, p of n_saved entries
  uint64_t n_saved;
};

// one simulation of a batch
struct BatchItem {
  const DevPlan* plan;
  const float* tables;
  DevBeam beam;
  uint64_t seed;
  uint64_t id0;  // first history id
  double* hist;
};

// a range of histories [id0 + first, id0 + first + count) of one item
struct BatchChunk {
  uint32_t item;
  uint32_t count;
  uint64_t first;
};

struct DevRecord {  // mirrors mcv_packet_record
  uint64_t id;
  uint32_t lineage;
  int32_t order;
  float pos[3];
  float vel[3];
  float t;
  float w;
  int64_t bin;
  float value;
  float tof;
  int32_t tube;
  int32_t pixel;
};

struct DevEvent {  // mirrors mcv_event
  uint32_t pixel;
  float tof;
  float value;
  int32_t order;
};

// Mapping of detector data to (Q, E) bins, binary32 (the reduction)
struct QEMap {
  float Ei;         // meV
  float ki2;        // k_i^2, 1/A^2
  float two_ki;     // 2 k_i
  float e_per_v2;   // meV per (m/s)^2
  float k_per_v;    // 1/A per m/s
  float q_lo, q_scale;  // nq / (q_hi - q_lo)
  float e_lo, e_scale;
  int32_t nq, ne;
  float tof_lo, dt;     // time bins of the detector
  int32_t ntof;
  uint32_t npixels;
  int32_t pad;
};

}  // namespace mcv

#endif
