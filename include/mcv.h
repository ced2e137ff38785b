/* mcv.h -- C ABI of the MI355X weighted neutron-transport library.
 *
 * The calls follow the paper's statement of the problem (arXiv:1504.02776,
 * Sec. 3 four-step workflow): a beam of neutron packets is sent through a
 * sample assembly (Sec. 2.4.1-2.4.3, composite scatterer, multiple
 * scattering; Supplement S3), the scattered packets are intercepted by a
 * detector system (Sec. 2.4.3, "Ray tracing in a detector system"), and the
 * intensity of a (pixel, time-of-flight) bin is the sum of the probabilities
 * of the packets recorded in it (Sec. 3, "Reduction").
 *
 * Conventions
 *   - Every call returns an mcv_status; mcv_last_error() gives a message for
 *     the last failing call of the calling thread.  No exception crosses the
 *     ABI.  A device fault of an earlier asynchronous launch is reported by a
 *     later call or by mcv_sync().
 *   - Units: energies meV; cross sections barn (absorption at 2200 m/s, 1/v
 *     law); number densities atoms per cubic angstrom; d-spacings, lattice
 *     constants angstrom; cell volumes cubic angstrom; geometry metre; time
 *     second; temperature kelvin; masses atomic mass units.
 *   - Lab frame: beam along +z, y vertical.  t = 0 when an incident packet
 *     crosses z = 0.
 *   - Handles (mcv_assembly, mcv_detector, mcv_plan) belong to the library
 *     and are released with their *_destroy call.  Host arrays passed to the
 *     builders are copied during the call.  Device buffers (histograms, packet
 *     records, counters, gradients, workspaces) belong to the caller; the
 *     library never frees them.
 *   - Streams are passed as `void*` holding a hipStream_t (NULL: the null
 *     stream).  Launches are asynchronous on that stream.
 *   - Precision: packet state and kernel sampling in binary32; histogram
 *     accumulation in binary64; host-side table preparation in binary64,
 *     stored as binary32 on the device.
 */
#ifndef MCV_H
#define MCV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MCV_OK = 0,
  MCV_EINVAL = 1,        /* bad argument; nothing was launched or changed */
  MCV_EUNSUPPORTED = 2,  /* outside the supported configuration space     */
  MCV_EOVERLAP = 3,      /* scatterer volumes may overlap                 */
  MCV_ENOMEM = 4,        /* device or host allocation failed              */
  MCV_ECAPACITY = 5,     /* an output buffer is too small                 */
  MCV_EHIP = 6           /* a HIP runtime call failed                     */
} mcv_status;

typedef struct mcv_assembly_s* mcv_assembly;
typedef struct mcv_detector_s* mcv_detector;
typedef struct mcv_plan_s* mcv_plan;

/* ---------------------------------------------------------------- shapes */
enum { MCV_SHAPE_BOX = 1, MCV_SHAPE_CYLINDER = 2, MCV_SHAPE_ANNULUS = 3 };

/* Sec. 2.4.2 (shapes of homogeneous scatterers).
 * BOX: dims = full lengths along local x, y, z.
 * CYLINDER: dims = {radius, height, unused}; axis = local y.
 * ANNULUS: dims = {inner radius, outer radius, height}; the outer cylinder
 *   minus the inner cylinder of the same height (a can wall, open ends).
 * pos: lab position of the shape centre; rot: local->lab rotation (row
 * major, orthonormal). */
typedef struct {
  int32_t type;
  int32_t reserved;
  double dims[3];
  double pos[3];
  double rot[9];
} mcv_shape;

/* Homogeneous material: n atoms/A^3 (or formula units, consistent with the
 * kernels' sigma), absorption cross section sigma_abs at 2200 m/s. */
typedef struct {
  double n_per_A3;
  double sigma_abs_b;
} mcv_material;

/* --------------------------------------------------------------- kernels */
enum {
  MCV_K_ISO_EL = 1,    /* incoherent elastic (Supplement S4)                  */
  MCV_K_POWDER = 2,    /* coherent elastic powder, Debye-Scherrer cones (S4)  */
  MCV_K_PHONON = 3,    /* incoherent one-phonon from a DOS (S4)               */
  MCV_K_SPINWAVE = 4,  /* dispersion surface E(Q), S(Q) = 1, Lorentzian (S4)  */
  MCV_K_SQE = 5,       /* tabulated isotropic S(Q,E) (Sec. 2.4.2)             */
  MCV_K_MULTIPHONON = 6, /* incoherent multi-phonon, orders 2..N (S4)         */
  MCV_K_DISPERSION = 7,  /* dispersion surface E(Q), exact delta (S4)         */
  MCV_K_COH_PHONON = 8   /* coherent one-phonon, powder, from BZ modes (S4)    */
};

/* One scattering kernel.  Only the fields of `type` are read.
 *   sigma_b: nominal cross section per atom; the kernel's attenuation
 *     coefficient is 100 n sigma_b per metre (not used by POWDER, whose cross
 *     section is the sum of its cones at the packet's wavelength).
 *   dw: 1 = multiply by the Debye-Waller factor exp(-2W), 2W = (hbar^2 Q^2 /
 *     2M) gamma_0, with M, T and gamma_0 from the PHONON kernel of the same
 *     scatterer (which must exist).
 *   POWDER: v0 cell volume; nrefl reflections with d-spacing d[i] and
 *     F2[i] = multiplicity * |F|^2 per cell (barn).
 *   PHONON: mass M_amu, temperature T_K (> 0), nbins DOS values dos[] (raw,
 *     >= 0, normalised by the library) on bins of width emax/nbins over
 *     [0, emax].
 *   MULTIPHONON: the same DOS fields, and max_phonons = N (2..8): S(Q,E) =
 *     sum_{n=2..N} (2W)^n/n! e^{-2W} A_n(E) with A_n the n-fold convolution
 *     of the one-phonon spectrum A_1 (Supplement S4, incoherent
 *     approximation); 2W and A_1 from this kernel's own DOS, M and T.  Its
 *     Debye-Waller factor is part of S_n, so dw must be 0.  Draws beyond the
 *     eight uniforms of a split come from blocks 2, 3, ... of the packet's
 *     scattering stream.  The adjoint does not differentiate through this
 *     kernel's DOS.
 *   SPINWAVE: E(Q) = 4 J S (3 - sum_a cos(Q_a a)), Q in the crystal frame
 *     crot * Q_lab; gamma = Lorentzian HWHM.
 *   DISPERSION: the same E(Q) (J S >= 0) with an exact delta function in
 *     energy, S(Q) = 1: for an isotropic outgoing direction the outgoing
 *     wave numbers solving E_i - E_f = E(Q) are bracketed on 256 equal cells
 *     of [0, k_i] (root pairs closer than a cell are not resolved) and one is
 *     taken at random; weight n k_f/k_i / |dG/dE_f|.  gamma is not read.
 *   SQE: S(Q,E) on nQ x nE cells over [0, Qmax] x [Emin, Emax], row major
 *     with Q slow; E is the energy transfer to the sample.
 *   COH_PHONON: coherent one-phonon scattering from a powder of a crystal
 *     with one atom of mass M_amu per primitive cell, temperature T_K (> 0).
 *     cell = the primitive lattice vectors a_1, a_2, a_3 (rows, A, crystal
 *     frame); modes = the phonons on the grid_n^3 points (2..128 per axis)
 *     of the reciprocal cell, point (i, j, k) = (i b_1 + j b_2 + k b_3) /
 *     grid_n with b_i . a_j = 2 pi delta_ij, at index ((i grid_n + j) grid_n
 *     + k) * 12: three mode energies (meV, >= 0) then their three unit
 *     polarization vectors (crystal frame).  A draw takes K uniform in the
 *     ball |K| <= k_i + k_f,max (k_f,max for E_i plus the largest mode
 *     energy), the modes of the grid point nearest to K (fractional
 *     coordinates K . a_j / 2 pi rounded, periodic), a branch at random,
 *     phonon creation with probability (n+1)/(2n+1), and the outgoing
 *     direction on the cone |k_i - k_f| = |K| about the incident direction;
 *     weight Q_max^3 coth(E_s/2kT) e^{-2W} (hbar^2/2M)(K.e_s)^2 / E_s /
 *     (2 k_i^2 |K|) (Supplement S4, per unit sigma_b).  Modes below 1e-3 meV
 *     scatter with weight 0.  The table lives in device memory (not LDS). */
typedef struct {
  int32_t type;
  int32_t dw;
  double sigma_b;
  double v0;
  int32_t nrefl;
  int32_t reserved0;
  const double* d;
  const double* F2;
  double M_amu;
  double T_K;
  int32_t nbins;
  int32_t max_phonons;
  double emax;
  const double* dos;
  double J, S, a, gamma;
  double crot[9];
  int32_t nQ, nE;
  double Qmax, Emin, Emax;
  const double* sqe;
  int32_t grid_n;
  int32_t reserved1;
  double cell[9];
  const double* modes;
} mcv_kernel;

/* ------------------------------------------------------------- assembly */
/* Sample assembly: up to 4 homogeneous scatterers, each with up to 3
 * kernels (Sec. 2.4.1 composite scatterer, flattened). */
mcv_status mcv_assembly_create(mcv_assembly* out);

/* Adds a scatterer; *idx receives its index.  Errors: MCV_EINVAL for a bad
 * shape, material or kernel; MCV_EUNSUPPORTED beyond 4 scatterers, 3
 * kernels, or 7 material intervals per ray over the assembly (box and
 * cylinder count 1, annulus 2); MCV_EOVERLAP when the new volume cannot be
 * shown disjoint from an existing one (disjoint bounding boxes, or the new
 * shape inside the hole of an annulus, or vice versa).  Arrays are copied. */
mcv_status mcv_assembly_add(mcv_assembly a, const mcv_shape* shape, const mcv_material* mat,
                            const mcv_kernel* kernels, int32_t nk, int32_t* idx);
mcv_status mcv_assembly_destroy(mcv_assembly a);

/* ------------------------------------------------------------- detectors */
/* Sphere of radius R about the origin (Sec. 2.4.3): bin = ring * n_tof +
 * tof_bin, ring = floor(2theta / (pi / n_2theta)) with 2theta the angle of
 * the hit point from +z; tof bins of equal width on [tof_lo, tof_hi);
 * packets outside the window are not recorded.  Recorded value = weight. */
mcv_status mcv_detector_sphere(mcv_detector* out, double R, int32_t n_2theta, int32_t n_tof,
                               double tof_lo, double tof_hi);

/* Vertical 3He tubes (Sec. 2.4.3, "Ray tracing in a detector system"): tube
 * (row r, column c) has its axis at (R sin phi_c, ., R cos phi_c), phi_c =
 * phi_lo + (c + 1/2)(phi_hi - phi_lo)/ncols, spanning y in row_y[r] -+
 * length/2; radius `radius`; 3He density n_he (atoms/A^3, absorption
 * 5333 b at 2200 m/s, 1/v).  Only the first tube on a packet's ray records:
 * value = weight * (1 - exp(-mu_He chord)); the absorption point is drawn
 * on the chord; pixel = floor(n_pix (y_abs - y_bottom) / length); bin =
 * ((tube * n_pix + pixel) * n_tof + tof_bin), tube = r * ncols + c.
 * Packs (Sec. 2.1 and 2.4.1: 8 tubes make an 8-pack, packs make the detector
 * system): with tubes_per_pack = P > 0 the columns form ncols / P packs with
 * pack_gap radians of extra azimuth between neighbouring packs, and the tube
 * pitch d = (phi_hi - phi_lo - (ncols/P - 1) pack_gap) / ncols puts column c
 * at phi_c = phi_lo + floor(c/P) pack_gap + (c + 1/2) d; P = 0: evenly
 * spaced columns (pack_gap not read).
 * Requirements: row_y ascending, nrows <= 8, neighbouring tubes do not
 * overlap, R >= 10 radius, P divides ncols, pack_gap >= 0. */
typedef struct {
  int32_t nrows, ncols;
  double R, phi_lo, phi_hi;
  double row_y[8];
  double length, radius, n_he;
  int32_t tubes_per_pack;
  int32_t reserved;
  double pack_gap;
} mcv_tube_layout;

mcv_status mcv_detector_tubes(mcv_detector* out, const mcv_tube_layout* layout, int32_t n_pix,
                              int32_t n_tof, double tof_lo, double tof_hi);
/* number of histogram bins (int64 so that 1.28e8-bin layouts are exact) */
int64_t mcv_detector_nbins(mcv_detector d);
mcv_status mcv_detector_destroy(mcv_detector d);

/* ----------------------------------------------------------------- plans */
/* max_orders: maximum number of scattering events of a packet (Supplement
 * S3 max_ms); packets that reach it cross the remaining material with
 * attenuation only.  min_prob: packets below it are not split (0 = off).
 * block_size: threads per workgroup (0 = default 256; 64, 128, 192 or 256).
 * waves_per_simd: grid depth, the waves per SIMD the grid of a launch is
 * sized for (0 = default 16, lowered for plans whose packet stacks would
 * pass 2 GiB): a launch spreads its histories over up to 2 x 4 x CUs x
 * waves_per_simd waves, each taking a contiguous id range of at least 512
 * histories once it has more than two rounds of 4 waves per SIMD.  The
 * plan's packet stacks are sized for that grid.
 * deterministic: 1 = mcv_run sums every histogram bin in a fixed order, so
 *   that two runs with the same arguments give bitwise equal histograms
 *   (Sec. 3: a bin's intensity is the sum of the probabilities of the
 *   packets recorded in it).  The ids are taken in chunks (at most 2^16
 *   histories); per chunk the packets recorded are sorted by (bin, history
 *   id, lineage), each bin's run is summed in that order in binary64 and
 *   added to the bin, chunks in id order.  mcv_run then waits for the
 *   stream once per chunk (it reads the number of recorded packets) and is
 *   several times slower; the plan holds a device workspace for it.  Other
 *   calls (mcv_trace, mcv_run_events, batches, the adjoint) are unaffected.
 *   0 = binary64 atomics in arrival order (sums equal up to rounding order).
 * max_waves: upper bound on the wavefronts a launch spreads its histories
 *   over (each wave then traces about n / max_waves histories one after
 *   another); 0 = enough waves to fill the device. */
typedef struct {
  int32_t max_orders;
  int32_t block_size;
  double min_prob;
  int32_t waves_per_simd;
  int32_t deterministic;
  int64_t max_waves;
} mcv_opts;

/* Validates the assembly with the detector and uploads the device tables to
 * `device`.  The plan keeps its own copies; assembly and detector may be
 * destroyed afterwards.  Errors: MCV_EINVAL, MCV_EUNSUPPORTED (sample not
 * well inside the detector radius, max_orders > 7), MCV_ENOMEM, MCV_EHIP. */
mcv_status mcv_plan_create(mcv_plan* out, mcv_assembly a, mcv_detector d, const mcv_opts* opts,
                           int32_t device);
mcv_status mcv_plan_destroy(mcv_plan p);
int64_t mcv_plan_nbins(mcv_plan p);

/* ------------------------------------------------------------------ beam */
enum { MCV_BEAM_MONO = 1, MCV_BEAM_GAUSS = 2, MCV_BEAM_SAVED = 3 };

/* Uniform W x H rectangle at z = z0 < 0, collimated along +z.  MONO: energy
 * E.  GAUSS: E (1 + sigma_rel g), g standard normal by Box-Muller, redrawn
 * while E <= 0 (sigma_rel <= 0.2).
 * SAVED: neutrons saved at the sample position by an earlier step of the
 * workflow (Sec. 3: the beam simulation's neutrons are saved and reused):
 * `saved` = device binary32 rows x, y, z (m), vx, vy, vz (m/s), t (s), p
 * (weight), each of n_saved entries (row r of entry i at saved[r * n_saved
 * + i]); history id i starts from entry i (ids must stay below n_saved;
 * the source stream is not used).  Entries with p <= 0, zero speed or a
 * non-finite value carry no history.  E, sigma_rel, W, H, z0 are not read;
 * the caller keeps the array alive and inside the detector's volume. */
typedef struct {
  int32_t type;
  int32_t reserved;
  double E, sigma_rel, W, H, z0;
  const float* saved;
  uint64_t n_saved;
} mcv_beam;

/* ------------------------------------------------------------ transport */
/* Traces histories first .. first+n-1 (ids) through the assembly and adds
 * their recorded values to hist[nbins] (device, binary64) and, if hist_w2 is
 * not NULL, their squares to hist_w2[nbins].  Random numbers: Philox4x32-10
 * keyed by `seed`, counter (id_lo, id_hi | stream << 30, lineage, block), so
 * disjoint id ranges are independent and their sums equal one larger run
 * (up to binary64 summation order).  Errors: MCV_EINVAL (null hist, n >
 * 2^62, bad beam), MCV_EHIP. */
mcv_status mcv_run(mcv_plan p, const mcv_beam* beam, uint64_t seed, uint64_t first, uint64_t n,
                   double* hist, double* hist_w2, void* stream);

/* One record per packet leaving the sample assembly (the paper's saved
 * scattered neutrons, Sec. 3 step 2, joined with the detector result). */
typedef struct {
  uint64_t id;       /* history id */
  uint32_t lineage;  /* 1 for the source packet; child of segment g of a
                        packet with lineage L: 8 L + g + 1 */
  int32_t order;     /* number of scattering events */
  float pos[3];      /* where it leaves the assembly */
  float vel[3];
  float t;
  float w;
  int64_t bin;       /* -1: missed or outside the window */
  float value;       /* recorded value */
  float tof;
  int32_t tube;      /* -1 for the sphere or a miss */
  int32_t pixel;
} mcv_packet_record;

/* Same transport as mcv_run, also writing records (device array of
 * `capacity`) in arbitrary order; *n_out_dev (device uint64, zeroed by the
 * caller) receives the number of packets, which may exceed capacity (then
 * only `capacity` records are written and the caller sees the overflow).
 * hist may be NULL here. */
mcv_status mcv_trace(mcv_plan p, const mcv_beam* beam, uint64_t seed, uint64_t first, uint64_t n,
                     double* hist, mcv_packet_record* records, uint64_t capacity,
                     uint64_t* n_out_dev, void* stream);

/* ----------------------------------------------------------- event mode */
/* One detector event (Sec. 2.4.3 and Sec. 3 step 3: a packet that a
 * detector records becomes an event of the virtual detector electronics,
 * with pixel identifier, time of flight and probability). */
typedef struct {
  uint32_t pixel;  /* bin / n_tof: tube * n_pix + pixel (tubes), ring (sphere) */
  float tof;       /* s, since the incident packet crossed z = 0 */
  float value;     /* recorded value (the packet's probability times the
                      absorption probability for tubes) */
  int32_t order;   /* number of scattering events of the packet */
} mcv_event;

/* Same transport as mcv_run, also appending one event per recorded packet
 * (bin >= 0) to events (device array of `capacity`) in arbitrary order.
 * *n_events_dev (device uint64) is advanced by the number of events: zeroed
 * by the caller, it receives the count, which may exceed capacity (then only
 * `capacity` events are written; the caller sees the overflow); not zeroed,
 * successive calls append.  hist and hist_w2 may be NULL (events only).
 * Errors as mcv_run; MCV_EINVAL for a null event buffer or counter. */
mcv_status mcv_run_events(mcv_plan p, const mcv_beam* beam, uint64_t seed, uint64_t first,
                          uint64_t n, double* hist, double* hist_w2, mcv_event* events,
                          uint64_t capacity, uint64_t* n_events_dev, void* stream);

/* ------------------------------------------------------------ reduction */
/* Powder reduction to I(Q, E) (Sec. 3, "Reduction": intensities are sums of
 * packet probabilities and are reduced exactly like measured counts).
 * Direct geometry with the scattering at the sample position: for a pixel
 * centre r_p (tubes: on the tube axis at the pixel's mid height; sphere:
 * ring centre (ring + 1/2) pi / n_2theta at radius R) and a time t (bin
 * centre tof_lo + (b + 1/2) dt, or the event's time): v_f = |r_p| / t,
 * E = Ei - m v_f^2 / 2, Q = |k_i - k_f| with k_i along +z of magnitude
 * sqrt(Ei / (hbar^2/2m)) and k_f along r_p.  Bins: iq = floor((Q - q_lo)
 * nq / (q_hi - q_lo)), ie likewise in E; entries outside the grid are
 * dropped.  Q and E are evaluated in binary32, the sums in binary64. */
typedef struct {
  double Ei;          /* meV: incident energy assumed by the reduction */
  double q_lo, q_hi;  /* 1/A */
  double e_lo, e_hi;  /* meV: energy transfer Ei - Ef */
  int32_t nq, ne;     /* >= 1 each */
} mcv_qe_grid;

/* Adds the histogram hist[mcv_plan_nbins(p)] (device binary64, laid out as
 * the plan's detector bins, 16-byte aligned) into iqe[nq * ne] (device
 * binary64, row-major in Q, zeroed by the caller), and, if both are given,
 * hist_w2 into iqe_w2.  Errors: MCV_EINVAL (null arguments, bad grid,
 * Ei <= 0, misaligned histogram), MCV_EHIP. */
mcv_status mcv_reduce_qe(mcv_plan p, const mcv_qe_grid* grid, const double* hist,
                         const double* hist_w2, double* iqe, double* iqe_w2, void* stream);

/* Adds events[0 .. min(*n_events_dev, capacity)) (device, as written by
 * mcv_run_events with this plan's detector) into iqe[nq * ne], and their
 * squared values into iqe_w2 when it is not NULL.  Events whose pixel is
 * outside the detector are ignored.  Errors as mcv_reduce_qe. */
mcv_status mcv_reduce_events_qe(mcv_plan p, const mcv_qe_grid* grid, const mcv_event* events,
                                const uint64_t* n_events_dev, uint64_t capacity, double* iqe,
                                double* iqe_w2, void* stream);

/* ------------------------------------------------------------- adjoint */
/* Parameters of a gradient (an extension of the paper's method: the
 * derivatives of the Monte Carlo estimate of I with every random choice held
 * fixed):
 *   - the raw values theta_b of the DOS of one one-phonon kernel (the kernel
 *     samples Z = theta / sum(theta de); Supplement S4), with
 *     multiphonon_kernel naming a multi-phonon kernel of the same scatterer
 *     that reads the same DOS (equal values, emax, M and T: its A_1 and S_n
 *     then follow theta as well), or -1;
 *   - the cells S_c of the grid of one tabulated S(Q,E) kernel (Sec. 2.4.2,
 *     the S(Q,omega) histogram kernel; the grid is the kernel's weight, its
 *     proposal does not depend on it);
 *   - sigma_abs of one scatterer and the nominal sigma of one non-powder
 *     kernel.
 * -1 in a *_scatterer field leaves that parameter group out.
 * Gradient layout: [theta_0 .. theta_{nb-1}, S_0 .. S_{nc-1}, sigma_abs,
 * sigma], nb = DOS bins (0 without DOS), nc = nQ nE cells (0 without a grid);
 * entries of parameters left out stay 0.  A table entry of value 0 gets
 * gradient 0 (the frozen proposal never draws a zero DOS bin; a packet that
 * reads a zero S(Q,E) cell has weight 0 and is not traced). */
typedef struct {
  int32_t dos_scatterer, dos_kernel;
  int32_t abs_scatterer;
  int32_t sigma_scatterer, sigma_kernel;
  int32_t sqe_scatterer, sqe_kernel;
  int32_t multiphonon_kernel;
} mcv_param_map;

/* number of gradient entries (nb + nc + 2), or -1 for an invalid map */
int64_t mcv_adjoint_nparams(mcv_plan p, const mcv_param_map* pm);

/* Re-traces histories first .. first+n-1 with the same random numbers as
 * mcv_run and adds to grad[nparams] (device, binary64, zeroed by the caller)
 * the sum over recorded packets of dL_dI[bin] * value * d log(value)/d theta,
 * where a packet's weight is its path density at theta over the density the
 * path was drawn from at the plan's parameters (at theta = the plan's values
 * this is the derivative of the estimate of sum_b dL_dI[b] I_b).  dL_dI:
 * device binary64 [nbins].  The plan keeps a binary64 workspace (4 + 2 nb +
 * nc values, allocated on first use): concurrent adjoint calls on one plan
 * race.  A packet carries at most 12 table indices, so max_orders times the
 * phonons of one draw (1, or max_phonons of a tied multi-phonon kernel) must
 * not exceed 12.  Errors: MCV_EINVAL, MCV_EUNSUPPORTED, MCV_ENOMEM, MCV_EHIP. */
mcv_status mcv_adjoint(mcv_plan p, const mcv_param_map* pm, const mcv_beam* beam, uint64_t seed,
                       uint64_t first, uint64_t n, const double* dL_dI, double* grad,
                       void* stream);

/* Adjoint tape: the same gradient as mcv_adjoint without re-tracing.  A
 * forward run writes, for every packet it records (bin >= 0), one entry with
 * the bin, the recorded value and the packet's carry for the parameter map
 * (d log w / d sigma_abs, d log w / d sigma, the Debye-Waller sum A, draw
 * counts, table indices: the terms mcv_adjoint gathers at a detection); the
 * backward pass reads the entries instead of tracing the histories again.
 * Layout: MCV_TAPE_FIELDS x capacity uint32 words, field-major ([field]
 * [entry]): 0 bin, 1 value (binary32 bits), 2 d sigma_abs, 3 d sigma, 4 A
 * (binary32 bits), 5 counts (DOS draws low 16 bits, table indices high 16),
 * 6..11 table indices (16 bits each, two per word; an entry with n indices
 * writes only words 6 .. 6 + ceil(n/2) - 1, the others keep what the buffer
 * held).  24 to 48 bytes per recorded packet: 5.3e6 entries for 1e7
 * histories of the powder cylinder seen by tubes (capacity x 48 bytes
 * allocated, 254 MB). */
#define MCV_TAPE_FIELDS 12

/* mcv_run (histogram hist, and Squared weights into hist_w2 when not NULL;
 * either may be NULL) that also appends one tape entry per recorded packet
 * to tape (device, capacity entries per field, 4-byte aligned), in
 * arbitrary order.  *n_tape_dev (device uint64, 8-byte aligned) is advanced
 * by the number of recorded packets: zeroed by the caller it receives their
 * count, which may exceed capacity (entries beyond it are not written and
 * the tape is incomplete).  The map must be the one later given to
 * mcv_adjoint_tape.  Errors as mcv_adjoint; MCV_EINVAL for a null or
 * misaligned tape or counter; MCV_EUNSUPPORTED for 2^32 or more bins. */
mcv_status mcv_run_tape(mcv_plan p, const mcv_param_map* pm, const mcv_beam* beam, uint64_t seed,
                        uint64_t first, uint64_t n, double* hist, double* hist_w2, uint32_t* tape,
                        uint64_t capacity, uint64_t* n_tape_dev, void* stream);

/* Adds to grad[nparams] (device binary64, zeroed by the caller) the
 * gradient that mcv_adjoint computes for the histories of the run that
 * wrote the tape: the sum over its entries of dL_dI[bin] * value *
 * d log(value)/d theta (dL_dI: device binary64 [nbins]).  Reads the count
 * from *n_tape_dev on the device (no host synchronisation); if it exceeds
 * capacity (an incomplete tape) every entry of grad becomes NaN.  Uses the
 * plan's binary64 workspace as mcv_adjoint does (concurrent adjoint calls
 * on one plan race).  Errors: MCV_EINVAL, MCV_EUNSUPPORTED, MCV_ENOMEM,
 * MCV_EHIP. */
mcv_status mcv_adjoint_tape(mcv_plan p, const mcv_param_map* pm, const uint32_t* tape,
                            uint64_t capacity, const uint64_t* n_tape_dev, const double* dL_dI,
                            double* grad, void* stream);

/* mcv_adjoint_tape for the weighted least squares loss L = sum_b w_b (I_b -
 * T_b)^2 of the histogram I that the run writing the tape produced (zeroed
 * before that run) against a target T with weights w (device binary64
 * [nbins] each): dL/dI_b = 2 w_b (I_b - T_b) is formed at each entry's bin,
 * so no dL/dI array is read or written.  Since I_b is the sum of the values v
 * of the entries in bin b, L = sum_b w_b T_b^2 + sum over entries of v w_b
 * (I_b - 2 T_b); the second term is added to *loss (device binary64) and the
 * first, a constant of the target, is the caller's (mcv_loss_grad of a zero
 * histogram against T and w gives it).  When L is much smaller than that
 * constant the two terms cancel: their binary64 sum keeps about 16 +
 * log10(L / constant) digits.  Incomplete tape: grad and *loss become NaN.
 * Errors as mcv_adjoint_tape. */
mcv_status mcv_adjoint_tape_wl2(mcv_plan p, const mcv_param_map* pm, const uint32_t* tape,
                                uint64_t capacity, const uint64_t* n_tape_dev, const double* I,
                                const double* T, const double* w, double* loss, double* grad,
                                void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): mcv_adjoint with
 * its binary64 workspace in static device memory of the library (32768
 * values = 256 KiB per device, held until the process ends) instead of
 * plan-owned memory; no allocation, no host-to-device copy.  Same arguments,
 * kernels and result as mcv_adjoint.  The caller still provides dL_dI and
 * grad.  Every call on one device shares that device's workspace, and each
 * call re-initialises it: calls that overlap on one device (other streams,
 * other threads) race.  Errors as mcv_adjoint, and MCV_ECAPACITY when 4 + 2
 * nb + nc (nb DOS bins, nc S(Q,E) cells of the map) exceeds 32768. */
mcv_status mcv_adjoint_noalloc(mcv_plan p, const mcv_param_map* pm, const mcv_beam* beam,
                               uint64_t seed, uint64_t first, uint64_t n, const double* dL_dI,
                               double* grad, void* stream);

/* Sets n binary64 values of device memory to zero: the histogram that an
 * accumulation of recorded probabilities starts from (Sec. 3, the detector
 * result is the sum of the recorded packets' probabilities; mcv_run adds).
 * A fill kernel, not a memset, so that it may be captured in a HIP graph.
 * p: device, 8-byte aligned (any n >= 0).  Asynchronous on `stream`.
 * Errors: MCV_EINVAL (n < 0, NULL p with n > 0, misaligned p), MCV_EHIP. */
mcv_status mcv_zero(double* p, int64_t n, void* stream);

/* Weighted L2 loss of a histogram against a target (streaming): *loss +=
 * sum_b w_b (I_b - T_b)^2 and dL_dI_b = 2 w_b (I_b - T_b).  Device binary64
 * arrays of n entries, 16-byte aligned; *loss is accumulated into. */
mcv_status mcv_loss_grad(const double* I, const double* T, const double* w, int64_t n,
                         double* dL_dI, double* loss, void* stream);

/* ------------------------------------------------------------- batches */
/* Many independent simulations in one persistent launch (an extension of
 * the paper's method, whose runs are independent MC streams, Sec. 3).  Each
 * item is a plan, a beam, a seed, an id range and its own histogram. */
typedef struct mcv_batch_s* mcv_batch;

typedef struct {
  mcv_plan plan;
  mcv_beam beam;
  uint64_t seed;
  uint64_t first;
  uint64_t n;
  double* hist;  /* device binary64 [mcv_plan_nbins(plan)] */
} mcv_batch_item;

/* block_size: 64..256, multiple of 64 (0: 256); chunk: histories per work
 * item of the queue (0: 4096); wgs_per_cu: cap on resident workgroups per CU
 * (0: as many as fit); zero_hists: 1 = every run zeroes the histograms first
 * (otherwise runs accumulate). */
typedef struct {
  int32_t block_size;
  int32_t chunk;
  int32_t wgs_per_cu;
  int32_t zero_hists;
} mcv_tuning;

/* Builds the work queue (chunks of (item, id range), longest estimated
 * first), uploads it, and captures [histogram zeroing + queue reset +
 * persistent kernel] into a HIP graph.  Items may share one histogram (it is
 * zeroed before the transport and receives the sum of their ranges).  The
 * histograms and plans must stay alive until mcv_batch_destroy.  Errors:
 * MCV_EINVAL, MCV_EUNSUPPORTED, MCV_EHIP. */
mcv_status mcv_batch_create(mcv_batch* out, const mcv_batch_item* items, int32_t n,
                            const mcv_tuning* tuning, int32_t device);
/* Replays the graph on `stream`.  Each item's histogram receives the same
 * values as mcv_run of that item (up to binary64 summation order).  Runs of
 * one batch must not overlap. */
mcv_status mcv_batch_run(mcv_batch b, void* stream);
mcv_status mcv_batch_destroy(mcv_batch b);

/* Times mcv_batch_run for block sizes {64, 128, 192, 256} x chunks {1024,
 * 4096, 16384, 65536} (reps runs each after one warm-up) and returns the
 * fastest tuning and its time per run (ms).  The histograms are
 * overwritten. */
mcv_status mcv_autotune(const mcv_batch_item* items, int32_t n, int32_t device, int32_t reps,
                        mcv_tuning* best, double* best_ms);

/* Waits for the stream and reports a pending device error. */
mcv_status mcv_sync(void* stream);
const char* mcv_last_error(void);
int32_t mcv_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MCV_H */
