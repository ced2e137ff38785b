// mcv_transport.hip -- gfx950 kernels of the weighted neutron-transport path.
//
// Method (arXiv:1504.02776): a source packet is traced through the sample
// assembly; at every material interval on its ray it is split into a
// transmitted part (weight times e^{-mu L}) and a scattered part born at a
// random point of the interval with a randomly chosen kernel (Sec. 2.4.3
// "Multiple Scattering"; Supplement S3, interactM1).  Scattered packets are
// split again up to the maximum order (Supplement S3, scatterM), then every
// packet leaving the assembly is handed to the detector (Sec. 2.4.3,
// "Ray tracing in a detector system") and its value is added to I(pixel, tof)
// (Sec. 3, intensity = sum of packet probabilities).
//
// GPU organisation (MI355X, wave64):
//   * one lane owns one history at a time and walks its packet tree depth
//     first; the first child of a flight stays in registers and the others
//     go to a per-lane stack in LDS whose depth is bounded by
//     (segments per flight - 1) * max order;
//   * each wave owns a contiguous range of history ids; when lanes run out
//     of work they take new histories together (ballot + prefix count), so
//     lanes stay busy until the range is exhausted;
//   * the plan (scatterers, kernels, detector) and its binary32 tables are
//     copied to LDS once per workgroup, so divergent per-lane lookups are
//     LDS reads;
//   * every random number is a word of a Philox4x32-10 block addressed by
//     (seed, id, stream, lineage, block): the traversal order is free;
//   * recorded values go to the binary64 histogram with hardware FP64
//     atomics.
// Nothing here is a dense contraction; the kernel is bound by VALU issue and
// by the histogram atomics.

#include <hip/hip_runtime.h>

#include <vector>

#include "mcv_internal.h"

// resident waves per SIMD the kernels are compiled for (register budget
// 512 / N per lane).  The transport kernels keep their packet stacks in
// device memory, so LDS does not cap their occupancy: 4 waves per SIMD
// (measured on the crystal in its can, 1e8 histories: 4 waves 111 ms, 5
// waves 150 ms, 6 waves 173 ms, with the stacks in LDS and 2 waves 151 ms).
// The persistent batch kernel does the same.
#ifndef MCV_WAVES_PER_EU
#define MCV_WAVES_PER_EU 4
#endif
#ifndef MCV_WAVES_PER_EU_MAX
#define MCV_WAVES_PER_EU_MAX 4
#endif
#ifndef MCV_BATCH_WAVES_PER_EU
#define MCV_BATCH_WAVES_PER_EU 4
#endif

namespace mcv {
namespace dev {

constexpr float kKperV = 1.588253594514238e-3f;  // k [1/A] per m/s
constexpr float kVperK = 629.6223748234908f;      // m/s per 1/A
constexpr float kEperV2 = 5.22703759e-6f;         // meV per (m/s)^2
constexpr float kHb2m = 2.0721249f;               // hbar^2/2m_n, meV A^2
constexpr float kTwoPi = 6.283185307179586f;
constexpr float kInvPi = 0.3183098861837907f;
constexpr float kSurf = 1e-7f;                    // m
constexpr float kBig = 1e30f;

// ------------------------------------------------------------------ RNG
// Philox4x32-10 (Salmon et al., SC'11).
__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 multiply gives both halves (v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    c0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    c1 = (uint32_t)p1;
    c2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c3 = (uint32_t)p0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// 23 bits -> odd multiple of 2^-24 in (0,1), exact in binary32
__device__ __forceinline__ float unif(uint32_t x) {
  return (float)(x >> 9) * 0x1p-23f + 0x1p-24f;
}

__device__ __forceinline__ void draw4(uint64_t id, uint32_t stream, uint32_t lin, uint32_t block,
                                      uint64_t seed, float* u) {
  uint32_t c0 = (uint32_t)id, c1 = (uint32_t)(id >> 32) | (stream << 30), c2 = lin, c3 = block;
  philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  u[0] = unif(c0);
  u[1] = unif(c1);
  u[2] = unif(c2);
  u[3] = unif(c3);
}

// ------------------------------------------------------------------ packets
struct Pk {
  float px, py, pz;
  float dx, dy, dz;  // unit direction
  float sp;          // speed, m/s
  float t, w;
  uint32_t lin;
};

__device__ __forceinline__ int order_of(uint32_t lin) { return (31 - __clz(lin)) / 3; }

// ------------------------------------------------------------------ geometry
// Intervals in "centre +- half" form keep the length of an interval exact
// when both of its ends come from the same surface pair.
struct Iv {
  float lo, hi, len;
  int entry;  // surface the interval is entered through (see snap_entry)
};

// entry-surface codes: 1..3 box face normal to local x, y, z; 4 outer
// cylinder wall; 5 inner (annulus) wall; 6 end cap
enum { ENTRY_NONE = 0, ENTRY_BOX_X = 1, ENTRY_OUTER = 4, ENTRY_INNER = 5, ENTRY_CAP = 6 };

// slab |q + s d| <= h; returns false on a miss.  (c - hw, c + hw)
__device__ __forceinline__ bool slab(float q, float d, float h, float& c, float& hw) {
  if (d == 0.0f) {
    if (fabsf(q) > h) return false;
    c = 0.0f;
    hw = kBig;
    return true;
  }
  c = -q / d;
  hw = h / fabsf(d);
  return true;
}

// infinite cylinder x^2 + z^2 <= r^2; sq = sqrt(r^2 a - cross^2) for annuli
__device__ __forceinline__ bool radial(float qx, float qz, float dx, float dz, float r, float& c,
                                       float& hw, float& sq, float& a_out) {
  const float a = dx * dx + dz * dz;
  a_out = a;
  if (a == 0.0f) {
    if (qx * qx + qz * qz > r * r) return false;
    c = 0.0f;
    hw = kBig;
    sq = 0.0f;
    return true;
  }
  const float cr = qx * dz - qz * dx;
  const float disc = r * r * a - cr * cr;
  if (disc <= 0.0f) return false;
  sq = sqrtf(disc);
  c = -(qx * dx + qz * dz) / a;
  hw = sq / a;
  return true;
}

// finite cylinder (radial x slab in y) from its radial and axial parts;
// lo_rad / hi_rad: the interval starts / ends on the radial surface
__device__ __forceinline__ bool cyl_of(float cr, float hr, float cs, float hs, Iv& iv, int& lo_rad,
                                       int& hi_rad) {
  const float l1 = cr - hr, l2 = cs - hs, h1 = cr + hr, h2 = cs + hs;
  lo_rad = l1 >= l2;
  hi_rad = h1 <= h2;
  iv.lo = lo_rad ? l1 : l2;
  iv.hi = hi_rad ? h1 : h2;
  if (!(iv.hi > iv.lo)) return false;
  if (lo_rad && hi_rad) iv.len = 2.0f * hr;
  else if (!lo_rad && !hi_rad) iv.len = 2.0f * hs;
  else iv.len = iv.hi - iv.lo;
  return true;
}

// finite cylinder (radial x slab in y)
__device__ __forceinline__ bool cyl(float qx, float qy, float qz, float dx, float dy, float dz,
                                    float r, float hh, Iv& iv, float& sq, float& a, int& lo_rad,
                                    int& hi_rad) {
  float cr, hr, cs, hs;
  if (!radial(qx, qz, dx, dz, r, cr, hr, sq, a)) return false;
  if (!slab(qy, dy, hh, cs, hs)) return false;
  return cyl_of(cr, hr, cs, hs, iv, lo_rad, hi_rad);
}

// the shape frame: local = R^T (p - pos); identity rotations (flagged in the
// plan) skip the products, which give the same values
__device__ __forceinline__ void to_local(const DevScat& S, const Pk& P, float& qx, float& qy,
                                         float& qz, float& dx, float& dy, float& dz) {
  const float rx = P.px - S.pos[0], ry = P.py - S.pos[1], rz = P.pz - S.pos[2];
  if (S.ident) {
    qx = rx;
    qy = ry;
    qz = rz;
    dx = P.dx;
    dy = P.dy;
    dz = P.dz;
    return;
  }
  const float* R = S.rot;
  qx = R[0] * rx + R[3] * ry + R[6] * rz;
  qy = R[1] * rx + R[4] * ry + R[7] * rz;
  qz = R[2] * rx + R[5] * ry + R[8] * rz;
  dx = R[0] * P.dx + R[3] * P.dy + R[6] * P.dz;
  dy = R[1] * P.dx + R[4] * P.dy + R[7] * P.dz;
  dz = R[2] * P.dx + R[5] * P.dy + R[8] * P.dz;
}

// intervals of scatterer S along p + s d (lab); returns count (0..2)
__device__ __forceinline__ int shape_iv(const DevScat& S, const Pk& P, Iv& i0, Iv& i1) {
  float qx, qy, qz, dx, dy, dz;
  to_local(S, P, qx, qy, qz, dx, dy, dz);
  if (S.shape == SHAPE_BOX) {
    float c0, h0, c1, h1, c2, h2;
    if (!slab(qx, dx, S.h[0], c0, h0) || !slab(qy, dy, S.h[1], c1, h1) ||
        !slab(qz, dz, S.h[2], c2, h2))
      return 0;
    float lo = c0 - h0, hi = c0 + h0, hl = h0;
    int alo = 0, ahi = 0;
    if (c1 - h1 > lo) { lo = c1 - h1; alo = 1; }
    if (c2 - h2 > lo) { lo = c2 - h2; alo = 2; }
    if (c1 + h1 < hi) { hi = c1 + h1; ahi = 1; hl = h1; }
    if (c2 + h2 < hi) { hi = c2 + h2; ahi = 2; hl = h2; }
    if (!(hi > lo)) return 0;
    i0.lo = lo;
    i0.hi = hi;
    i0.len = (alo == ahi) ? 2.0f * hl : hi - lo;
    i0.entry = ENTRY_BOX_X + alo;
    return 1;
  }
  float sq_o, a, sq_i;
  int lr_o, hr_o, lr_i, hr_i;
  const float r_out = S.shape == SHAPE_CYLINDER ? S.h[0] : S.h[1];
  const float hh = S.shape == SHAPE_CYLINDER ? S.h[1] : S.h[2];
  // radial and axial parts of the outer cylinder; the inner one of an
  // annulus shares the axis, the caps and every term but the radius
  float cr, hr, cs, hs;
  if (!radial(qx, qz, dx, dz, r_out, cr, hr, sq_o, a)) return 0;
  if (!slab(qy, dy, hh, cs, hs)) return 0;
  Iv o;
  if (!cyl_of(cr, hr, cs, hs, o, lr_o, hr_o)) return 0;
  o.entry = lr_o ? ENTRY_OUTER : ENTRY_CAP;
  if (S.shape == SHAPE_CYLINDER) {
    i0 = o;
    return 1;
  }
  Iv in;
  bool hit_in;
  {
    const float r_in = S.h[0];
    if (a == 0.0f) {
      hit_in = qx * qx + qz * qz <= r_in * r_in;
      sq_i = 0.0f;
      if (hit_in) hit_in = cyl_of(0.0f, kBig, cs, hs, in, lr_i, hr_i);
    } else {
      const float xr = qx * dz - qz * dx;
      const float disc = r_in * r_in * a - xr * xr;
      hit_in = disc > 0.0f;
      sq_i = hit_in ? sqrtf(disc) : 0.0f;
      if (hit_in) hit_in = cyl_of(cr, sq_i / a, cs, hs, in, lr_i, hr_i);
    }
  }
  if (!hit_in || in.hi <= o.lo || in.lo >= o.hi) {
    i0 = o;
    return 1;
  }
  // wall thickness along the ray when both ends are on the two radial surfaces
  const float wall = (a > 0.0f) ? (r_out * r_out - S.h[0] * S.h[0]) / (sq_o + sq_i) : 0.0f;
  int n = 0;
  if (in.lo > o.lo) {
    i0.lo = o.lo;
    i0.hi = in.lo;
    i0.len = (lr_o && lr_i) ? wall : in.lo - o.lo;
    i0.entry = o.entry;
    n = 1;
  }
  if (o.hi > in.hi) {
    Iv& t = n == 0 ? i0 : i1;
    t.lo = in.hi;
    t.hi = o.hi;
    t.len = (hr_o && hr_i) ? wall : o.hi - in.hi;
    t.entry = hr_i ? ENTRY_INNER : ENTRY_CAP;
    ++n;
  }
  return n;
}

// Puts an entry point computed as start + s d exactly onto the surface it
// enters (in the shape frame): a packet that comes from afar would otherwise
// carry the rounding of its long approach (ulp of 0.1 m ~ 7e-9 m) into the
// birth point of its children, which grazing exits amplify.
__device__ __forceinline__ void snap_entry(const DevScat& S, int code, float dx, float dy,
                                           float dz, float& x, float& y, float& z) {
  if (code == ENTRY_NONE) return;
  const float* R = S.rot;
  const float rx = x - S.pos[0], ry = y - S.pos[1], rz = z - S.pos[2];
  float q[3], dl[3];
  if (S.ident) {
    q[0] = rx;
    q[1] = ry;
    q[2] = rz;
    dl[0] = dx;
    dl[1] = dy;
    dl[2] = dz;
  } else {
    q[0] = R[0] * rx + R[3] * ry + R[6] * rz;
    q[1] = R[1] * rx + R[4] * ry + R[7] * rz;
    q[2] = R[2] * rx + R[5] * ry + R[8] * rz;
    dl[0] = R[0] * dx + R[3] * dy + R[6] * dz;
    dl[1] = R[1] * dx + R[4] * dy + R[7] * dz;
    dl[2] = R[2] * dx + R[5] * dy + R[8] * dz;
  }
  if (code >= ENTRY_BOX_X && code <= ENTRY_BOX_X + 2) {
    const int a = code - ENTRY_BOX_X;
#pragma unroll
    for (int i = 0; i < 3; ++i)
      if (i == a) q[i] = dl[i] > 0.0f ? -S.h[i] : S.h[i];
  } else if (code == ENTRY_OUTER || code == ENTRY_INNER) {
    const float r = (code == ENTRY_INNER || S.shape == SHAPE_CYLINDER) ? S.h[0] : S.h[1];
    const float f = r * rsqrtf(q[0] * q[0] + q[2] * q[2]);
    q[0] *= f;
    q[2] *= f;
  } else if (code == ENTRY_CAP) {
    const float hh = S.shape == SHAPE_CYLINDER ? S.h[1] : S.h[2];
    q[1] = dl[1] > 0.0f ? -hh : hh;
  } else {
    return;
  }
  if (S.ident) {
    x = S.pos[0] + q[0];
    y = S.pos[1] + q[1];
    z = S.pos[2] + q[2];
    return;
  }
  x = S.pos[0] + R[0] * q[0] + R[1] * q[1] + R[2] * q[2];
  y = S.pos[1] + R[3] * q[0] + R[4] * q[1] + R[5] * q[2];
  z = S.pos[2] + R[6] * q[0] + R[7] * q[1] + R[8] * q[2];
}

// Orthonormal basis perpendicular to unit n (Duff et al., JCGT 6(1), 2017)
__device__ __forceinline__ void perp_basis(float nx, float ny, float nz, float& e1x, float& e1y,
                                           float& e1z, float& e2x, float& e2y, float& e2z) {
  const float sg = nz >= 0.0f ? 1.0f : -1.0f;
  const float a = -1.0f / (sg + nz);
  const float b = nx * ny * a;
  e1x = 1.0f + sg * nx * nx * a;
  e1y = sg * b;
  e1z = -sg * nx;
  e2x = b;
  e2y = sg + ny * ny * a;
  e2z = -ny;
}

// isotropic direction from two uniforms: cos = 2u - 1, phi = 2 pi u'
__device__ __forceinline__ void iso_dir(float uc, float up, float& x, float& y, float& z) {
  const float c = 2.0f * uc - 1.0f;
  const float s = 2.0f * sqrtf(uc * (1.0f - uc));
  float sn, cs;
  sincospif(2.0f * up, &sn, &cs);
  x = s * cs;
  y = s * sn;
  z = c;
}

// number of reflections with d > lambda/2 in a table sorted by descending d
__device__ __forceinline__ int n_active(const float* d, int n, float half_lambda) {
  int lo = 0, hi = n;  // first index with d <= half_lambda
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (d[mid] > half_lambda) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// first index i with x < a[i] in an ascending table (n if none)
__device__ __forceinline__ int first_above(const float* a, int n, float x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (x < a[mid]) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

struct Mu {
  float k[kMaxKern];
  float scat, total;
};

__device__ __forceinline__ Mu attenuation(const DevScat& S, const float* tab, float sp) {
  Mu m;
  m.scat = 0.0f;
#pragma unroll
  for (int j = 0; j < kMaxKern; ++j) {
    float mu = 0.0f;
    if (j < S.nk) {
      const DevKernel& K = S.k[j];
      if (K.type == K_POWDER) {
        const float lambda = kTwoPi / (sp * kKperV);
        const int na = n_active(tab + K.t_d, K.nrefl, 0.5f * lambda);
        mu = na > 0 ? K.bragg_coef * lambda * lambda * tab[K.t_pref + na - 1] : 0.0f;
      } else {
        mu = K.mu;
      }
    }
    m.k[j] = mu;
    m.scat += mu;
  }
  m.total = m.scat + S.mu_abs2200 / sp;
  return m;
}

// ------------------------------------------------------------------ kernels
// Each returns the outgoing direction and speed and the weight factor
// (true cross section per unit nominal cross section / proposal density).
struct Out {
  float dx, dy, dz, sp, f;
  float dwq2;  // Q^2 of the Debye-Waller factor applied (0 if none)
  int bin;     // DOS bin of a one-phonon draw, grid cell of an S(Q,E) draw (-1 otherwise)
};

// |k_i - k_f|^2 without cancellation: (ki - kf)^2 + ki kf |d_i - d_f|^2
__device__ __forceinline__ float q2_of(float ki, float kf, float dk, const Pk& P, float ox,
                                       float oy, float oz) {
  const float ex = P.dx - ox, ey = P.dy - oy, ez = P.dz - oz;
  return dk * dk + ki * kf * (ex * ex + ey * ey + ez * ez);
}

__device__ __forceinline__ Out k_iso(const DevKernel& K, const DevScat& S, const Pk& P,
                                     const float* u) {
  Out o;
  iso_dir(u[2], u[3], o.dx, o.dy, o.dz);
  o.sp = P.sp;
  o.f = 1.0f;
  o.dwq2 = 0.0f;
  o.bin = -1;
  if (K.dw) {
    const float k = P.sp * kKperV;
    o.dwq2 = q2_of(k, k, 0.0f, P, o.dx, o.dy, o.dz);
    o.f = expf(-S.dw_coef * o.dwq2);
  }
  return o;
}

// Per-kernel forms of the isotropic elastic (above), powder Bragg,
// one-phonon and spin-wave draws: the cost probe prices each kernel alone
// with them; the transport kernels evaluate them through k_shared, which
// computes the same values (the instantiations with the heavy kernels call
// k_iso and k_spinwave themselves).
__device__ __forceinline__ Out k_powder(const DevKernel& K, const DevScat& S, const float* tab,
                                        const Pk& P, const float* u) {
  Out o;
  const float lambda = kTwoPi / (P.sp * kKperV);
  const int na = n_active(tab + K.t_d, K.nrefl, 0.5f * lambda);
  const float* pref = tab + K.t_pref;
  const float target = u[2] * pref[na - 1];
  int i = first_above(pref, na, target);
  if (i > na - 1) i = na - 1;
  const float d = tab[K.t_d + i];
  const float sb = lambda / (2.0f * d);              // sin(theta_B)
  const float cb = sqrtf((1.0f - sb) * (1.0f + sb));  // cos(theta_B)
  const float c2 = (cb - sb) * (cb + sb);             // cos(2 theta_B)
  const float s2 = 2.0f * sb * cb;                    // sin(2 theta_B)
  float e1x, e1y, e1z, e2x, e2y, e2z;
  perp_basis(P.dx, P.dy, P.dz, e1x, e1y, e1z, e2x, e2y, e2z);
  float sn, cs;
  sincospif(2.0f * u[3], &sn, &cs);
  o.dx = c2 * P.dx + s2 * (cs * e1x + sn * e2x);
  o.dy = c2 * P.dy + s2 * (cs * e1y + sn * e2y);
  o.dz = c2 * P.dz + s2 * (cs * e1z + sn * e2z);
  o.sp = P.sp;
  o.f = 1.0f;
  o.dwq2 = 0.0f;
  o.bin = -1;
  if (K.dw) {
    const float q = kTwoPi / d;
    o.dwq2 = q * q;
    o.f = expf(-S.dw_coef * o.dwq2);
  }
  return o;
}

__device__ __forceinline__ Out k_phonon(const DevKernel& K, const DevScat& S, const float* tab,
                                        const Pk& P, const float* u) {
  Out o;
  int b = first_above(tab + K.t_cdf, K.nbins, u[2]);
  if (b > K.nbins - 1) b = K.nbins - 1;
  const float e = ((float)b + u[3]) * K.de;
  const float x = e / K.kT;
  // m = 1 - e^{-x} without cancellation: (n+1)/(2n+1) = 1/(2 - m) and
  // coth(x/2) = (2 - m)/m
  const float m = -expm1f(-x);
  const float p_create = 1.0f / (2.0f - m);
  const bool create = u[4] < p_create;
  const float Ei = kEperV2 * P.sp * P.sp;
  const float Ef = create ? Ei - e : Ei + e;
  iso_dir(u[5], u[6], o.dx, o.dy, o.dz);
  o.bin = b;
  o.dwq2 = 0.0f;
  if (!(Ef > 0.0f)) {
    o.sp = P.sp;
    o.f = 0.0f;
    return o;
  }
  const float ki = P.sp * kKperV;
  const float kf = sqrtf(Ef / kHb2m);
  const float dk = (create ? e : -e) / (kHb2m * (ki + kf));
  const float q2 = q2_of(ki, kf, dk, P, o.dx, o.dy, o.dz);
  const float dw = K.dw ? expf(-S.dw_coef * q2) : 1.0f;
  o.dwq2 = K.dw ? q2 : 0.0f;
  const float coth = (2.0f - m) / m;
  o.sp = kf * kVperK;
  o.f = (kf / ki) * K.h2m * q2 * dw * coth / e;
  return o;
}


// Coherent one-phonon scattering from a powder (Supplement S4).  Averaging
// over crystallite orientations turns every point K of reciprocal space
// (crystal frame) and branch s into a cone of final states with |Q| = |K|
// and E_f = E_i -+ E_s(K); per unit sigma and unit K volume its cross
// section is (1/4pi)(k_f/k_i) e^{-2W} hbar^2 (K.e_s)^2/(2M E_s) {coth -+ 1}/2
// / (2 k_i k_f |K|).  Draw: K uniform in the ball |K| <= Q_max = k_i +
// k_f,max (u2 radial, u3 u4 direction), the modes of the grid point nearest
// to K (grid coordinates K . (n a_j / 2pi) rounded, periodic; a 48-byte
// gather from the table in device memory), branch s = floor(3 u5) taken
// exactly from the integer behind u5, creation with probability
// (n+1)/(2n+1) (u6), azimuth of the cone u7.  Weight = cross section over
// that density.  Modes below 1e-3 meV scatter with weight 0.
__device__ __forceinline__ Out k_cohphonon(const DevKernel& K, const DevScat& S, const Pk& P,
                                           const float* u) {
  Out o;
  o.dx = P.dx;
  o.dy = P.dy;
  o.dz = P.dz;
  o.sp = P.sp;
  o.f = 0.0f;
  o.dwq2 = 0.0f;
  o.bin = -1;
  const float ki = P.sp * kKperV;
  const float Ei = kEperV2 * P.sp * P.sp;
  const float qmax = ki + sqrtf((Ei + K.wmax) / kHb2m);
  const float km = qmax * cbrtf(u[2]);
  float kx, ky, kz;
  iso_dir(u[3], u[4], kx, ky, kz);
  kx *= km;
  ky *= km;
  kz *= km;
  const int n = K.nbins;
  int idx = 0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float g = kx * K.crot[3 * j] + ky * K.crot[3 * j + 1] + kz * K.crot[3 * j + 2];
    int i = (int)floorf(g + 0.5f) % n;
    if (i < 0) i += n;
    idx = idx * n + i;
  }
  typedef float fv4 __attribute__((ext_vector_type(4)));
  const fv4* m = reinterpret_cast<const fv4*>(
      (const float*)(((uint64_t)K.grid_hi << 32) | (uint64_t)K.grid_lo) + 12 * (size_t)idx);
  const fv4 m0 = m[0], m1 = m[1], m2 = m[2];
  // u5 = (j + 1/2) 2^-23 exactly: floor(3 u5) = (6 j + 3) >> 24
  const int s = (6 * (int)(u[5] * 8388608.0f) + 3) >> 24;
  const float Es = s == 0 ? m0.x : (s == 1 ? m0.y : m0.z);
  const float ex = s == 0 ? m0.w : (s == 1 ? m1.z : m2.y);
  const float ey = s == 0 ? m1.x : (s == 1 ? m1.w : m2.z);
  const float ez = s == 0 ? m1.y : (s == 1 ? m2.x : m2.w);
  if (!(Es >= 1e-3f)) return o;
  const float mm = -expm1f(-Es / K.kT);
  const bool create = u[6] < 1.0f / (2.0f - mm);
  const float Ef = create ? Ei - Es : Ei + Es;
  if (!(Ef > 0.0f)) return o;
  const float kf = sqrtf(Ef / kHb2m);
  const float c = (ki * ki + kf * kf - km * km) / (2.0f * ki * kf);
  if (!(fabsf(c) <= 1.0f)) return o;
  const float sn2 = sqrtf(fmaxf(0.0f, (1.0f - c) * (1.0f + c)));
  float e1x, e1y, e1z, e2x, e2y, e2z;
  perp_basis(P.dx, P.dy, P.dz, e1x, e1y, e1z, e2x, e2y, e2z);
  float sn, cs;
  sincospif(2.0f * u[7], &sn, &cs);
  o.dx = c * P.dx + sn2 * (cs * e1x + sn * e2x);
  o.dy = c * P.dy + sn2 * (cs * e1y + sn * e2y);
  o.dz = c * P.dz + sn2 * (cs * e1z + sn * e2z);
  o.sp = kf * kVperK;
  const float ke = kx * ex + ky * ey + kz * ez;
  const float dw = K.dw ? expf(-S.dw_coef * km * km) : 1.0f;
  o.dwq2 = K.dw ? km * km : 0.0f;
  const float coth = (2.0f - mm) / mm;
  o.f = qmax * qmax * qmax * coth * dw * K.h2m * ke * ke / Es / (2.0f * ki * ki * km);
  return o;
}

__device__ __forceinline__ Out k_spinwave(const DevKernel& K, const Pk& P, const float* u) {
  Out o;
  const float Ei = kEperV2 * P.sp * P.sp;
  const float lo = -10.0f * K.gamma;
  const float hi = fminf(K.wmax + 10.0f * K.gamma, 0.99f * Ei);
  iso_dir(u[3], u[4], o.dx, o.dy, o.dz);
  o.sp = P.sp;
  o.dwq2 = 0.0f;
  o.bin = -1;
  if (!(hi > lo)) {
    o.f = 0.0f;
    return o;
  }
  const float E = lo + u[2] * (hi - lo);
  const float ki = P.sp * kKperV;
  const float kf = sqrtf((Ei - E) / kHb2m);
  const float qx = ki * P.dx - kf * o.dx, qy = ki * P.dy - kf * o.dy, qz = ki * P.dz - kf * o.dz;
  const float* C = K.crot;
  const float cx = C[0] * qx + C[1] * qy + C[2] * qz;
  const float cy = C[3] * qx + C[4] * qy + C[5] * qz;
  const float cz = C[6] * qx + C[7] * qy + C[8] * qz;
  const float w = K.j4s * (3.0f - cosf(cx * K.a) - cosf(cy * K.a) - cosf(cz * K.a));
  const float xx = E - w;
  const float lor = K.gamma * kInvPi / (xx * xx + K.gamma * K.gamma);
  o.sp = kf * kVperK;
  o.f = (kf / ki) * lor * (hi - lo);
  return o;
}

// Isotropic elastic, powder Bragg, incoherent one-phonon and spin-wave
// draws (Supplement S4), as the per-kernel functions above compute them:
//   Isotropic elastic: isotropic direction (u2, u3), speed kept; weight the
//   Debye-Waller factor when the scatterer has one.
//   Powder Bragg: a reflection d > lambda/2 chosen in proportion to its
//   cross section (inverse CDF of the cumulative d|F|^2 of the active
//   reflections, u2); the outgoing direction on the Debye-Scherrer cone
//   2 theta_B = 2 asin(lambda / 2d) about the incident one, uniform in
//   azimuth (u3); weight the Debye-Waller factor at Q = 2 pi / d.
//   One-phonon: energy e from the normalised DOS (bin by inverse CDF, u2;
//   uniform in the bin, u3), phonon creation with probability (n+1)/(2n+1)
//   (u4), isotropic direction (u5, u6); weight (k_f/k_i) (hbar^2 Q^2 / 2M)
//   e^{-2W} coth(e / 2kT) / e, zero when E_f <= 0.
//   Spin wave: energy transfer uniform on [-10 Gamma, min(omega_max +
//   10 Gamma, 0.99 E_i)] (u2), isotropic direction (u3, u4); weight (k_f/k_i)
//   times the Lorentzian of half width Gamma about omega(Q) times the range.
// One function evaluates all four so that the steps they share run once for
// the lanes of a wave that draw any of them, not once per kernel type: the
// inverse-CDF search of a table in LDS (Bragg lines or DOS bins), the sincos
// of the azimuth and the direction about its axis (the incident direction
// for a cone, the lab z axis otherwise: c a + s (cos phi e1 + sin phi e2)
// with a = z, e1 = x, e2 = y gives the isotropic direction's components
// exactly), the Debye-Waller exponential.  Measured: powder 1e7 1.45 ->
// 1.36 ms with the first two kernels shared, crystal in its can 1e8 80.3 ->
// 79.1 ms with all four.  ALL = false: powder Bragg and one-phonon only (the
// other two compiled out); the instantiations with the heavy kernels use
// that form (the coherent one-phonon plate took 1.67 instead of 1.50 ms with
// all four).
template <bool ALL>
__device__ __forceinline__ Out k_shared(const DevKernel& K, const DevScat& S, const float* tab,
                                        const Pk& P, const float* u) {
  const bool pw = K.type == K_POWDER;
  const bool ph = K.type == K_PHONON;
  const bool sw = ALL && K.type == K_SPINWAVE;
  Out o;
  o.bin = -1;
  // table search
  int i = 0;
  float lambda = 0.0f;
  if (pw || ph) {
    const float* tbl;
    int n;
    float target;
    if (pw) {
      lambda = kTwoPi / (P.sp * kKperV);
      const int na = n_active(tab + K.t_d, K.nrefl, 0.5f * lambda);
      tbl = tab + K.t_pref;
      n = na;
      target = u[2] * tbl[na - 1];
    } else {
      tbl = tab + K.t_cdf;
      n = K.nbins;
      target = u[2];
    }
    i = first_above(tbl, n, target);
    if (i > n - 1) i = n - 1;
  }
  // polar angle about the axis and azimuth
  float c, s, up;
  float q2 = 0.0f;  // Q^2 of the Debye-Waller factor
  if (pw) {
    const float d = tab[K.t_d + i];
    const float sb = lambda / (2.0f * d);              // sin(theta_B)
    const float cb = sqrtf((1.0f - sb) * (1.0f + sb));  // cos(theta_B)
    c = (cb - sb) * (cb + sb);                          // cos(2 theta_B)
    s = 2.0f * sb * cb;                                 // sin(2 theta_B)
    up = u[3];
    const float q = kTwoPi / d;
    q2 = q * q;
  } else {
    // uniforms by value (a select of array elements would index the array)
    const float u2 = u[2], u3 = u[3], u4 = u[4], u5 = u[5], u6 = u[6];
    const float uc = ph ? u5 : sw ? u3 : u2;
    c = 2.0f * uc - 1.0f;
    s = 2.0f * sqrtf(uc * (1.0f - uc));
    up = ph ? u6 : sw ? u4 : u3;
  }
  float sn, cs;
  sincospif(2.0f * up, &sn, &cs);
  float ax = 0.0f, ay = 0.0f, az = 1.0f;
  float e1x = 1.0f, e1y = 0.0f, e1z = 0.0f, e2x = 0.0f, e2y = 1.0f, e2z = 0.0f;
  if (pw) {
    ax = P.dx;
    ay = P.dy;
    az = P.dz;
    perp_basis(P.dx, P.dy, P.dz, e1x, e1y, e1z, e2x, e2y, e2z);
  }
  o.dx = c * ax + s * (cs * e1x + sn * e2x);
  o.dy = c * ay + s * (cs * e1y + sn * e2y);
  o.dz = c * az + s * (cs * e1z + sn * e2z);
  o.sp = P.sp;
  float pre = 1.0f;  // phonon weight before the Debye-Waller factor
  float m = 0.0f, e = 0.0f;
  float fsw = 0.0f;  // spin-wave weight
  bool ok = true;    // false: no Debye-Waller factor (a phonon with E_f <= 0)
  if (ph) {
    e = ((float)i + u[3]) * K.de;
    const float x = e / K.kT;
    // m = 1 - e^{-x} without cancellation: (n+1)/(2n+1) = 1/(2 - m) and
    // coth(x/2) = (2 - m)/m
    m = -expm1f(-x);
    const float p_create = 1.0f / (2.0f - m);
    const bool create = u[4] < p_create;
    const float Ei = kEperV2 * P.sp * P.sp;
    const float Ef = create ? Ei - e : Ei + e;
    o.bin = i;
    if (!(Ef > 0.0f)) {
      ok = false;
    } else {
      const float ki = P.sp * kKperV;
      const float kf = sqrtf(Ef / kHb2m);
      const float dk = (create ? e : -e) / (kHb2m * (ki + kf));
      q2 = q2_of(ki, kf, dk, P, o.dx, o.dy, o.dz);
      o.sp = kf * kVperK;
      pre = (kf / ki) * K.h2m * q2;
    }
  } else if (sw) {
    const float Ei = kEperV2 * P.sp * P.sp;
    const float lo = -10.0f * K.gamma;
    const float hi = fminf(K.wmax + 10.0f * K.gamma, 0.99f * Ei);
    if (hi > lo) {
      const float E = lo + u[2] * (hi - lo);
      const float ki = P.sp * kKperV;
      const float kf = sqrtf((Ei - E) / kHb2m);
      const float qx = ki * P.dx - kf * o.dx, qy = ki * P.dy - kf * o.dy,
                  qz = ki * P.dz - kf * o.dz;
      const float* C = K.crot;
      const float cx = C[0] * qx + C[1] * qy + C[2] * qz;
      const float cy = C[3] * qx + C[4] * qy + C[5] * qz;
      const float cz = C[6] * qx + C[7] * qy + C[8] * qz;
      const float w = K.j4s * (3.0f - cosf(cx * K.a) - cosf(cy * K.a) - cosf(cz * K.a));
      const float xx = E - w;
      const float lor = K.gamma * kInvPi / (xx * xx + K.gamma * K.gamma);
      o.sp = kf * kVperK;
      fsw = (kf / ki) * lor * (hi - lo);
    }
  } else if (ALL && !pw && K.dw) {
    const float k = P.sp * kKperV;
    q2 = q2_of(k, k, 0.0f, P, o.dx, o.dy, o.dz);
  }
  const bool dwf = K.dw && ok && !sw;
  const float dw = dwf ? expf(-S.dw_coef * q2) : 1.0f;
  o.dwq2 = dwf ? q2 : 0.0f;
  if (sw) {
    o.f = fsw;
  } else if (ph) {
    const float coth = (2.0f - m) / m;
    o.f = ok ? pre * dw * coth / e : 0.0f;
  } else {
    o.f = dw;
  }
  return o;
}

// Dispersion surface with an exact delta function (Supplement S4, E_vQ
// kernel, S(Q) = 1): for the isotropic outgoing direction d, the outgoing
// wave numbers are the roots of g(k) = E_i - c k^2 - omega(k_i - k d) on
// [0, k_i].  They are bracketed by the sign changes of g (g > 0 against
// g <= 0) at kDispCells + 1 equally spaced k, one is picked (u2) and refined
// to the root in its cell, and the weight n (k_f/k_i) / |dG/dE_f| with
// dG/dE_f = -1 + (grad omega . d) / (2 c k_f) carries the delta function.
// The scan steps
// the cosines of the phases Q_a a, linear in k, with Reinsch's form of the
// cosine recurrence (c_{m+1} = c_m + e_m, e_{m+1} = e_m + lambda c_{m+1},
// lambda = -4 sin^2(theta/2) for a step theta; stable for small theta),
// restarted from sincos every 32 cells, and evaluates g at cell j as
// j4s (cos_x + cos_y + cos_z) - (c h^2 j^2 + 3 j4s - E_i), exact in j^2;
// the cells with a sign change are kept as a bit mask.
constexpr int kDispCells = 256;

__device__ __forceinline__ float disp_g(float Ei, float k, float q0x, float q0y, float q0z,
                                        float dcx, float dcy, float dcz, float a, float j4s) {
  return Ei - kHb2m * k * k -
         j4s * (3.0f - cosf((q0x - k * dcx) * a) - cosf((q0y - k * dcy) * a) -
                cosf((q0z - k * dcz) * a));
}

// one step theta of the phase: lambda = 2 (cos theta - 1) and sin theta
__device__ __forceinline__ void reinsch_step(float theta, float& lam, float& st) {
  float s, c;
  sincosf(0.5f * theta, &s, &c);
  lam = -4.0f * s * s;
  st = 2.0f * s * c;
}

__device__ __forceinline__ Out k_dispersion(const DevKernel& K, const Pk& P, const float* u) {
  Out o;
  o.bin = -1;
  o.dwq2 = 0.0f;
  o.f = 0.0f;
  o.sp = P.sp;
  iso_dir(u[3], u[4], o.dx, o.dy, o.dz);
  const float Ei = kEperV2 * P.sp * P.sp;
  const float ki = P.sp * kKperV;
  const float* C = K.crot;
  const float q0x = ki * (C[0] * P.dx + C[1] * P.dy + C[2] * P.dz);
  const float q0y = ki * (C[3] * P.dx + C[4] * P.dy + C[5] * P.dz);
  const float q0z = ki * (C[6] * P.dx + C[7] * P.dy + C[8] * P.dz);
  const float dcx = C[0] * o.dx + C[1] * o.dy + C[2] * o.dz;
  const float dcy = C[3] * o.dx + C[4] * o.dy + C[5] * o.dz;
  const float dcz = C[6] * o.dx + C[7] * o.dy + C[8] * o.dz;
  const float a = K.a, j4s = K.j4s;
  const float h = ki * (1.0f / (float)kDispCells);
  float lx, ly, lz, tx, ty, tz;  // per cell: lambda and sin(theta) of each phase
  reinsch_step(-h * dcx * a, lx, tx);
  reinsch_step(-h * dcy * a, ly, ty);
  reinsch_step(-h * dcz * a, lz, tz);
  const float ch2 = kHb2m * h * h, r0 = 3.0f * j4s - Ei;
  uint32_t mask[kDispCells / 32];
  bool prev = false;
  int n = 0;
#pragma unroll
  for (int w = 0; w < kDispCells / 32; ++w) {
    const float k0 = (float)(32 * w) * h;
    float sx, cx, sy, cy, sz, cz;
    sincosf((q0x - k0 * dcx) * a, &sx, &cx);
    sincosf((q0y - k0 * dcy) * a, &sy, &cy);
    sincosf((q0z - k0 * dcz) * a, &sz, &cz);
    if (w == 0) prev = fmaf(j4s, cx + cy + cz, -r0) > 0.0f;
    // e = cos(phase + theta) - cos(phase)
    float ex = fmaf(0.5f * lx, cx, -sx * tx);
    float ey = fmaf(0.5f * ly, cy, -sy * ty);
    float ez = fmaf(0.5f * lz, cz, -sz * tz);
    uint32_t bits = 0u;
#pragma unroll 4
    for (int j = 0; j < 32; ++j) {
      cx += ex;
      ex = fmaf(lx, cx, ex);
      cy += ey;
      ey = fmaf(ly, cy, ey);
      cz += ez;
      ez = fmaf(lz, cz, ez);
      const float jf = (float)(32 * w + j + 1);
      const bool pos = fmaf(j4s, cx + cy + cz, -fmaf(ch2, jf * jf, r0)) > 0.0f;
      bits |= (uint32_t)(pos != prev) << j;
      prev = pos;
    }
    mask[w] = bits;
    n += __popc(bits);
  }
  if (n == 0) return o;
  int pick = (int)floorf(u[2] * (float)n);
  pick = pick > n - 1 ? n - 1 : pick;
  int cell = 0;
#pragma unroll
  for (int w = 0; w < kDispCells / 32; ++w) {
    const int c = __popc(mask[w]);
    if (pick >= 0 && pick < c) {
      uint32_t b = mask[w];
      for (int q = 0; q < pick; ++q) b &= b - 1u;
      cell = 32 * w + __ffs(b) - 1;
    }
    pick -= c;
  }
  // refinement: bisection down to h/256 (one root left in the bracket
  // unless g is tangent there), then two Newton steps from its midpoint
  // (a step longer than the bracket, as at a tangency, is not taken)
  float lo = (float)cell * h, hi = (float)(cell + 1) * h;
  const bool slo = disp_g(Ei, lo, q0x, q0y, q0z, dcx, dcy, dcz, a, j4s) > 0.0f;
  for (int it = 0; it < 8; ++it) {
    const float mid = 0.5f * (lo + hi);
    if ((disp_g(Ei, mid, q0x, q0y, q0z, dcx, dcy, dcz, a, j4s) > 0.0f) == slo) lo = mid;
    else hi = mid;
  }
  float kf = 0.5f * (lo + hi);
  const float wb = hi - lo;
  for (int it = 0; it < 2; ++it) {
    float sx, cx, sy, cy, sz, cz;
    sincosf((q0x - kf * dcx) * a, &sx, &cx);
    sincosf((q0y - kf * dcy) * a, &sy, &cy);
    sincosf((q0z - kf * dcz) * a, &sz, &cz);
    const float g = Ei - kHb2m * kf * kf - j4s * (3.0f - cx - cy - cz);
    const float dg = j4s * a * (sx * dcx + sy * dcy + sz * dcz) - 2.0f * kHb2m * kf;
    const float step = g / dg;
    if (fabsf(step) <= wb) kf -= step;
  }
  if (!(kf > 0.0f)) return o;
  const float ga = j4s * a;
  const float A = ga * (sinf((q0x - kf * dcx) * a) * dcx + sinf((q0y - kf * dcy) * a) * dcy +
                        sinf((q0z - kf * dcz) * a) * dcz) / (2.0f * kHb2m * kf);
  const float J = A - 1.0f;
  if (J == 0.0f) return o;
  o.sp = kf * kVperK;
  o.f = (float)n * (kf / ki) / fabsf(J);
  return o;
}

__device__ __forceinline__ Out k_sqe(const DevKernel& K, const float* tab, const Pk& P,
                                     const float* u) {
  Out o;
  const float Ei = kEperV2 * P.sp * P.sp;
  const float E = K.Emin + u[2] * (K.Emax - K.Emin);
  const float Ef = Ei - E;
  iso_dir(u[3], u[4], o.dx, o.dy, o.dz);
  o.sp = P.sp;
  o.dwq2 = 0.0f;
  o.bin = -1;
  if (!(Ef > 0.0f)) {
    o.f = 0.0f;
    return o;
  }
  const float ki = P.sp * kKperV;
  const float kf = sqrtf(Ef / kHb2m);
  const float dk = E / (kHb2m * (ki + kf));
  const float q = sqrtf(q2_of(ki, kf, dk, P, o.dx, o.dy, o.dz));
  const int iq = (int)floorf(q * K.q_scale);
  int ie = (int)floorf((E - K.Emin) * K.e_scale);
  ie = ie < 0 ? 0 : (ie > K.nE - 1 ? K.nE - 1 : ie);
  o.sp = kf * kVperK;
  o.bin = iq < K.nQ ? iq * K.nE + ie : -1;  // the grid cell read (adjoint)
  o.f = iq < K.nQ ? (kf / ki) * tab[K.t_s + iq * K.nE + ie] * (K.Emax - K.Emin) : 0.0f;
  return o;
}

// Incoherent multi-phonon scattering (incoherent approximation, Supplement
// S4): order n uniform on 2..N, direction isotropic, energy loss the sum of
// n independent draws from the one-phonon spectrum A_1 (so that it follows
// the n-fold convolution A_n exactly), weight (k_f/k_i) S_n(Q) (N - 1) with
// S_n = (2W)^n/n! e^{-2W}.  Phonon i uses words 2(i mod 2) and 2(i mod 2)+1
// of block 2 + i/2 of the packet's scattering stream.  The loss is summed
// as whole bins (exact) plus the in-bin fractions, then scaled once.
__device__ __forceinline__ Out k_multiphonon(const DevKernel& K, const float* tab, const Pk& P,
                                             const float* u, uint64_t id, uint32_t lin,
                                             uint64_t seed) {
  Out o;
  o.bin = -1;
  o.dwq2 = 0.0f;
  const int N = K.nmax;
  int n = 2 + (int)floorf(u[2] * (float)(N - 1));
  n = n > N ? N : n;
  iso_dir(u[3], u[4], o.dx, o.dy, o.dz);
  const int nb2 = 2 * K.nbins;
  int whole = 0;
  float frac = 0.0f;
  float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int i = 0; i < n; ++i) {
    if ((i & 1) == 0) draw4(id, STREAM_SCATTER, lin, 2u + (uint32_t)(i >> 1), seed, v);
    const float ub = (i & 1) ? v[2] : v[0];
    const float up = (i & 1) ? v[3] : v[1];
    int j = first_above(tab + K.t_cdf, nb2, ub);
    j = j > nb2 - 1 ? nb2 - 1 : j;
    whole += j - K.nbins;
    frac += up;
  }
  const float e = ((float)whole + frac) * K.de;
  const float Ei = kEperV2 * P.sp * P.sp;
  const float Ef = Ei - e;
  o.sp = P.sp;
  if (!(Ef > 0.0f)) {
    o.f = 0.0f;
    return o;
  }
  const float ki = P.sp * kKperV;
  const float kf = sqrtf(Ef / kHb2m);
  const float dk = e / (kHb2m * (ki + kf));  // k_i - k_f
  const float q2 = q2_of(ki, kf, dk, P, o.dx, o.dy, o.dz);
  const float w2 = K.dw_self * q2;
  float sn = expf(-w2);
  for (int m = 1; m <= n; ++m) sn *= w2 / (float)m;
  o.dwq2 = q2;  // Q^2 of 2W in S_n (adjoint of a tied DOS)
  o.sp = kf * kVperK;
  o.f = (kf / ki) * sn * (float)(N - 1);
  return o;
}

// ------------------------------------------------------------------ detectors
struct Hit {
  int64_t bin;
  float value, tof;
  int tube, pixel;
};

__device__ __forceinline__ int tof_bin(const DevDet& D, float tof) {
  const float ft = (tof - D.tof_lo) * D.inv_dt;
  if (!(ft >= 0.0f)) return -1;
  const int it = (int)floorf(ft);
  return it < D.ntof ? it : -1;
}

__device__ __forceinline__ Hit detect_sphere(const DevDet& D, const Pk& P) {
  Hit h;
  h.bin = -1;
  h.value = 0.0f;
  h.tof = 0.0f;
  h.tube = -1;
  h.pixel = -1;
  const float b = P.px * P.dx + P.py * P.dy + P.pz * P.dz;
  const float r2 = P.px * P.px + P.py * P.py + P.pz * P.pz;
  const float c = r2 - D.R * D.R;
  if (c >= 0.0f) return h;
  const float s = -b + sqrtf(b * b - c);
  const float cz = fminf(1.0f, fmaxf(-1.0f, (P.pz + s * P.dz) / D.R));
  int ring = (int)floorf(acosf(cz) * D.ring_scale);
  ring = ring > D.n2t - 1 ? D.n2t - 1 : (ring < 0 ? 0 : ring);
  h.tof = P.t + s / P.sp;
  const int it = tof_bin(D, h.tof);
  if (it < 0) return h;
  h.bin = (int64_t)ring * D.ntof + it;
  h.value = P.w;
  return h;
}

// First tube on the ray among the few whose axis can come within a radius
// of it: the columns around the azimuth where the ray crosses radius R, in
// the rows its height range overlaps.  Exact cylinder tests decide.
// The first steps of the tube test: the rows (bit mask) whose height range
// the ray meets at radius R and the column at its azimuth there.  False if
// the ray can meet no tube; detect_tubes takes these steps first, so a
// packet for which this is false is one detect_tubes records no hit for.
__device__ __forceinline__ bool tube_column(const DevDet& D, const Pk& P, float& a, uint32_t& rows,
                                            int& col) {
  a = P.dx * P.dx + P.dz * P.dz;
  if (a == 0.0f) return false;
  const float bq = P.px * P.dx + P.pz * P.dz;
  const float cq = P.px * P.px + P.pz * P.pz - D.R * D.R;
  const float sR = (-bq + sqrtf(bq * bq - a * cq)) / a;
  const float xR = P.px + sR * P.dx, zR = P.pz + sR * P.dz, yR = P.py + sR * P.dy;
  const float ra = sqrtf(a);
  const float dyr = 1.25f * D.radius * fabsf(P.dy) / ra + 1e-4f;
  // rows whose height range the ray can meet (most rays that miss the
  // detector pass above or below every row: they leave here, before the
  // azimuth); the row index is data, so lanes in different rows share one
  // pass of the candidate tests
  rows = 0u;
  for (int r = 0; r < D.nrows; ++r) {
    const float yc = D.row_y[r];
    if (!(yR + dyr < yc - D.half_len || yR - dyr > yc + D.half_len)) rows |= 1u << r;
  }
  if (rows == 0u) return false;
  // fractional column at the azimuth where the ray crosses radius R; with
  // packs, a ray in the gap after a pack counts as its last column (the
  // neighbours tested in detect_tubes include the next pack's first tube)
  const float ax = atan2f(xR, zR) - D.phi_lo;
  float fc = ax * D.inv_dphi;
  if (D.tpp > 0) {
    const float pk = floorf(ax * D.inv_pack_pitch);
    const float within = (ax - pk * D.pack_pitch) * D.inv_tube_pitch;
    fc = pk * (float)D.tpp + fminf(within, (float)D.tpp - 0.5f);
  }
  if (!(fc > -2.0f && fc < (float)D.ncols + 1.0f)) return false;
  col = (int)floorf(fc);
  return true;
}

__device__ __forceinline__ Hit detect_tubes(const DevDet& D, const float* tab, const Pk& P,
                                            uint64_t id, uint64_t seed) {
  Hit h;
  h.bin = -1;
  h.value = 0.0f;
  h.tof = 0.0f;
  h.tube = -1;
  h.pixel = -1;
  float a;
  uint32_t rows;
  int col;
  if (!tube_column(D, P, a, rows, col)) return h;
  float best = kBig, best_hi = 0.0f, best_len = 0.0f;
  int best_tube = -1, best_row = 0;
  while (rows != 0u) {
    const int r = __ffs(rows) - 1;
    rows &= rows - 1u;
    const float yc = D.row_y[r];
#pragma unroll
    for (int dc = -1; dc <= 1; ++dc) {
      const int cc = col + dc;
      if (cc < 0 || cc >= D.ncols) continue;
      const float qx = P.px - tab[D.t_cols + 2 * cc];
      const float qz = P.pz - tab[D.t_cols + 2 * cc + 1];
      const float qy = P.py - yc;
      Iv iv;
      float sq, aa;
      int lr, hr;
      if (!cyl(qx, qy, qz, P.dx, P.dy, P.dz, D.radius, D.half_len, iv, sq, aa, lr, hr)) continue;
      if (!(iv.hi > 0.0f)) continue;
      float lo = iv.lo, len = iv.len;
      if (lo < 0.0f) {
        lo = 0.0f;
        len = iv.hi;
      }
      if (lo < best) {
        best = lo;
        best_hi = iv.hi;
        best_len = len;
        best_tube = r * D.ncols + cc;
        best_row = r;
      }
    }
  }
  if (best_tube < 0) return h;
  (void)best_hi;
  const float mu = D.mu_he2200 / P.sp;
  const float pabs = -expm1f(-mu * best_len);
  float u[4];
  draw4(id, STREAM_DETECT, P.lin, 0u, seed, u);
  const float s_a = best - log1pf(-u[0] * pabs) / mu;
  const float y_a = P.py + s_a * P.dy;
  int pix = (int)floorf((y_a - (D.row_y[best_row] - D.half_len)) * D.pix_scale);
  pix = pix < 0 ? 0 : (pix > D.npix - 1 ? D.npix - 1 : pix);
  h.tof = P.t + s_a / P.sp;
  h.tube = best_tube;
  h.pixel = pix;
  const int it = tof_bin(D, h.tof);
  if (it < 0) return h;
  h.bin = ((int64_t)best_tube * D.npix + pix) * D.ntof + it;
  h.value = P.w * pabs;
  return h;
}

// ------------------------------------------------------------------ source
__device__ __forceinline__ Pk source(const DevBeam& B, uint64_t id, uint64_t seed) {
  if (B.type == 3) {
    // a neutron saved at the sample position: entry id of the rows
    const uint64_t n = B.n_saved;
    const float* r = B.saved;
    Pk P;
    P.px = r[id];
    P.py = r[n + id];
    P.pz = r[2 * n + id];
    const float vx = r[3 * n + id], vy = r[4 * n + id], vz = r[5 * n + id];
    P.t = r[6 * n + id];
    P.w = r[7 * n + id];
    const float sp = sqrtf(vx * vx + vy * vy + vz * vz);
    P.lin = 1u;
    if (!(sp > 0.0f) || !(sp < 3.0e38f) || !(P.w > 0.0f) || !(P.w < 3.0e38f) ||
        !(fabsf(P.t) < 3.0e38f)) {
      P.dx = 0.0f;
      P.dy = 0.0f;
      P.dz = 1.0f;
      P.sp = 1.0f;
      P.w = 0.0f;
      return P;
    }
    P.dx = vx / sp;
    P.dy = vy / sp;
    P.dz = vz / sp;
    P.sp = sp;
    return P;
  }
  float u[4];
  draw4(id, STREAM_SOURCE, 1u, 0u, seed, u);
  Pk P;
  P.px = (u[0] - 0.5f) * B.W;
  P.py = (u[1] - 0.5f) * B.H;
  P.pz = B.z0;
  float E = B.E;
  if (B.type == 2) {
    uint32_t blk = 0;
    for (;;) {
      E = B.E * (1.0f + B.sigma_rel * sqrtf(-2.0f * logf(u[2])) * cospif(2.0f * u[3]));
      if (E > 0.0f || blk >= 63u) break;
      draw4(id, STREAM_SOURCE, 1u, ++blk, seed, u);
    }
  }
  P.dx = 0.0f;
  P.dy = 0.0f;
  P.dz = 1.0f;
  P.sp = E > 0.0f ? sqrtf(E / kEperV2) : 1.0f;
  P.t = B.z0 / P.sp;
  P.w = E > 0.0f ? 1.0f : 0.0f;
  P.lin = 1u;
  return P;
}

// ------------------------------------------------------------------ stack
// Adjoint carry of a packet: d log(w)/d sigma_abs, d log(w)/d sigma, the sum
// A of Q^2 over its Debye-Waller events and tied multi-phonon draws (the
// constant is applied at the end), the number of DOS draws (low 16 bits of
// cnt) and of carried table indices (high 16 bits), and the indices into
// the table parameter vector [DOS | S(Q,E) cells] of the entries its
// ancestry drew (16 bits each, kAdjMaxSparse at most).
struct Adj {
  float dabs, dsig, A;
  uint32_t cnt;
  uint32_t s[kAdjMaxSparse / 2];
};
static_assert(sizeof(Adj) == 4 * kAdjFields, "adjoint carry words");

__device__ __forceinline__ Adj adj_zero() {
  Adj a;
  a.dabs = a.dsig = a.A = 0.0f;
  a.cnt = 0u;
#pragma unroll
  for (int w = 0; w < kAdjMaxSparse / 2; ++w) a.s[w] = 0u;
  return a;
}

// appends a table index (static register indexing; the host bounds the
// count per packet by kAdjMaxSparse)
__device__ __forceinline__ void adj_push(Adj& a, uint32_t idx) {
  const uint32_t n = a.cnt >> 16;
  if (n >= (uint32_t)kAdjMaxSparse) return;
  const uint32_t sh = 16u * (n & 1u);
#pragma unroll
  for (int w = 0; w < kAdjMaxSparse / 2; ++w)
    if ((n >> 1) == (uint32_t)w) a.s[w] |= idx << sh;
  a.cnt += 1u << 16;
}

// The code a pending child carries: -1 none; 4 s + k: kernel k of
// scatterer s still to be evaluated; kUnbuilt | s << 2 | e << 5: a
// forced-collision child of scatterer s not built yet (free path, birth
// point, time, weight and kernel are drawn when it is taken up; its packet
// fields then hold the parent's ray: the flight's start point and time, the
// parent's weight at the interval, and e is the surface the interval is
// entered through).
constexpr int kUnbuilt = 16;

// Gathering of exact-delta dispersion draws in the walk loop: a wave
// evaluates them once at least kDispMin lanes hold one, and no draw waits
// more than kDispWaitMax iterations.
constexpr int kDispMin = 32;
constexpr int kDispWaitMax = 4;

// A stacked packet, one contiguous entry per lane and slot (stack_words
// binary32 words, moved with 16-byte accesses): position, direction, speed,
// time, weight, lineage, its code, then (LAZY: children not built yet) the
// distance to the interval and the interaction probability in it, then the
// adjoint carry in adjoint mode.  A lane's entries follow each other, `cap`
// of them per lane.
static_assert(kFields == 13 && kAdjFields == 10 && kAdjMaxSparse == 12, "stack entry layout");
template <bool ADJ, bool LAZY = false>
__device__ __forceinline__ void push(float* st, int slot, int cap, int tid, const Pk& C,
                                     const Adj& a, int code, float slo = 0.0f,
                                     float pint = 0.0f) {
  constexpr int NW = stack_words(ADJ);
  float4* b = reinterpret_cast<float4*>(st + ((size_t)tid * cap + slot) * NW);
  b[0] = make_float4(C.px, C.py, C.pz, C.dx);
  b[1] = make_float4(C.dy, C.dz, C.sp, C.t);
  b[2] = make_float4(C.w, __uint_as_float(C.lin), __uint_as_float((uint32_t)code), slo);
  if (ADJ) {
    b[3] = make_float4(pint, a.dabs, a.dsig, a.A);
    b[4] = make_float4(__uint_as_float(a.cnt), __uint_as_float(a.s[0]), __uint_as_float(a.s[1]),
                       __uint_as_float(a.s[2]));
    b[5] = make_float4(__uint_as_float(a.s[3]), __uint_as_float(a.s[4]), __uint_as_float(a.s[5]),
                       0.0f);
  } else if (LAZY) {
    b[3] = make_float4(pint, 0.0f, 0.0f, 0.0f);
  }
}

template <bool ADJ, bool LAZY = false>
__device__ __forceinline__ void pop(const float* st, int slot, int cap, int tid, Pk& C, Adj& a,
                                    int& code, float& slo, float& pint) {
  constexpr int NW = stack_words(ADJ);
  const float4* b = reinterpret_cast<const float4*>(st + ((size_t)tid * cap + slot) * NW);
  const float4 v0 = b[0], v1 = b[1], v2 = b[2];
  C.px = v0.x;
  C.py = v0.y;
  C.pz = v0.z;
  C.dx = v0.w;
  C.dy = v1.x;
  C.dz = v1.y;
  C.sp = v1.z;
  C.t = v1.w;
  C.w = v2.x;
  C.lin = __float_as_uint(v2.y);
  code = (int)__float_as_uint(v2.z);
  slo = v2.w;
  if (LAZY || ADJ) {
    const float4 v3 = b[3];
    pint = v3.x;
    if (ADJ) {
      const float4 v4 = b[4], v5 = b[5];
      a.dabs = v3.y;
      a.dsig = v3.z;
      a.A = v3.w;
      a.cnt = __float_as_uint(v4.x);
      a.s[0] = __float_as_uint(v4.y);
      a.s[1] = __float_as_uint(v4.z);
      a.s[2] = __float_as_uint(v4.w);
      a.s[3] = __float_as_uint(v5.x);
      a.s[4] = __float_as_uint(v5.y);
      a.s[5] = __float_as_uint(v5.z);
    }
  }
}

// ------------------------------------------------------------------ flight
// Splits P at every material interval on its ray (children: first in *nxt,
// the others pushed on the lane stack) and moves it to where it leaves.  In
// adjoint mode the carries follow: each crossed length L adds -L dmu/dtheta,
// each birth adds d log(mu_k) - x dmu/dtheta and the kernel's terms.
// Interval slots of a flight: scatterer s owns slot s, or slots 2s and 2s+1
// when the assembly has an annulus (TWO).  NSC = scatterers the code is
// compiled for; the slot arrays then live in registers with static indices.
template <int NSC, bool TWO>
struct Slots {
  static constexpr int N = TWO ? 2 * NSC : NSC;
  static __device__ __forceinline__ constexpr int of(int s, int i) { return TWO ? 2 * s + i : s; }
  static __device__ __forceinline__ constexpr int scat(int j) { return TWO ? j >> 1 : j; }
};

// attenuation coefficients at speed sp, transmission exp(-mu L) and the
// probability 1 - exp(-mu L) to interact within the interval length L
__device__ __forceinline__ void segment_terms(const DevScat& S, const float* tab, float sp,
                                              float L, Mu& mu, float& att, float& pint) {
  mu = attenuation(S, tab, sp);
  const float ml = mu.total * L;
  att = expf(-ml);
  pint = -expm1f(-ml);
}

// (id, lin, seed): the packet's scattering stream, for kernels that draw
// beyond the split's eight uniforms.  HEAVY: also the exact-delta kernel
// and the coherent one-phonon kernel, whose root scan and table gather
// would otherwise raise the register count of every plan (plans without
// them use the instantiations without those cases).
// SEPARATE: the per-kernel powder and one-phonon forms (cost probe).
template <bool HEAVY, bool SEPARATE = false>
__device__ __forceinline__ Out kernel_eval(const DevKernel& K, const DevScat& S,
                                           const float* tab, const Pk& P, const float* u,
                                           uint64_t id, uint32_t lin, uint64_t seed) {
  if constexpr (HEAVY) {
    if (K.type == K_DISPERSION) return k_dispersion(K, P, u);
    if (K.type == K_COH_PHONON) return k_cohphonon(K, S, P, u);
    if (K.type == K_ISO_EL) return k_iso(K, S, P, u);
    if (K.type == K_SPINWAVE) return k_spinwave(K, P, u);
  }
  if constexpr (SEPARATE) {
    if (K.type == K_POWDER) return k_powder(K, S, tab, P, u);
    if (K.type == K_PHONON) return k_phonon(K, S, tab, P, u);
  }
  switch (K.type) {
    case K_ISO_EL:
    case K_POWDER:
    case K_PHONON:
    case K_SPINWAVE: return k_shared<!HEAVY>(K, S, tab, P, u);
    case K_MULTIPHONON: return k_multiphonon(K, tab, P, u, id, lin, seed);
    default: return k_sqe(K, tab, P, u);
  }
}

// The child of a forced collision in one interval: free path x from the
// truncated exponential, birth point on the ray (from the entry point put on
// its surface), time, weight w mu_s/mu (1 - exp(-mu L)), and the kernel k
// chosen with probability mu_k / mu_s (first k with u mu_s below the running
// sum).  Returns k.
__device__ __forceinline__ int split_child(const DevScat& S, const Mu& mu, float pint,
                                           const Pk& P, float sx, float sy, float sz, float t0,
                                           float slo, int code, const float* u, uint32_t lin,
                                           Pk& C, float& x) {
  x = -log1pf(-u[0] * pint) / mu.total;
  float ex = sx + slo * P.dx, ey = sy + slo * P.dy, ez = sz + slo * P.dz;
  snap_entry(S, code, P.dx, P.dy, P.dz, ex, ey, ez);
  C.px = ex + x * P.dx;
  C.py = ey + x * P.dy;
  C.pz = ez + x * P.dz;
  C.t = t0 + (slo + x) / P.sp;
  C.w = P.w * (mu.scat / mu.total) * pint;
  C.lin = lin;
  const float target = u[1] * mu.scat;
  float cum = 0.0f;
  int kk = S.nk - 1;
  bool found = false;
#pragma unroll
  for (int q = 0; q < kMaxKern; ++q) {
    if (q < S.nk && !found) {
      cum += mu.k[q];
      if (target < cum) {
        kk = q;
        found = true;
      }
    }
  }
  return kk;
}

// The material intervals of one packet's ray, walked nearest first; the
// arrays have static indices (registers).  Intervals that end behind the
// packet are dropped; a packet inside a scatterer starts its interval at 0.
template <int NSC, bool TWO>
struct Flight {
  static constexpr int NS = Slots<NSC, TWO>::N;
  float lo[NS], hi[NS], len[NS];
  uint32_t valid, codes;
  float sx, sy, sz, t0, s_end;
  uint32_t g;  // intervals crossed so far (segment index of the next child)
  // attenuation coefficients mu and mu_s of each scatterer at the packet's
  // speed (filled by flight_coefs; used by flight_step with LAZY)
  float mt[NSC], ms[NSC];
};

// The packet's speed is the same over its whole flight: the coefficients
// of every scatterer are computed once, each for all lanes together (the
// same function and operands as segment_terms, so the same values).
template <int NSC, bool TWO>
__device__ __forceinline__ void flight_coefs(const DevPlan& PL, const float* tab, float sp,
                                             Flight<NSC, TWO>& F) {
#pragma unroll
  for (int s = 0; s < NSC; ++s) {
    F.mt[s] = F.ms[s] = 0.0f;
    if (s < PL.nscat) {
      const Mu mu = attenuation(PL.s[s], tab, sp);
      F.mt[s] = mu.total;
      F.ms[s] = mu.scat;
    }
  }
}

template <int NSC, bool TWO>
__device__ __forceinline__ void flight_setup(const DevPlan& PL, const Pk& P, Flight<NSC, TWO>& F) {
  using SL = Slots<NSC, TWO>;
  F.valid = 0u;
  F.codes = 0u;
#pragma unroll
  for (int s = 0; s < NSC; ++s) {
    Iv a, b;
    a.lo = a.hi = a.len = b.lo = b.hi = b.len = 0.0f;
    a.entry = b.entry = ENTRY_NONE;
    const int n = s < PL.nscat ? shape_iv(PL.s[s], P, a, b) : 0;
    const int j0 = SL::of(s, 0);
    F.lo[j0] = a.lo;
    F.hi[j0] = a.hi;
    F.len[j0] = a.len;
    F.codes |= (uint32_t)a.entry << (4 * j0);
    if (n > 0 && a.hi > kSurf) F.valid |= 1u << j0;
    if (TWO) {
      const int j1 = SL::of(s, 1);
      F.lo[j1] = b.lo;
      F.hi[j1] = b.hi;
      F.len[j1] = b.len;
      F.codes |= (uint32_t)b.entry << (4 * j1);
      if (n > 1 && b.hi > kSurf) F.valid |= 1u << j1;
    }
  }
#pragma unroll
  for (int j = 0; j < SL::N; ++j) {
    if (F.lo[j] <= 0.0f) {
      F.lo[j] = 0.0f;
      F.len[j] = F.hi[j];
      F.codes &= ~(0xFu << (4 * j));
    }
  }
  F.sx = P.px;
  F.sy = P.py;
  F.sz = P.pz;
  F.t0 = P.t;
  F.s_end = 0.0f;
  F.g = 0u;
}

// moves the packet to the exit of the last interval it crossed
template <int NSC, bool TWO>
__device__ __forceinline__ void flight_exit(Pk& P, const Flight<NSC, TWO>& F) {
  if (F.g > 0u) {
    P.px = F.sx + F.s_end * P.dx;
    P.py = F.sy + F.s_end * P.dy;
    P.pz = F.sz + F.s_end * P.dz;
    P.t = F.t0 + F.s_end / P.sp;
  }
}

// The adjoint terms of a kernel event: d log(mu_k)/d sigma for the
// differentiated kernel; for the scatterer of the DOS parameters, the Q^2 of
// its Debye-Waller factors and the DOS bin of a one-phonon draw; for a
// multi-phonon kernel tied to that DOS, the Q^2 of S_n and the DOS bins of
// its n phonons (replayed from the same words of blocks 2, 3, ... of the
// packet's scattering stream that k_multiphonon drew), n draws in all; for
// the S(Q,E) kernel of the grid parameters, the cell read.
__device__ __forceinline__ void kernel_carries(const AdjArgs& AA, const DevScat& S,
                                               const DevKernel& K, const float* tab, int si,
                                               int kk, const Out& o, const float* u, uint64_t id,
                                               uint32_t lin, uint64_t seed, Adj& ca) {
  if (si == AA.sig_s && kk == AA.sig_k) ca.dsig += S.n100 / K.mu;
  if (si == AA.dos_s) {
    if (K.type == K_MULTIPHONON) {
      if (kk == AA.mp_k) {
        ca.A += o.dwq2;
        const int N = K.nmax;
        int n = 2 + (int)floorf(u[2] * (float)(N - 1));
        n = n > N ? N : n;
        const int nb2 = 2 * K.nbins;
        float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int i = 0; i < n; ++i) {
          if ((i & 1) == 0) draw4(id, STREAM_SCATTER, lin, 2u + (uint32_t)(i >> 1), seed, v);
          int j = first_above(tab + K.t_cdf, nb2, (i & 1) ? v[2] : v[0]);
          j = j > nb2 - 1 ? nb2 - 1 : j;
          adj_push(ca, (uint32_t)(j >= K.nbins ? j - K.nbins : K.nbins - 1 - j));
        }
        ca.cnt += (uint32_t)n;
      }
    } else {
      ca.A += o.dwq2;
      if (kk == AA.dos_k && o.bin >= 0) {
        adj_push(ca, (uint32_t)o.bin);
        ca.cnt += 1u;
      }
    }
  }
  if (si == AA.sqe_s && kk == AA.sqe_k && o.bin >= 0) adj_push(ca, (uint32_t)(AA.nb + o.bin));
}

// Evaluates the kernel of a child born with DEFER (code = 4 s + k): the same
// uniforms (blocks 0 and 1 of its scattering stream) and the same incoming
// direction and speed as at its birth, so the result is the one an immediate
// evaluation gives.  LAZY: a child not built yet (code with kUnbuilt) is
// first built by split_child from the parent's ray it carries, the
// attenuation coefficients recomputed at its speed, and block 0's
// uniforms, i.e. from the operands flight_step would have used at its birth.
// Builds an unbuilt child (code with kUnbuilt) from the parent's ray it
// carries, with block 0's uniforms u[0], u[1]; returns its kernel index.
__device__ __forceinline__ int build_child(const DevScat& S, const float* tab, Pk& C, int code,
                                           float slo, float pint, const float* u) {
  const Mu mu = attenuation(S, tab, C.sp);
  Pk B;
  float x;
  const int kk = split_child(S, mu, pint, C, C.px, C.py, C.pz, C.t, slo, (code >> 5) & 15, u,
                             C.lin, B, x);
  C.px = B.px;
  C.py = B.py;
  C.pz = B.pz;
  C.t = B.t;
  C.w = B.w;
  return kk;
}

template <bool ADJ, bool HEAVY, bool LAZY = false>
__device__ __forceinline__ void eval_deferred(const DevPlan& PL, const float* tab,
                                              const AdjArgs& AA, Pk& C, Adj& ca, int code,
                                              uint64_t id, uint64_t seed, float slo = 0.0f,
                                              float pint = 0.0f) {
  const int si = (code >> 2) & 3;
  int kk = code & 3;
  const DevScat& S = PL.s[si];
  float u[8];
  draw4(id, STREAM_SCATTER, C.lin, 0u, seed, u);
  draw4(id, STREAM_SCATTER, C.lin, 1u, seed, u + 4);
  if constexpr (LAZY) {
    if (code & kUnbuilt) kk = build_child(S, tab, C, code, slo, pint, u);
  }
  const DevKernel& K = S.k[kk];
  const Out o = kernel_eval<HEAVY>(K, S, tab, C, u, id, C.lin, seed);
  C.dx = o.dx;
  C.dy = o.dy;
  C.dz = o.dz;
  C.sp = o.sp;
  C.w *= o.f;
  if (ADJ) kernel_carries(AA, S, K, tab, si, kk, o, u, id, C.lin, seed, ca);
}

// The nearest remaining interval of a flight: the packet is attenuated by
// e^{-mu L}; with SPLIT (and order < K, w >= min_prob, mu_s > 0) a
// forced-collision child is born in it and its kernel drawn.  The kernel is
// evaluated at once, or, with DEFER, when the child is taken up (its code
// travels with it; `nxt_code`).  With LAZY (which implies DEFER) the child
// itself is built then too: it is kept as the parent's ray, the interval's
// distance and interaction probability (`nxt_slo`, `nxt_pint` for the first
// child), and only its weight is computed here, to drop a child of weight
// zero as the immediate form does.  The first child of a flight is kept in
// `nxt`, further ones go to the stack.
template <bool ADJ, bool SPLIT, bool DEFER, int NSC, bool TWO, bool HEAVY, bool LAZY = false>
__device__ __forceinline__ void flight_step(const DevPlan& PL, const float* tab,
                                            const AdjArgs& AA, Pk& P, Adj& pa,
                                            Flight<NSC, TWO>& F, uint64_t id, uint64_t seed,
                                            Pk& nxt, Adj& na, int& nxt_code, bool& has_nxt,
                                            float* st, int& nst, int nthreads, int tid,
                                            float& nxt_slo, float& nxt_pint) {
  static_assert(!LAZY || (DEFER && !ADJ), "children are built lazily only with deferred kernels");
  using SL = Slots<NSC, TWO>;
  constexpr int NS = SL::N;
  // nearest remaining interval; ties to the lower scatterer index
  int j = 0;
  float best = kBig;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    if ((F.valid >> q) & 1u) {
      if (F.lo[q] < best) {
        best = F.lo[q];
        j = q;
      }
    }
  }
  F.valid &= ~(1u << j);
  float slo = 0.0f, shi = 0.0f, sl = 0.0f;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    if (q == j) {
      slo = F.lo[q];
      shi = F.hi[q];
      sl = F.len[q];
    }
  }
  const int si = SL::scat(j);
  const DevScat& S = PL.s[si];
  Mu mu;
  float att, pint;
  if constexpr (LAZY) {
    // segment_terms with the flight's coefficients (mu.k is not needed here)
    mu.total = mu.scat = 0.0f;
#pragma unroll
    for (int q = 0; q < NSC; ++q) {
      if (q == si) {
        mu.total = F.mt[q];
        mu.scat = F.ms[q];
      }
    }
    const float ml = mu.total * sl;
    att = expf(-ml);
    pint = -expm1f(-ml);
  } else {
    segment_terms(S, tab, P.sp, sl, mu, att, pint);
  }
  float dmu_abs = 0.0f, dmu_sig = 0.0f;
  if (ADJ) {
    if (si == AA.abs_s) dmu_abs = S.n100 * 2200.0f / P.sp;
    if (si == AA.sig_s) dmu_sig = S.n100;
  }
  const bool split = SPLIT && order_of(P.lin) < PL.K && P.w >= PL.min_prob && mu.scat > 0.0f;
  if (LAZY && split) {
    if (P.w * (mu.scat / mu.total) * pint > 0.0f) {  // split_child's weight
      Pk C = P;
      C.px = F.sx;
      C.py = F.sy;
      C.pz = F.sz;
      C.t = F.t0;
      C.lin = P.lin * 8u + F.g + 1u;
      const int code = kUnbuilt | si << 2 | (int)((F.codes >> (4 * j)) & 0xFu) << 5;
      if (!has_nxt) {
        nxt = C;
        nxt_code = code;
        nxt_slo = slo;
        nxt_pint = pint;
        has_nxt = true;
      } else if (nst < PL.stack_cap) {
        push<false, true>(st, nst, PL.stack_cap, tid, C, pa, code, slo, pint);
        ++nst;
      }
    }
  } else if (!LAZY && split) {
    const uint32_t lin = P.lin * 8u + F.g + 1u;
    float u[8];
    draw4(id, STREAM_SCATTER, lin, 0u, seed, u);
    if (!DEFER) draw4(id, STREAM_SCATTER, lin, 1u, seed, u + 4);
    Pk C;
    float x;
    const int kk = split_child(S, mu, pint, P, F.sx, F.sy, F.sz, F.t0, slo,
                               (int)((F.codes >> (4 * j)) & 0xFu), u, lin, C, x);
    Adj ca;
    if (ADJ) {
      ca = pa;
      ca.dabs -= x * dmu_abs;
      ca.dsig -= x * dmu_sig;
    }
    int code = -1;
    if (DEFER) {
      C.dx = P.dx;
      C.dy = P.dy;
      C.dz = P.dz;
      C.sp = P.sp;
      code = 4 * si + kk;
    } else {
      const DevKernel& K = S.k[kk];
      const Out o = kernel_eval<HEAVY>(K, S, tab, P, u, id, lin, seed);
      C.dx = o.dx;
      C.dy = o.dy;
      C.dz = o.dz;
      C.sp = o.sp;
      C.w *= o.f;
      if (ADJ) kernel_carries(AA, S, K, tab, si, kk, o, u, id, lin, seed, ca);
    }
    if (C.w > 0.0f) {
      if (!has_nxt) {
        nxt = C;
        nxt_code = code;
        if (ADJ) na = ca;
        has_nxt = true;
      } else if (nst < PL.stack_cap) {
        push<ADJ>(st, nst, PL.stack_cap, tid, C, ca, code);
        ++nst;
      }
    }
  }
  P.w *= att;
  if (ADJ) {
    pa.dabs -= sl * dmu_abs;
    pa.dsig -= sl * dmu_sig;
  }
  F.s_end = shi;
  ++F.g;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// MODE_TAPE: the run's histogram plus, per recorded packet, a tape entry
// with the adjoint carry (for a later pass that needs no re-trace).
enum { MODE_RUN = 0, MODE_TRACE = 1, MODE_ADJOINT = 2, MODE_TAPE = 3 };

// modes whose packets carry the adjoint terms
__host__ __device__ constexpr bool carries(int mode) {
  return mode == MODE_ADJOINT || mode == MODE_TAPE;
}

// Resident waves per SIMD a transport kernel is compiled for, i.e. its
// register budget (512 / waves VGPRs per lane).  The run kernels take 4.
// The adjoint carry (10 words per packet) and the trace records need more
// registers: at 4 waves the walk-loop kernels of those modes spill 40-180
// VGPRs.  Measured (ms; 4 / 3 / 2 waves): powder at 1e7, re-trace 1.67 /
// 1.90 / 2.38 and histogram fill + tape run 2.18 / 1.99 / 2.49; crystal in
// its can at 1e7, re-trace 29.3 / 23.8 / 19.4 and tape run 31.5 / 23.3 /
// 19.3.  So walk loops take 2 waves outside the run mode, the phased loop 4
// (3 for the tape run).  The run kernels keep 4 waves despite a few spilled
// registers in the multi-interval and heavy ones: at 3 waves (no spills) the
// crystal took 119.3 ms instead of 113.3 ms at 1e8, the exact-delta crystal
// 30.0 ms instead of 26.9 ms at 1e7, and the batch kernel's graph 34.4 ms
// instead of 32.8 ms.
__host__ __device__ constexpr int kernel_waves(int mode, bool phased) {
  return mode == MODE_RUN ? MCV_WAVES_PER_EU
         : !phased        ? 2
         : mode == MODE_TAPE ? 3
                             : 4;
}
__host__ __device__ constexpr int kernel_waves_max(int mode, bool phased) {
  return kernel_waves(mode, phased) > MCV_WAVES_PER_EU_MAX ? kernel_waves(mode, phased)
                                                           : MCV_WAVES_PER_EU_MAX;
}

// where recorded values go (global memory only: the backend takes pointers
// that arrive in kernel arguments to be global, so LDS addresses never
// travel in this struct)
struct Sinks {
  double* hist;
  double* hist_w2;
  DevRecord* rec;
  uint64_t cap;
  unsigned long long* n_out;
  DevEvent* ev;  // event mode (MODE_RUN only; NULL: off)
  uint64_t ev_cap;
  unsigned long long* n_ev;
  int ev_hot_n;              // bin cache slots of event launches
  DevEvent* stage;           // this wave's LDS event stage (set in the kernel)
  volatile int* stage_n;     // events in the stage
  float* gstack;             // per-lane packet stacks in device memory (plan-owned)
  // deterministic summation (MODE_RUN; NULL: off): one (key, value) entry
  // per recorded packet, key = bin << (id_bits + lin_bits) | (id - det_first)
  // << lin_bits | lineage, staged like events
  uint64_t* dkeys;
  float* dvals;
  uint64_t det_cap;
  unsigned long long* n_det;
  uint64_t det_first;
  int det_lin_bits, det_id_bits;
  // adjoint tape (MODE_TAPE)
  uint32_t* tape;
  uint64_t tape_cap;
  unsigned long long* n_tape;
};

// Event mode: every wave stages its events in LDS (kEvStage entries) and
// copies the stage to the output with one counter atomic per kEvStage
// events or fewer, instead of one atomic per recording step, since all
// waves of the device share the one counter.
constexpr int kEvStage = 64;
constexpr int kEvStageWords = kEvStage * 4 + 4;  // per wave: events, count

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

// copies the first n staged events to the output; the active lanes of the
// wave (any subset) share the copy
__device__ __forceinline__ void ev_flush(const Sinks& out, int n) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  const uint64_t act = __ballot(1);
  const int lead = __ffsll((unsigned long long)act) - 1;
  const int na = __popcll(act);
  const int me = __popcll(act & lanemask_lt());
  unsigned long long base = 0ull;
  if ((int)__lane_id() == lead) base = atomicAdd(out.n_ev, (unsigned long long)n);
  base = readlane64(base, lead);
  for (int i = me; i < n; i += na) {
    const uint64_t slot = base + (uint64_t)i;
    if (slot < out.ev_cap) out.ev[slot] = out.stage[i];
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// stages one event per active lane with a recorded packet (divergent code)
__device__ __forceinline__ void event_append(const Sinks& out, int ntof, const Hit& hh,
                                             int order) {
  const bool rec = hh.bin >= 0;
  const uint64_t m = __ballot(rec);
  if (m == 0ull) return;
  const uint64_t act = __ballot(1);
  const int k = __popcll(m);
  int n = *out.stage_n;
  if (n + k > kEvStage) {
    ev_flush(out, n);
    n = 0;
  }
  if (rec) {
    DevEvent e;
    e.pixel = (uint32_t)hh.bin / (uint32_t)ntof;
    e.tof = hh.tof;
    e.value = hh.value;
    e.order = order;
    out.stage[n + __popcll(m & lanemask_lt())] = e;
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  if ((int)__lane_id() == __ffsll((unsigned long long)act) - 1) *out.stage_n = n + k;
}

// Deterministic summation: the wave's staged (key, value) entries are
// copied to the caller-sized arrays with one counter atomic per stage (the
// order they land in does not matter: they are sorted by key afterwards)
__device__ __forceinline__ void det_flush(const Sinks& out, int n) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  const uint64_t act = __ballot(1);
  const int lead = __ffsll((unsigned long long)act) - 1;
  const int na = __popcll(act);
  const int me = __popcll(act & lanemask_lt());
  unsigned long long base = 0ull;
  if ((int)__lane_id() == lead) base = atomicAdd(out.n_det, (unsigned long long)n);
  base = readlane64(base, lead);
  for (int i = me; i < n; i += na) {
    const uint64_t slot = base + (uint64_t)i;
    if (slot < out.det_cap) {
      const DevEvent e = out.stage[i];
      out.dkeys[slot] = ((uint64_t)(uint32_t)__float_as_uint(e.tof) << 32) | e.pixel;
      out.dvals[slot] = e.value;
    }
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// stages one (key, value) entry per active lane with a recorded packet
__device__ __forceinline__ void det_append(const Sinks& out, const Hit& hh, uint64_t hid,
                                           uint32_t lin) {
  const bool rec = hh.bin >= 0;
  const uint64_t m = __ballot(rec);
  if (m == 0ull) return;
  const uint64_t act = __ballot(1);
  const int k = __popcll(m);
  int n = *out.stage_n;
  if (n + k > kEvStage) {
    det_flush(out, n);
    n = 0;
  }
  if (rec) {
    const uint64_t key = ((uint64_t)hh.bin << (out.det_id_bits + out.det_lin_bits)) |
                         ((hid - out.det_first) << out.det_lin_bits) | (uint64_t)lin;
    DevEvent e;
    e.pixel = (uint32_t)key;
    e.tof = __uint_as_float((uint32_t)(key >> 32));
    e.value = hh.value;
    e.order = 0;
    out.stage[n + __popcll(m & lanemask_lt())] = e;
  }
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  if ((int)__lane_id() == __ffsll((unsigned long long)act) - 1) *out.stage_n = n + k;
}

// Histogram bins that many lanes of a wave hit at the same step (the
// unscattered beam lands in one pixel and one time bin for every history)
// would serialise on one global address.  Such lanes combine their values
// with a wave sum, and the group's first lane adds the sum into a
// per-workgroup LDS cache of n slots (direct mapped on the bin index, a slot
// claimed by compare-and-swap of its tag), which is flushed with one global
// atomic per slot when the workgroup ends.  For small histograms (`all`)
// lanes alone in their bin go through the cache as well, since a few hundred
// bins then take most updates; otherwise they add directly.
// Cache layout in LDS: double v[n], double v2[n], int tag[n] (-1 = free),
// n a power of two.
constexpr int kHotRounds = 2;

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ void hot_init(double* hot, int n, int nthreads, int tid) {
  int* tag = reinterpret_cast<int*>(hot + 2 * n);
  for (int i = tid; i < n; i += nthreads) {
    hot[i] = 0.0;
    hot[n + i] = 0.0;
    tag[i] = -1;
  }
}

// adds the cache into the histogram and clears it (after a barrier)
__device__ __forceinline__ void hot_flush(double* hot, int n, double* hist, double* hist_w2,
                                          int nthreads, int tid) {
  int* tag = reinterpret_cast<int*>(hot + 2 * n);
  for (int i = tid; i < n; i += nthreads) {
    const int b = tag[i];
    if (b >= 0) {
      if (hist) unsafeAtomicAdd(hist + b, hot[i]);
      if (hist_w2) unsafeAtomicAdd(hist_w2 + b, hot[n + i]);
    }
    hot[i] = 0.0;
    hot[n + i] = 0.0;
    tag[i] = -1;
  }
}

// adds (s, s2) for bin b into its cache slot if the slot holds b or is free;
// false if another bin owns it
__device__ __forceinline__ bool hot_put(double* hot, int n, int b, double s, double s2) {
  int* tag = reinterpret_cast<int*>(hot + 2 * n);
  const int slot = b & (n - 1);
  int t = tag[slot];
  if (t < 0) {
    const int old = atomicCAS(&tag[slot], -1, b);
    t = old < 0 ? b : old;
  }
  if (t != b) return false;
  atomicAdd(&hot[slot], s);
  atomicAdd(&hot[n + slot], s2);
  return true;
}

// one histogram contribution per lane (bin < 0: none); whole wave active
__device__ __forceinline__ void hist_add(double* hist, double* hist_w2, double* hot, int n,
                                         bool all, int bin, float value) {
  uint64_t pend = __ballot(bin >= 0);
  bool done = bin < 0;
  for (int r = 0; r < kHotRounds && pend != 0ull; ++r) {
    const int lead = __ffsll((unsigned long long)pend) - 1;
    const int lb = __builtin_amdgcn_readlane(bin, lead);
    const bool mine = bin == lb;
    const uint64_t grp = __ballot(mine);
    pend &= ~grp;
    if (__popcll(grp) < 2) continue;
    const double d = mine ? (double)value : 0.0;
    const double s = wave_sum(d);
    const double s2 = hist_w2 ? wave_sum(d * d) : 0.0;
    done = done || mine;
    if ((int)__lane_id() == lead && !hot_put(hot, n, lb, s, s2)) {
      if (hist) unsafeAtomicAdd(hist + lb, s);
      if (hist_w2) unsafeAtomicAdd(hist_w2 + lb, s2);
    }
  }
  if (!done) {
    const double v = (double)value;
    if (!(all && hot_put(hot, n, bin, v, v * v))) {
      if (hist) unsafeAtomicAdd(hist + bin, v);
      if (hist_w2) unsafeAtomicAdd(hist_w2 + bin, v * v);
    }
  }
}

// Appends one tape entry per active lane with a recorded packet (any subset
// of the wave may be active): one counter atomic per call, entries of a call
// at consecutive slots.  Entries beyond the capacity are counted, not
// written.
__device__ __forceinline__ void tape_append(const Sinks& out, int bin, float value, const Adj& a) {
  const bool rec = bin >= 0;
  const uint64_t m = __ballot(rec);
  if (m == 0ull) return;
  const int lead = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0ull;
  if ((int)__lane_id() == lead) base = atomicAdd(out.n_tape, (unsigned long long)__popcll(m));
  base = readlane64(base, lead);
  if (!rec) return;
  const uint64_t slot = base + (uint64_t)__popcll(m & lanemask_lt());
  if (slot >= out.tape_cap) return;
  const uint64_t c = out.tape_cap;
  uint32_t* t = out.tape + slot;
  __builtin_nontemporal_store((uint32_t)bin, t);
  __builtin_nontemporal_store(__float_as_uint(value), t + c);
  __builtin_nontemporal_store(__float_as_uint(a.dabs), t + 2 * c);
  __builtin_nontemporal_store(__float_as_uint(a.dsig), t + 3 * c);
  __builtin_nontemporal_store(__float_as_uint(a.A), t + 4 * c);
  __builtin_nontemporal_store(a.cnt, t + 5 * c);
  // only the words that hold the entry's table indices (the backward pass
  // reads no others): ceil(n / 2) for n indices
  const uint32_t nw = ((a.cnt >> 16) + 1u) >> 1;
#pragma unroll
  for (int w = 0; w < kAdjMaxSparse / 2; ++w)
    if ((uint32_t)w < nw) __builtin_nontemporal_store(a.s[w], t + (6 + w) * c);
}

// Lane states of the transport loop
enum { LANE_NEED = 0, LANE_SETUP = 1, LANE_FLY = 2, LANE_DET = 3, LANE_DONE = 4 };

// Recording of one packet leaving the sample: detector, histogram value or
// adjoint gather, and the packet record in MODE_TRACE.
// In adjoint mode with `sc` given, the four scalar partials (g d log w /
// d sigma_abs, d sigma, g A, g n_draws) are returned there for the caller to
// combine over the wave; otherwise they are added to the LDS partials here.
template <int MODE>
__device__ __forceinline__ void record_packet(const DevPlan& PL, const float* tab,
                                              const Sinks& out, const AdjArgs& AA, double* acc,
                                              const Pk& cur, const Adj& ca, uint64_t hid,
                                              uint64_t seed, int& hbin, float& hval,
                                              double* sc_out = nullptr) {
  constexpr bool GATHER = MODE == MODE_ADJOINT;
  const Hit hh = PL.det.type == DET_SPHERE ? detect_sphere(PL.det, cur)
                                           : detect_tubes(PL.det, tab, cur, hid, seed);
  if (MODE == MODE_TAPE) tape_append(out, hh.bin, hh.value, ca);
  if (hh.bin >= 0) {
    if (GATHER) {
      const double gv = AA.dLdI[hh.bin] * (double)hh.value;
      if (gv != 0.0) {
        // LDS partials: [table entries (when they fit) | 4 scalars]
        if (sc_out) {
          sc_out[0] = gv * (double)ca.dabs;
          sc_out[1] = gv * (double)ca.dsig;
          sc_out[2] = gv * (double)ca.A;
          sc_out[3] = gv * (double)(ca.cnt & 0xFFFFu);
        } else {
          double* sc = acc + (AA.sparse_lds ? AA.nb + AA.nc : 0);
          atomicAdd(&sc[0], gv * (double)ca.dabs);
          atomicAdd(&sc[1], gv * (double)ca.dsig);
          atomicAdd(&sc[2], gv * (double)ca.A);
          atomicAdd(&sc[3], gv * (double)(ca.cnt & 0xFFFFu));
        }
        const uint32_t ns = ca.cnt >> 16;
#pragma unroll
        for (int w = 0; w < kAdjMaxSparse / 2; ++w) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            if ((uint32_t)(2 * w + h) < ns) {
              const uint32_t idx = (ca.s[w] >> (16 * h)) & 0xFFFFu;
              if (AA.sparse_lds) atomicAdd(&acc[idx], gv);
              else unsafeAtomicAdd(&AA.grad[idx], gv * AA.ws[4 + idx]);
            }
          }
        }
      }
    } else {
      hbin = hh.bin;
      hval = hh.value;
    }
  }
  if (MODE == MODE_RUN && out.ev != nullptr) event_append(out, PL.det.ntof, hh, order_of(cur.lin));
  if (MODE == MODE_RUN && out.dkeys != nullptr) det_append(out, hh, hid, cur.lin);
  if (MODE == MODE_TRACE) {
    const unsigned long long slot = atomicAdd(out.n_out, 1ull);
    if (slot < out.cap) {
      DevRecord r;
      r.id = hid;
      r.lineage = cur.lin;
      r.order = order_of(cur.lin);
      r.pos[0] = cur.px;
      r.pos[1] = cur.py;
      r.pos[2] = cur.pz;
      r.vel[0] = cur.dx * cur.sp;
      r.vel[1] = cur.dy * cur.sp;
      r.vel[2] = cur.dz * cur.sp;
      r.t = cur.t;
      r.w = cur.w;
      r.bin = hh.bin;
      r.value = hh.value;
      r.tof = hh.tof;
      r.tube = hh.tube;
      r.pixel = hh.pixel;
      out.rec[slot] = r;
    }
  }
}

// Detection queue of a wave (phased loop, tube detectors, run and trace
// modes): of the packets recorded in a D phase, only those whose ray passes
// the first steps of the tube test (tube_column: about one in six for the
// powder) need the rest of it (candidate tubes, absorption, a Philox block,
// bin).  Run in the D phase, that rest would take the whole wave for the few
// lanes holding such packets; instead they are appended to a per-wave LDS
// queue of Q packets, which the wave records together (one packet per lane)
// when the next D phase would overflow it, and at the end.  The walk loop
// does the same with its recording step.  Layout: [field][entry], 12 fields
// (position, direction, speed, time, weight, lineage, history id low and
// high words), then the adjoint carry in adjoint launches.
constexpr int kDqFields = 12;
constexpr int kDqAdjFields = kDqFields + kAdjFields;  // adjoint: the carry follows
constexpr int kDqPhased = 64;     // entries per wave, phased loop
constexpr int kDqWalk = 64;       // entries per wave, walk loop

template <int Q, bool ADJ>
__device__ __forceinline__ void dq_put(float* q, int slot, const Pk& P, uint64_t hid,
                                       const Adj& a) {
  constexpr int kDqEntries = Q;
  float* b = q + slot;
  b[0 * kDqEntries] = P.px;
  b[1 * kDqEntries] = P.py;
  b[2 * kDqEntries] = P.pz;
  b[3 * kDqEntries] = P.dx;
  b[4 * kDqEntries] = P.dy;
  b[5 * kDqEntries] = P.dz;
  b[6 * kDqEntries] = P.sp;
  b[7 * kDqEntries] = P.t;
  b[8 * kDqEntries] = P.w;
  b[9 * kDqEntries] = __uint_as_float(P.lin);
  b[10 * kDqEntries] = __uint_as_float((uint32_t)hid);
  b[11 * kDqEntries] = __uint_as_float((uint32_t)(hid >> 32));
  if (ADJ) {
    b[12 * kDqEntries] = a.dabs;
    b[13 * kDqEntries] = a.dsig;
    b[14 * kDqEntries] = a.A;
    b[15 * kDqEntries] = __uint_as_float(a.cnt);
#pragma unroll
    for (int w = 0; w < kAdjMaxSparse / 2; ++w)
      b[(16 + w) * kDqEntries] = __uint_as_float(a.s[w]);
  }
}

// records the n queued packets, one per lane (called with the whole wave
// active; a wave of fewer lanes takes several passes).  In adjoint mode the
// scalar partials of the pass are summed over the wave and added to LDS by
// one lane.
template <int MODE, int Q>
__device__ __forceinline__ void dq_run(const DevPlan& PL, const float* tab, const Sinks& out,
                                       const AdjArgs& AA, double* acc, int hot_n, const float* q,
                                       int n, uint64_t seed) {
  constexpr bool ADJ = carries(MODE);
  constexpr bool GATHER = MODE == MODE_ADJOINT;
  constexpr int kDqEntries = Q;
  const int nl = __popcll(__ballot(1));
  for (int base = 0; base < n; base += nl) {
    const int i = base + (int)__lane_id();
    int hbin = -1;
    float hval = 0.0f;
    double sc[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < n) {
      const float* b = q + i;
      Pk P;
      P.px = b[0 * kDqEntries];
      P.py = b[1 * kDqEntries];
      P.pz = b[2 * kDqEntries];
      P.dx = b[3 * kDqEntries];
      P.dy = b[4 * kDqEntries];
      P.dz = b[5 * kDqEntries];
      P.sp = b[6 * kDqEntries];
      P.t = b[7 * kDqEntries];
      P.w = b[8 * kDqEntries];
      P.lin = __float_as_uint(b[9 * kDqEntries]);
      const uint64_t hid = (uint64_t)__float_as_uint(b[10 * kDqEntries]) |
                           ((uint64_t)__float_as_uint(b[11 * kDqEntries]) << 32);
      Adj ca = adj_zero();
      if (ADJ) {
        ca.dabs = b[12 * kDqEntries];
        ca.dsig = b[13 * kDqEntries];
        ca.A = b[14 * kDqEntries];
        ca.cnt = __float_as_uint(b[15 * kDqEntries]);
#pragma unroll
        for (int w = 0; w < kAdjMaxSparse / 2; ++w)
          ca.s[w] = __float_as_uint(b[(16 + w) * kDqEntries]);
      }
      record_packet<MODE>(PL, tab, out, AA, acc, P, ca, hid, seed, hbin, hval,
                          GATHER ? sc : nullptr);
    }
    if (GATHER) {
      double* dst = acc + (AA.sparse_lds ? AA.nb + AA.nc : 0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double v = wave_sum(sc[k]);
        if (__lane_id() == 0 && v != 0.0) atomicAdd(&dst[k], v);
      }
    } else if (out.hist != nullptr || out.hist_w2 != nullptr) {
      hist_add(out.hist, out.hist_w2, acc, hot_n, PL.hot_all != 0, hbin, hval);
    }
  }
}

// One wave traces histories first+begin .. first+end-1.  Every lane walks
// the packet tree of one history depth first (first child in registers,
// further children on its LDS stack) and takes the next history of the range
// when its tree is done (ballot + prefix count).  Two loop shapes:
//
// trace_walk: every iteration, each lane takes one packet through all the
// material intervals of its ray (splitting where it may) and records it.
// Lanes stay in step when the packets of a history are alike (one scatterer
// and single scattering, or several scatterers whose flights vary anyway).
// With several scatterers, an annulus or the heavy kernels, a child's kernel
// is evaluated when the child is taken up, at the top of an iteration where
// most lanes take up a child together, rather than inside the interval loop
// where only the lanes that split in that interval are active.
//
// trace_phased: the work of a packet is split into two phases that the wave
// runs one at a time, whichever has more lanes waiting, so that lanes in the
// same phase run together:
//   I: one material interval of a packet that can still scatter
//      (attenuation, forced-collision child, kernel);
//   D: detection and histogram of a finished packet, then the next packet
//      (first child, stack, or a new history) and the intervals of its ray;
//      a packet that can no longer scatter crosses all of them here with
//      attenuation only and waits for the next D phase.
// Called with the whole wave active.  `acc` is the workgroup's LDS block:
// adjoint partials (MODE_ADJOINT) or the histogram bin cache (otherwise).
template <int MODE, int NSC, bool TWO, bool HEAVY, int DQ>
__device__ __forceinline__ void trace_phased(const DevPlan& PL, const float* tab, float* st,
                                             const DevBeam& beam, uint64_t seed, uint64_t first,
                                             uint64_t begin, uint64_t end, const Sinks& out,
                                             const AdjArgs& AA, double* acc, int hot_n,
                                             int nthreads, int tid, float* dq) {
  constexpr bool ADJ = carries(MODE);
  static_assert(DQ == 0 || DQ == kDqPhased, "phased-loop queue size");
  const uint64_t lt = lanemask_lt();
  Pk cur;
  cur.lin = 0u;
  Pk nxt;
  nxt.lin = 0u;
  Adj ca = adj_zero();
  Adj na = ca;
  bool has_nxt = false;
  int code = -1;  // kernels are evaluated at birth in this loop (no deferral)
  float unused = 0.0f;
  Flight<NSC, TWO> F;
  F.valid = 0u;
  F.g = 0u;
  uint64_t hid = 0;
  int nst = 0;
  int state = LANE_NEED;
  uint64_t next = begin;
  int qn = 0;  // packets in the detection queue (the same in every lane)
  while (true) {
    const uint64_t mI = __ballot(state == LANE_FLY);
    const uint64_t mD = __ballot(state == LANE_NEED || state == LANE_DET);
    if ((mI | mD) == 0ull) {
      if (DQ && qn > 0) dq_run<MODE, DQ>(PL, tab, out, AA, acc, hot_n, dq, qn, seed);
      break;
    }
    if (__popcll(mI) >= __popcll(mD)) {
      if (state == LANE_FLY) {
        flight_step<ADJ, true, false, NSC, TWO, HEAVY>(PL, tab, AA, cur, ca, F, hid, seed, nxt, na,
                                                     code, has_nxt, st, nst, nthreads, tid, unused,
                                                     unused);
        if (F.valid == 0u) {
          flight_exit(cur, F);
          state = LANE_DET;
        }
      }
      continue;
    }
    int hbin = -1;
    float hval = 0.0f;
    if constexpr (DQ > 0) {
      float a;
      uint32_t rows;
      int col;
      const bool q = state == LANE_DET && tube_column(PL.det, cur, a, rows, col);
      const uint64_t mq = __ballot(q);
      const int k = __popcll(mq);
      if (qn + k > DQ) {
        dq_run<MODE, DQ>(PL, tab, out, AA, acc, hot_n, dq, qn, seed);
        qn = 0;
      }
      if (q) dq_put<DQ, ADJ>(dq, qn + __popcll(mq & lt), cur, hid, ca);
      qn += k;
      // a packet that meets no tube leaves no histogram entry; trace mode
      // still writes its record
      if (MODE == MODE_TRACE && state == LANE_DET && !q)
        record_packet<MODE>(PL, tab, out, AA, acc, cur, ca, hid, seed, hbin, hval);
    }
    if (state == LANE_DET) {
      if (!DQ) record_packet<MODE>(PL, tab, out, AA, acc, cur, ca, hid, seed, hbin, hval);
      if (has_nxt) {
        cur = nxt;
        if (ADJ) ca = na;
        has_nxt = false;
        state = LANE_SETUP;
      } else {
        state = LANE_NEED;
      }
    }
    if (state == LANE_NEED && nst > 0) {
      --nst;
      pop<ADJ>(st, nst, PL.stack_cap, tid, cur, ca, code, unused, unused);
      state = LANE_SETUP;
    }
    const bool need = state == LANE_NEED;
    const uint64_t m = __ballot(need);
    if (need) {
      const uint64_t h = next + (uint64_t)__popcll(m & lt);
      if (h < end) {
        hid = first + h;
        cur = source(beam, hid, seed);
        ca = adj_zero();
        if (cur.w > 0.0f) state = LANE_SETUP;
      } else {
        state = LANE_DONE;
      }
    }
    next += (uint64_t)__popcll(m);
    if (state == LANE_SETUP) {
      flight_setup(PL, cur, F);
      if (order_of(cur.lin) >= PL.K || cur.w < PL.min_prob) {
        while (F.valid != 0u)
          flight_step<ADJ, false, false, NSC, TWO, HEAVY>(PL, tab, AA, cur, ca, F, hid, seed, nxt,
                                                        na, code, has_nxt, st, nst, nthreads, tid,
                                                        unused, unused);
      }
      if (F.valid != 0u) {
        state = LANE_FLY;
      } else {
        flight_exit(cur, F);
        state = LANE_DET;
      }
    }
    if (MODE != MODE_ADJOINT && !DQ && (out.hist != nullptr || out.hist_w2 != nullptr))
      hist_add(out.hist, out.hist_w2, acc, hot_n, PL.hot_all != 0, hbin, hval);
  }
}

template <int MODE, int NSC, bool TWO, bool HEAVY, int DQ>
__device__ __forceinline__ void trace_walk(const DevPlan& PL, const float* tab, float* st,
                                           const DevBeam& beam, uint64_t seed, uint64_t first,
                                           uint64_t begin, uint64_t end, const Sinks& out,
                                           const AdjArgs& AA, double* acc, int hot_n,
                                           int nthreads, int tid, float* dq) {
  constexpr bool ADJ = carries(MODE);
  static_assert(DQ == 0 || DQ == kDqWalk, "walk-loop queue size");
  constexpr bool DEFER = NSC > 1 || TWO || HEAVY;
  // children built when taken up (run and trace modes with deferred kernels)
  constexpr bool LAZY = DEFER && !ADJ;
  // exact-delta dispersion draws gathered across iterations (see below)
  constexpr bool GATHER_DISP = HEAVY && LAZY;
  int waited = 0;  // iterations this lane's dispersion draw has waited
  const uint64_t lt = lanemask_lt();
  Pk cur;
  cur.lin = 0u;
  Adj ca = adj_zero();
  bool has = false;
  int code = -1;
  float cslo = 0.0f, cpint = 0.0f;  // an unbuilt current child's interval
  uint64_t hid = 0;
  int nst = 0;
  uint64_t next = begin;
  int qn = 0;  // packets in the detection queue (the same in every lane)
  while (true) {
    if (!has && nst > 0) {
      --nst;
      pop<ADJ, LAZY>(st, nst, PL.stack_cap, tid, cur, ca, code, cslo, cpint);
      has = true;
    }
    const bool need = !has;
    const uint64_t m = __ballot(need);
    if (need) {
      const uint64_t h = next + (uint64_t)__popcll(m & lt);
      if (h < end) {
        hid = first + h;
        cur = source(beam, hid, seed);
        ca = adj_zero();
        code = -1;
        has = cur.w > 0.0f;
      }
    }
    next += (uint64_t)__popcll(m);
    if (__ballot(has) == 0ull) {
      // every lane drew a history that carries nothing (a saved-beam entry
      // of weight zero) while ids remain: draw again (next is the same in
      // every lane, so the whole wave takes this branch together)
      if (next < end) continue;
      if (DQ && qn > 0) dq_run<MODE, DQ>(PL, tab, out, AA, acc, hot_n, dq, qn, seed);
      break;
    }
    // With the exact-delta kernel, a child that draws it waits (keeps its
    // code and skips this iteration) unless at least kDispMin lanes draw it
    // now, no lane has other work, or some lane has waited kDispWaitMax
    // iterations: the kernel's root scan then runs for many lanes at once
    // instead of for the few of each iteration.  Every wait ends (the last
    // two conditions); the draws are those of an immediate evaluation.
    bool wait = false;
    if constexpr (GATHER_DISP) {
      if (has && code >= 0 && (code & kUnbuilt)) {
        float u[4];
        draw4(hid, STREAM_SCATTER, cur.lin, 0u, seed, u);
        const int si = (code >> 2) & 3;
        code = 4 * si + build_child(PL.s[si], tab, cur, code, cslo, cpint, u);
      }
      const bool disp = has && code >= 0 && PL.s[(code >> 2) & 3].k[code & 3].type == K_DISPERSION;
      const uint64_t md = __ballot(disp);
      const bool others = __ballot(has && !disp) != 0ull;
      const bool overdue = __ballot(disp && waited >= kDispWaitMax) != 0ull;
      wait = disp && others && !overdue && __popcll(md) < kDispMin;
      waited = wait ? waited + 1 : 0;
    }
    if (DEFER && has && code >= 0 && !wait) {
      eval_deferred<ADJ, HEAVY, LAZY>(PL, tab, AA, cur, ca, code, hid, seed, cslo, cpint);
      code = -1;
      has = cur.w > 0.0f;  // a kernel of weight zero ends the child
    }
    const bool go = has && !wait;  // this lane's packet flies in this iteration
    int hbin = -1;
    float hval = 0.0f;
    Pk nxt;
    nxt.lin = 0u;
    Adj na = ca;
    int nxt_code = -1;
    float nxt_slo = 0.0f, nxt_pint = 0.0f;
    bool has_nxt = false;
    if (go) {
      Flight<NSC, TWO> F;
      flight_setup(PL, cur, F);
      if (LAZY) flight_coefs(PL, tab, cur.sp, F);
      while (F.valid != 0u)
        flight_step<ADJ, true, DEFER, NSC, TWO, HEAVY, LAZY>(PL, tab, AA, cur, ca, F, hid, seed,
                                                            nxt, na, nxt_code, has_nxt, st, nst,
                                                            nthreads, tid, nxt_slo, nxt_pint);
      flight_exit(cur, F);
      if (!DQ) record_packet<MODE>(PL, tab, out, AA, acc, cur, ca, hid, seed, hbin, hval);
    }
    if constexpr (DQ > 0) {
      float a;
      uint32_t rows;
      int col;
      const bool q = go && tube_column(PL.det, cur, a, rows, col);
      const uint64_t mq = __ballot(q);
      const int k = __popcll(mq);
      if (qn + k > DQ) {
        dq_run<MODE, DQ>(PL, tab, out, AA, acc, hot_n, dq, qn, seed);
        qn = 0;
      }
      if (q) dq_put<DQ, ADJ>(dq, qn + __popcll(mq & lt), cur, hid, ca);
      qn += k;
      if (MODE == MODE_TRACE && go && !q)
        record_packet<MODE>(PL, tab, out, AA, acc, cur, ca, hid, seed, hbin, hval);
    }
    if (go) {
      if (has_nxt) {
        cur = nxt;
        code = nxt_code;
        cslo = nxt_slo;
        cpint = nxt_pint;
        if (ADJ) ca = na;
      } else {
        has = false;
      }
    }
    if (MODE != MODE_ADJOINT && !DQ && (out.hist != nullptr || out.hist_w2 != nullptr))
      hist_add(out.hist, out.hist_w2, acc, hot_n, PL.hot_all != 0, hbin, hval);
  }
}

// The phased loop pays off for one convex scatterer with multiple
// scattering (every flight one interval, a quarter to a half of the packets
// unable to scatter); the walk is faster for single scattering and for
// assemblies whose flights cross several intervals (measured).
__host__ __device__ constexpr bool use_phased(int nscat, bool two, int K) {
  return nscat <= 1 && !two && K >= 2;
}

template <int MODE, int NSC, bool TWO, bool PHASED, bool HEAVY, int DQ = 0>
__device__ __forceinline__ void trace_range(const DevPlan& PL, const float* tab, float* st,
                                            const DevBeam& beam, uint64_t seed, uint64_t first,
                                            uint64_t begin, uint64_t end, const Sinks& out,
                                            const AdjArgs& AA, double* acc, int hot_n,
                                            int nthreads, int tid, float* dq = nullptr) {
  if constexpr (PHASED)
    trace_phased<MODE, NSC, TWO, HEAVY, DQ>(PL, tab, st, beam, seed, first, begin, end, out, AA,
                                            acc, hot_n, nthreads, tid, dq);
  else
    trace_walk<MODE, NSC, TWO, HEAVY, DQ>(PL, tab, st, beam, seed, first, begin, end, out, AA, acc,
                                          hot_n, nthreads, tid, dq);
}

// copies a plan and its tables into LDS (whole workgroup)
__device__ __forceinline__ void stage_plan(DevPlan& PL, float* dyn, const DevPlan* gplan,
                                           const float* gtab, int nthreads, int tid) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(gplan);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&PL);
  for (int i = tid; i < (int)(sizeof(DevPlan) / 4); i += nthreads) dst[i] = src[i];
  const int nt = gplan->n_tables;
  for (int i = tid; i < nt; i += nthreads) dyn[i] = gtab[i];
}

// MODE_RUN: histogram only.  MODE_TRACE: also one record per packet leaving
// the sample.  MODE_ADJOINT: re-traces the same histories (same random
// numbers) and accumulates dL/dtheta = sum over recorded packets of
// dL/dI[bin] * value * d log(w)/d theta into FP64 LDS partials, flushed once
// per workgroup.  MODE_TAPE: the run's histogram, and the packets carry the
// adjoint terms as in MODE_ADJOINT, written to the tape when recorded.
template <int MODE, int NSC, bool TWO, bool PHASED, bool HEAVY, int DQ = 0>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(kernel_waves(MODE, PHASED), kernel_waves_max(MODE, PHASED))))
transport(const DevPlan* __restrict__ gplan, const float* __restrict__ gtab, DevBeam beam,
          uint64_t seed, uint64_t first, uint64_t n, uint64_t per_wave, Sinks out, AdjArgs AA) {
  constexpr bool ADJ = MODE == MODE_ADJOINT;  // LDS partials instead of the bin cache
  constexpr bool CARRY = carries(MODE);
  __shared__ DevPlan PL;
  extern __shared__ __align__(16) float dyn[];
  const int tid = threadIdx.x;
  const int nthreads = blockDim.x;
  stage_plan(PL, dyn, gplan, gtab, nthreads, tid);
  const int tab_words = (gplan->n_tables + 3) & ~3;
  // adjoint partials: per table entry (sum of g; when they fit in LDS), then
  // sigma_abs, sigma, A, DOS draws; otherwise the histogram bin cache
  double* acc = reinterpret_cast<double*>(dyn + tab_words);
  const bool events = MODE == MODE_RUN && (out.ev != nullptr || out.dkeys != nullptr);
  const int hot_n = events ? out.ev_hot_n : gplan->hot_n;
  const int ntab = ADJ && AA.sparse_lds ? AA.nb + AA.nc : 0;
  const int acc_words = ADJ ? 2 * (((ntab + 4) + 1) & ~1) : hot_words(hot_n);
  if (ADJ)
    for (int i = tid; i < ntab + 4; i += nthreads) acc[i] = 0.0;
  else
    hot_init(acc, hot_n, nthreads, tid);
  __syncthreads();
  // the workgroup's packet stacks in device memory ([slot][field][lane],
  // consecutive lanes at consecutive addresses; a lane pushes only the
  // second and later children of a flight)
  float* st = out.gstack + (size_t)blockIdx.x * PL.stack_cap * stack_words(CARRY) * nthreads;
  // LDS after the bin cache: the waves' detection queues, then their event
  // stages
  float* dqs = dyn + tab_words + acc_words;
  const uint64_t wave = ((uint64_t)blockIdx.x * nthreads + tid) >> 6;
  const uint64_t begin = wave * per_wave;
  Sinks o = out;
  constexpr int DQF = CARRY ? kDqAdjFields : kDqFields;
  float* dq = dqs + (tid >> 6) * DQ * DQF;
  float* evs = dqs + (nthreads >> 6) * DQ * DQF;
  if (events) {
    float* sw = evs + (tid >> 6) * kEvStageWords;
    o.stage = reinterpret_cast<DevEvent*>(sw);
    o.stage_n = reinterpret_cast<volatile int*>(sw + kEvStage * 4);
    if ((tid & 63) == 0) *o.stage_n = 0;
  }
  if (begin < n) {  // uniform per wave
    trace_range<MODE, NSC, TWO, PHASED, HEAVY, DQ>(PL, dyn, st, beam, seed, first, begin,
                                                   begin + per_wave < n ? begin + per_wave : n, o,
                                                   AA, acc, hot_n, nthreads, tid, dq);
    if (events) {
      const int left = *o.stage_n;
      if (left > 0) {
        if (o.dkeys != nullptr) det_flush(o, left);
        else ev_flush(o, left);
      }
    }
  }
  if (!ADJ) {
    __syncthreads();
    hot_flush(acc, hot_n, out.hist, out.hist_w2, nthreads, tid);
  }
  if (ADJ) {
    __syncthreads();
    for (int i = tid; i < ntab; i += nthreads)
      if (acc[i] != 0.0) unsafeAtomicAdd(&AA.grad[i], acc[i] * AA.ws[4 + i]);
    if (tid == 0) {
      const int np = AA.nb + AA.nc;
      unsafeAtomicAdd(&AA.grad[np], acc[ntab]);
      unsafeAtomicAdd(&AA.grad[np + 1], acc[ntab + 1]);
      unsafeAtomicAdd(&AA.ws[0], acc[ntab + 2]);
      unsafeAtomicAdd(&AA.ws[1], acc[ntab + 3]);
    }
  }
}

// Persistent batched transport: workgroups pop chunks (simulation, id
// range) from a global cursor until the list is exhausted (every workgroup
// reads the same popped index after a barrier, so all leave together).  A
// workgroup re-stages plan and tables in LDS only when the simulation
// changes; its waves split the chunk's ids.  The list is sorted by
// estimated cost, longest first.  HV: some plan of the batch has an
// exact-delta or coherent-phonon kernel (the instantiation without them
// keeps their register budget out of the other batches).
template <bool HV>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(MCV_BATCH_WAVES_PER_EU, MCV_WAVES_PER_EU_MAX)))
batch_persistent(const BatchItem* __restrict__ items, const BatchChunk* __restrict__ chunks,
                 uint32_t n_chunks, uint32_t* __restrict__ cursor, int hot_n, int dq_off,
                 float* __restrict__ gstack, int stack_max) {
  __shared__ DevPlan PL;
  __shared__ uint32_t s_chunk;
  extern __shared__ __align__(16) float dyn[];
  const int tid = threadIdx.x;
  const int nthreads = blockDim.x;
  const int nwaves = nthreads >> 6;
  const int wid = tid >> 6;
  int staged = -1;
  AdjArgs AA = {};
  double* hot = reinterpret_cast<double*>(dyn);
  hot_init(hot, hot_n, nthreads, tid);
  for (;;) {
    if (tid == 0) s_chunk = atomicAdd(cursor, 1u);
    __syncthreads();
    const uint32_t c = s_chunk;
    if (c >= n_chunks) break;
    const BatchChunk ch = chunks[c];
    const BatchItem& it = items[ch.item];
    if ((int)ch.item != staged) {
      stage_plan(PL, dyn + hot_words(hot_n), it.plan, it.tables, nthreads, tid);
      staged = (int)ch.item;
    }
    __syncthreads();
    const int tab_words = (PL.n_tables + 3) & ~3;
    float* tab = dyn + hot_words(hot_n);
    // the workgroup's packet stacks in device memory, sized for the largest
    // stack of the batch's plans
    float* st = gstack + (size_t)blockIdx.x * stack_max * stack_words(false) * nthreads;
    const uint64_t per = (ch.count + nwaves - 1) / nwaves;
    const uint64_t b = ch.first + per * wid;
    const uint64_t e = ch.first + ch.count;
    Sinks out = {it.hist, nullptr, nullptr, 0, nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr,
                 nullptr, nullptr, nullptr, 0, nullptr, 0, 0, 0};
    const uint64_t ee = b + per < e ? b + per : e;
    // the waves' detection queues sit behind the largest tables and stacks
    float* dq = dyn + dq_off;  // this wave's queue: dq + wid Q kDqFields
    // the same specialisation as a plain launch of this plan, so that both
    // evaluate identical arithmetic
    const bool two = PL.smax > PL.nscat;
#define MCV_BATCH_TRACE(NSC_, TWO_, PH_, HV_)                                            \
  do {                                                                                     \
    constexpr int Q_ = PH_ ? kDqPhased : kDqWalk;                                          \
    if (PL.det.type == DET_TUBES)                                                          \
      trace_range<MODE_RUN, NSC_, TWO_, PH_, HV_, Q_>(PL, tab, st, it.beam, it.seed,       \
                                                      it.id0, b, ee, out, AA, hot, hot_n,  \
                                                      nthreads, tid,                       \
                                                      dq + wid * Q_ * kDqFields);          \
    else                                                                                   \
      trace_range<MODE_RUN, NSC_, TWO_, PH_, HV_>(PL, tab, st, it.beam, it.seed, it.id0,   \
                                                  b, ee, out, AA, hot, hot_n, nthreads,    \
                                                  tid);                                    \
  } while (0)
#define MCV_BATCH_SHAPES(HV_)                                                       \
  if (PL.nscat <= 1) {                                                              \
    if (two) MCV_BATCH_TRACE(1, true, false, HV_);                                  \
    else if (use_phased(PL.nscat, two, PL.K)) MCV_BATCH_TRACE(1, false, true, HV_); \
    else MCV_BATCH_TRACE(1, false, false, HV_);                                     \
  } else if (PL.nscat == 2) {                                                       \
    if (two) MCV_BATCH_TRACE(2, true, false, HV_);                                  \
    else MCV_BATCH_TRACE(2, false, false, HV_);                                     \
  } else {                                                                          \
    if (two) MCV_BATCH_TRACE(4, true, false, HV_);                                  \
    else MCV_BATCH_TRACE(4, false, false, HV_);                                     \
  }
    if (b < e) {
      if (HV && PL.heavy) {
        MCV_BATCH_SHAPES(HV)
      } else {
        MCV_BATCH_SHAPES(false)
      }
    }
#undef MCV_BATCH_SHAPES
#undef MCV_BATCH_TRACE
    __syncthreads();
    hot_flush(hot, hot_n, it.hist, nullptr, nthreads, tid);
  }
}

// zeroes a list of FP64 arrays and the chunk cursor (graph-capturable; no
// memset nodes)
__global__ void batch_cursor_reset(uint32_t* cursor) {
  if (threadIdx.x == 0) *cursor = 0u;
}

// n binary64 zeros from p (8-byte aligned): one scalar store for a head
// that is not 16-byte aligned, then one 16-byte store per lane over a grid
// that covers the array (measured on 1.024 GB: 6.9 TB/s; a grid of 8
// workgroups per CU looping over it, plain or non-temporal: 4.3-4.8 TB/s)
__global__ void __launch_bounds__(256) fill_zero(double* __restrict__ p, uint64_t n) {
  typedef double zvec2 __attribute__((ext_vector_type(2)));
  const uint64_t head = ((uintptr_t)p & 15u) ? 1u : 0u;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0 && head && n > 0) p[0] = 0.0;
  if (n <= head) return;
  zvec2* q = reinterpret_cast<zvec2*>(p + head);
  const uint64_t m = (n - head) / 2;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const zvec2 z = {0.0, 0.0};
  for (uint64_t i = gid; i < m; i += stride) q[i] = z;
  if (gid == 0 && ((n - head) & 1u)) p[n - 1] = 0.0;
}

// L = sum_b w_b (I_b - T_b)^2 and dL/dI_b = 2 w_b (I_b - T_b), streaming;
// one atomic per workgroup for L.  Every element is touched once, so loads
// and stores are non-temporal; one 16-byte pair of each array per lane per
// pass over a grid of 64 workgroups per CU (measured on 1.28e8 bins: 5.0
// TB/s, against 4.6 TB/s for 8 workgroups per CU with two pairs in flight
// per lane and 4.3-4.9 TB/s for plain loads).
typedef double dvec2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ double loss_pair(const dvec2 a, const dvec2 b, const dvec2 c,
                                            dvec2* o) {
  const double d0 = a.x - b.x, d1 = a.y - b.y;
  dvec2 g;
  g.x = 2.0 * c.x * d0;
  g.y = 2.0 * c.y * d1;
  __builtin_nontemporal_store(g, o);
  return c.x * d0 * d0 + c.y * d1 * d1;
}

__global__ void __launch_bounds__(256) loss_grad(const double* __restrict__ I,
                                                 const double* __restrict__ T,
                                                 const double* __restrict__ w, int64_t n,
                                                 double* __restrict__ dLdI,
                                                 double* __restrict__ loss) {
  __shared__ double part[4];
  double acc = 0.0;
  const dvec2* I2 = reinterpret_cast<const dvec2*>(I);
  const dvec2* T2 = reinterpret_cast<const dvec2*>(T);
  const dvec2* w2 = reinterpret_cast<const dvec2*>(w);
  dvec2* o2 = reinterpret_cast<dvec2*>(dLdI);
  const int64_t n2 = n / 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n2; q += stride)
    acc += loss_pair(__builtin_nontemporal_load(I2 + q), __builtin_nontemporal_load(T2 + q),
                     __builtin_nontemporal_load(w2 + q), o2 + q);
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t i = n - 1;
    const double d0 = I[i] - T[i];
    dLdI[i] = 2.0 * w[i] * d0;
    acc += w[i] * d0 * d0;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += part[i];
    unsafeAtomicAdd(loss, t);
  }
}

}  // namespace dev

// ------------------------------------------------------------------ launch
// LDS of the waves' detection queues, for plans that use them: phased loop
// (one convex scatterer, K >= 2) and a tube detector, outside the adjoint
int transport_dq_entries(const DevPlan& P) {
  if (P.det.type != DET_TUBES) return 0;
  return dev::use_phased(P.nscat, P.smax > P.nscat, P.K) ? dev::kDqPhased : dev::kDqWalk;
}
int batch_dq_entries(const DevPlan& P) { return transport_dq_entries(P); }
size_t transport_dq_bytes(int block, int entries, bool adjoint) {
  return sizeof(float) * (size_t)entries * (adjoint ? dev::kDqAdjFields : dev::kDqFields) *
         (size_t)(block / 64);
}

// adj_ntab: kLdsNoAdjoint outside the adjoint, else the table partials kept
// in LDS
size_t transport_lds_bytes(int n_tables, int stack_cap, int block, int adj_ntab, int hot_n) {
  const size_t tab = (size_t)((n_tables + 3) & ~3);
  const size_t acc = adj_ntab >= 0 ? 2 * (size_t)(((adj_ntab + 4) + 1) & ~1)
                                   : (size_t)hot_words(hot_n);
  const size_t nf = kFields + (adj_ntab >= 0 ? kAdjFields : 0);
  return sizeof(float) * (tab + acc + (size_t)stack_cap * nf * block);
}

namespace {

template <int MODE, int NSC, bool TWO, bool PHASED, bool HEAVY, int DQ = 0>
void launch_one(int grid, int block, size_t lds, hipStream_t stream, const DevPlan* plan,
                const float* tables, const DevBeam& beam, uint64_t seed, uint64_t first,
                uint64_t n, uint64_t per_wave, const dev::Sinks& out, const AdjArgs& AA) {
  hipLaunchKernelGGL((dev::transport<MODE, NSC, TWO, PHASED, HEAVY, DQ>), dim3(grid), dim3(block), lds,
                     stream, plan,
                     tables, beam, seed, first, n, per_wave, out, AA);
}

template <int MODE, bool HEAVY>
void launch_shapes(int nsc, bool two, bool phased, bool dq, int grid, int block, size_t lds,
                   hipStream_t stream, const DevPlan* plan, const float* tables,
                   const DevBeam& beam, uint64_t seed, uint64_t first, uint64_t n,
                   uint64_t per_wave, const dev::Sinks& out, const AdjArgs& AA) {
  // with a detection queue (dq: run and trace modes, tube detectors) or without
#define MCV_LAUNCH(NSC_, TWO_, PH_)                                                            \
  do {                                                                                         \
    if (dq)                                                                                    \
      launch_one<MODE, NSC_, TWO_, PH_, HEAVY, PH_ ? dev::kDqPhased : dev::kDqWalk>(            \
          grid, block, lds, stream, plan, tables, beam, seed, first, n, per_wave, out, AA);    \
    else                                                                                       \
      launch_one<MODE, NSC_, TWO_, PH_, HEAVY>(grid, block, lds, stream, plan, tables, beam,   \
                                               seed, first, n, per_wave, out, AA);             \
  } while (0)
  if (nsc <= 1) {
    if (two) MCV_LAUNCH(1, true, false);
    else if (phased) MCV_LAUNCH(1, false, true);
    else MCV_LAUNCH(1, false, false);
  } else if (nsc == 2) {
    if (two) MCV_LAUNCH(2, true, false);
    else MCV_LAUNCH(2, false, false);
  } else {
    if (two) MCV_LAUNCH(4, true, false);
    else MCV_LAUNCH(4, false, false);
  }
#undef MCV_LAUNCH
}

template <int MODE>
void launch_mode(int nsc, bool two, bool phased, bool dq, bool heavy, int grid, int block,
                 size_t lds, hipStream_t stream, const DevPlan* plan, const float* tables,
                 const DevBeam& beam, uint64_t seed, uint64_t first, uint64_t n,
                 uint64_t per_wave, const dev::Sinks& out, const AdjArgs& AA) {
  if (heavy)
    launch_shapes<MODE, true>(nsc, two, phased, dq, grid, block, lds, stream, plan, tables, beam,
                              seed, first, n, per_wave, out, AA);
  else
    launch_shapes<MODE, false>(nsc, two, phased, dq, grid, block, lds, stream, plan, tables, beam,
                               seed, first, n, per_wave, out, AA);
}

}  // namespace

hipError_t launch_transport(const DevPlan* plan, const DevPlan& host_plan, const float* tables,
                            const DevBeam& beam, uint64_t seed, uint64_t first, uint64_t n,
                            int grid, int block, uint64_t per_wave, double* hist, double* hist_w2,
                            DevRecord* rec, uint64_t cap, unsigned long long* n_out,
                            DevEvent* ev, uint64_t ev_cap, unsigned long long* n_ev,
                            const AdjArgs* adj, float* gstack, const DetArgs* det,
                            const TapeArgs* tape, hipStream_t stream) {
  AdjArgs AA = {};
  AA.dos_s = AA.dos_k = AA.abs_s = AA.sig_s = AA.sig_k = AA.sqe_s = AA.sqe_k = AA.mp_k = -1;
  if (adj) AA = *adj;
  dev::Sinks out = {hist, hist_w2, rec, cap, n_out, ev, ev_cap, n_ev, 0, nullptr, nullptr, gstack,
                    nullptr, nullptr, 0, nullptr, 0, 0, 0};
  if (det) {
    out.dkeys = det->keys;
    out.dvals = det->vals;
    out.det_cap = det->cap;
    out.n_det = det->n;
    out.det_first = det->first;
    out.det_lin_bits = det->lin_bits;
    out.det_id_bits = det->id_bits;
  }
  if (tape) {
    if (!adj) return hipErrorInvalidValue;  // the tape's carry follows a parameter map
    out.tape = tape->words;
    out.tape_cap = tape->cap;
    out.n_tape = tape->n;
  }
  // adjoint partials in LDS only for the re-trace; the tape run keeps the
  // histogram bin cache
  const int adj_lds = adj && !tape ? (adj->sparse_lds ? adj->nb + adj->nc : 0) : kLdsNoAdjoint;
  const int dq_n = transport_dq_entries(host_plan);
  const bool dq = dq_n > 0;
  const size_t qbytes = transport_dq_bytes(block, dq_n, adj != nullptr);
  const int stack_lds = 0;  // the packet stacks live in device memory
  size_t lds = transport_lds_bytes(host_plan.n_tables, stack_lds, block, adj_lds, host_plan.hot_n) +
               qbytes;
  if (ev || det) {
    // room for the event stages: a smaller bin cache, at most the same LDS
    // if the cache can give it
    const size_t stages = sizeof(float) * (size_t)dev::kEvStageWords * (block / 64);
    int hot = host_plan.hot_n;
    size_t need = transport_lds_bytes(host_plan.n_tables, stack_lds, block, kLdsNoAdjoint, hot) +
                  qbytes + stages;
    while (hot > kHotMin && need > lds) {
      hot >>= 1;
      need = transport_lds_bytes(host_plan.n_tables, stack_lds, block, kLdsNoAdjoint, hot) +
             qbytes + stages;
    }
    out.ev_hot_n = hot;
    lds = need;
  }
  if (lds + sizeof(DevPlan) > 160 * 1024) return hipErrorInvalidConfiguration;
  const int nsc = host_plan.nscat;
  const bool two = host_plan.smax > host_plan.nscat;
  const bool phased = dev::use_phased(nsc, two, host_plan.K);
  const bool heavy = host_plan.heavy != 0;
  if (tape) {
    launch_mode<dev::MODE_TAPE>(nsc, two, phased, dq, heavy, grid, block, lds, stream, plan,
                                tables, beam, seed, first, n, per_wave, out, AA);
  } else if (adj) {
    launch_mode<dev::MODE_ADJOINT>(nsc, two, phased, dq, heavy, grid, block, lds, stream, plan,
                                   tables, beam, seed, first, n, per_wave, out, AA);
  } else if (rec) {
    launch_mode<dev::MODE_TRACE>(nsc, two, phased, dq, heavy, grid, block, lds, stream, plan,
                                 tables, beam, seed, first, n, per_wave, out, AA);
  } else {
    launch_mode<dev::MODE_RUN>(nsc, two, phased, dq, heavy, grid, block, lds, stream, plan,
                               tables, beam, seed, first, n, per_wave, out, AA);
  }
  return hipGetLastError();
}

// zero_ptrs, zero_sizes: host arrays (device pointers and lengths of the
// histograms to zero); the fills and the cursor reset are kernels, so the
// whole sequence can be captured in a graph without memset nodes
hipError_t launch_batch(const BatchItem* items, const BatchChunk* chunks, uint32_t n_chunks,
                        uint32_t* cursor, double* const* zero_ptrs, const uint64_t* zero_sizes,
                        int n_zero, int grid, int block, size_t lds, int hot_n, int dq_off,
                        float* gstack, int stack_max, bool heavy, hipStream_t stream) {
  hipLaunchKernelGGL(dev::batch_cursor_reset, dim3(1), dim3(64), 0, stream, cursor);
  for (int k = 0; k < n_zero; ++k) {
    uint64_t g = (zero_sizes[k] / 2 + 255) / 256;
    if (g > ((uint64_t)1 << 30)) g = (uint64_t)1 << 30;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(dev::fill_zero, dim3((unsigned)g), dim3(256), 0, stream, zero_ptrs[k],
                       zero_sizes[k]);
  }
  if (heavy)
    hipLaunchKernelGGL(dev::batch_persistent<true>, dim3(grid), dim3(block), lds, stream, items,
                       chunks, n_chunks, cursor, hot_n, dq_off, gstack, stack_max);
  else
    hipLaunchKernelGGL(dev::batch_persistent<false>, dim3(grid), dim3(block), lds, stream, items,
                       chunks, n_chunks, cursor, hot_n, dq_off, gstack, stack_max);
  return hipGetLastError();
}

hipError_t launch_fill_zero(double* p, uint64_t n, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(dev::fill_zero, dim3(grid), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

int batch_occupancy(int block, size_t lds, bool heavy) {
  int nb = 0;
  const hipError_t e =
      heavy ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, dev::batch_persistent<true>, block,
                                                           lds)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, dev::batch_persistent<false>, block,
                                                           lds);
  return e == hipSuccess ? nb : 0;
}

hipError_t launch_loss_grad(const double* I, const double* T, const double* w, int64_t n,
                            double* dLdI, double* loss, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(dev::loss_grad, dim3(grid), dim3(256), 0, stream, I, T, w, n, dLdI, loss);
  return hipGetLastError();
}

size_t transport_static_lds() { return sizeof(DevPlan); }

// resident waves per SIMD the transport kernels are compiled for
int transport_waves_per_eu(int, int) { return MCV_WAVES_PER_EU; }
int batch_waves_per_eu() { return MCV_BATCH_WAVES_PER_EU; }

namespace {
template <int MODE, bool HV, int QP, int QW>
void push_shapes_q(std::vector<const void*>& v) {
  v.push_back(reinterpret_cast<const void*>(&dev::transport<MODE, 1, false, false, HV, QW>));
  v.push_back(reinterpret_cast<const void*>(&dev::transport<MODE, 1, false, true, HV, QP>));
  v.push_back(reinterpret_cast<const void*>(&dev::transport<MODE, 1, true, false, HV, QW>));
  v.push_back(reinterpret_cast<const void*>(&dev::transport<MODE, 2, false, false, HV, QW>));
  v.push_back(reinterpret_cast<const void*>(&dev::transport<MODE, 2, true, false, HV, QW>));
  v.push_back(reinterpret_cast<const void*>(&dev::transport<MODE, 4, false, false, HV, QW>));
  v.push_back(reinterpret_cast<const void*>(&dev::transport<MODE, 4, true, false, HV, QW>));
}
template <int MODE, bool HV>
void push_shapes(std::vector<const void*>& v) {
  push_shapes_q<MODE, HV, 0, 0>(v);
  push_shapes_q<MODE, HV, dev::kDqPhased, dev::kDqWalk>(v);
}
template <int MODE>
void push_mode(std::vector<const void*>& v) {
  push_shapes<MODE, false>(v);
  push_shapes<MODE, true>(v);
}
}  // namespace

hipError_t set_transport_lds_limit(size_t bytes) {
  std::vector<const void*> fns;
  push_mode<dev::MODE_RUN>(fns);
  push_mode<dev::MODE_TRACE>(fns);
  push_mode<dev::MODE_ADJOINT>(fns);
  push_mode<dev::MODE_TAPE>(fns);
  fns.push_back(reinterpret_cast<const void*>(&dev::batch_persistent<false>));
  fns.push_back(reinterpret_cast<const void*>(&dev::batch_persistent<true>));
  // each kernel may use `bytes` of LDS in total, static part included
  for (const void* f : fns) {
    hipFuncAttributes at;
    hipError_t e = hipFuncGetAttributes(&at, f);
    if (e != hipSuccess) return e;
    const size_t dyn = bytes > at.sharedSizeBytes ? bytes - at.sharedSizeBytes : 0;
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mcv
