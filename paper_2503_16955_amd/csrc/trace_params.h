// Launch parameters of the trace kernels, prepared on the host from the
// public structs.  All geometry is expressed in a crystal-local frame: its
// origin is the flat crystal's front-face centre, or the point of the
// cylinder axis at z_c, which keeps coordinates small so that the FP32 path
// keeps nanometre resolution inside the crystal; its axes are the flat
// crystal's (e1, e2, normal), or (ref_dir, axis x ref_dir, axis) for the
// cylinder, so the kernels use those directions as the coordinate axes.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "mosaicrt.h"

namespace mrt {

constexpr int kMaxLines = 8;
// Largest tables (rocking-curve values plus spectrum CDF), kept small enough
// to stay cache-resident while the kernels read them.
constexpr int kMaxTableBytes = 64 * 1024;
// The library's own tables: the user's (at most kMaxTableBytes) plus the
// table curve's envelope, one word per bucket of at least 8 nodes.
constexpr int kMaxStagedTableBytes = kMaxTableBytes + kMaxTableBytes / 8;

// Parameters the FP32-mixed kernels use in FP32 arithmetic.  The host keeps an
// FP32 copy of each (rounded to nearest, as a device conversion would round
// it), so those kernels read them ready for use instead of converting them
// from FP64 inside the ray loop or holding converted copies in registers.
#define MRT_F32_SCALARS(X)                                                                    \
    X(vmax) X(hl) X(hw) X(T) X(R2) X(Ro2) X(inv_mu0) X(inv_mu_tot) X(p_a) X(inv_1mpa)          \
    X(m_eta) X(inv_eta) X(inv_1meta) X(vmf_s2) X(vmf_floor) X(lor_g) X(wl_half_g2) X(wl_z)     \
    X(swl_k) X(swl_d) X(gau_2s2) X(shift) X(g_k) X(g_k_log2e) X(pv_a) X(pv_b) X(pv_h2)         \
    X(lor_h2)                                                                                  \
    X(box_half) X(lut_x0) X(lut_x1) X(lut_scale) X(pitch) X(half_nx) X(half_ny)
#define MRT_F32_VECTORS(X) \
    X(so) X(sa) X(sb1) X(sb2) X(op) X(om) X(dP) X(dn) X(du) X(dv)

struct TraceParamsF32 {
#define MRT_F32_S(n) float n;
#define MRT_F32_V(n) float n[3];
    MRT_F32_SCALARS(MRT_F32_S)
    MRT_F32_VECTORS(MRT_F32_V)
#undef MRT_F32_S
#undef MRT_F32_V
};

struct TraceParams {
    // ---- source (sec. 2.1), local coordinates
    double so[3];                 // source origin
    double sa[3], sb1[3], sb2[3]; // cone axis and azimuth frame
    double vmax;                  // 1 - cos(half_angle), as 2 sin^2(half_angle / 2)
    int32_t spectrum, n_lines;
    double e_min, e_span;         // e_span = e_max - e_min
    double line_e[kMaxLines], line_sig[kMaxLines];
    double line_cum[kMaxLines];   // running weight sums / total, lines in order
    int32_t n_bins, pad0;
    const double *bin_cdf;        // n_bins + 1 normalised prefix sums (device)
    int32_t spot_kind, pad_s;     // finite source spot (MRT_SPOT_*)
    double spot_u[3], spot_v[3], spot_sigma[2];
    const double *user_o, *user_k, *user_e;   // user ray arrays (device) or NULL
    const double *user_p;         // user polarisations (device) or NULL

    // ---- crystal (sec. 2.2), in the local frame: flat normal z, length
    // axis x, width axis y; cylinder axis z through the local origin
    int32_t geometry, max_refl;
    double hl, hw, T;             // half length, half width, thickness
    double op[3], om[3];          // outward normals of the two azimuth edges (z = 0)
    double R, R2, Ro2;            // front radius, R^2, (R + T)^2
    double mu0, inv_mu0, inv_mu_tot, p_a, inv_1mpa;
    double two_d;                 // lattice spacing 2d (Angstrom)
    // reflecting planes (extended-input kernels): set 0 is the main set
    int32_t has_planes, n_planes;
    double plane_2d[4], plane_a[4], plane_scale[4], plane_shift[4], plane_inv_scale[4];
    double plane_ratio[4];        // 2d / 2d_j
    double hbar, plane_tot;       // H-bar / H ratio; sum_j a_j max(1, hbar)
    double origin[3];             // local origin in global coordinates
    double rot[3][3];             // rows: the local axes in global coordinates

    // ---- mosaic (sec. 2.2.2)
    int32_t mdf, pad1;
    double fwhm;
    double m_eta, inv_eta, inv_1meta;
    double vmf_s2, vmf_floor;     // s^2 and exp(-2 / s^2)
    double lor_g;                 // Gamma / 2
    double wl_half_g2, wl_z;      // g^2 / 2 and ln((g^2 + 4) / g^2)
    double swl_k, swl_d;          // 4 sinh^2(Gamma / 4) and cosh(Gamma / 2) + 1
    double gau_2s2;               // 2 s^2, s = Gamma / (2 sqrt(2 ln 2)): the Gaussian tilt

    // ---- rocking curve (sec. 2.2.1), all as r(x) / R_max
    int32_t irc, lut_n;
    double shift;
    double g_k;                   // 4 ln 2 / Lambda^2
    double g_k_log2e;             // g_k / ln 2, for exp2 in the FP32 filter
    double pv_a, pv_b, pv_h2;     // A h^2 / (h^2 + x^2) + B exp(-g_k x^2)
    double lor_h2, box_half;
    double lut_x0, lut_x1, lut_scale, lut_inv_max;
    const double *lut;            // device
    // the table's envelope: (min, max) of each bucket of 2^env_shift nodes,
    // at index env_at of the tables (device pointer lut_env)
    int32_t env_at, env_shift;
    const double *lut_env;
    int32_t dep_n, dep_at;        // energy-dependence nodes; their index in the tables
    const double *dep;            // dep_n energies, shifts, width scales (device)

    // ---- the paper's event model (sec. 2.2.3, 2.2.4; FP64 kernels only)
    int32_t burn_in, psi_nodes;   // sampler sweeps; psi quadrature intervals
    int32_t mwg_batch, irc_off;   // parked lanes that start the sampler; IRC disabled
    double q;                     // int r dx / mfp (Q R = r / mfp)
    double w_delta;               // sampler step in Delta
    double vmf_kappa, vmf_norm;   // density kappa e^{-kappa v} / (2 pi (1 - e^{-2 kappa}))
    double cau_g2, cau_norm;      // (Gamma/2)^2 and (Gamma/2) / (2 pi)
    double wl_g2, wl_norm;        // (Gamma/2)^2 and 1 / (pi ln((g^2 + 4) / g^2))
    double swl_a, swl_norm;       // 2 sinh^2(Gamma/4) and A (A + 2) / (4 pi)
    double gau_inv2s2, gau_norm;  // 1 / (2 s^2) and 1 / (2 pi s^2)
    const double *psi_tab;        // (sin^2(psi_j / 2), trapezoid weight w_j), j = 0..M (device)
    const double *psi_cos2;       // w_j cos(2 psi_j), j = 0..M (device; after psi_tab)

    // ---- detector (sec. 2.3), local coordinates
    double dP[3], dn[3], du[3], dv[3];
    int32_t nx, ny;
    double pitch, half_nx, half_ny;
    int32_t qe_n, qe_at;          // quantum-efficiency nodes; their index in the tables
    const double *qe;             // qe_n energies (keV), then qe_n values (device)

    // ---- run
    uint64_t first, n, seed;
    uint32_t key0, key1;          // Philox key: seed low and high words
    uint32_t max_events;
    uint32_t chunk;               // ray ids a wave claims at a time
    uint32_t refill_idle;         // refill a wave once this many lanes are idle
    int32_t records_mode;
    uint32_t exact;               // every acceptance decision in FP64 (extended kernels)
    uint32_t pad_run;
    uint64_t rec_cap;
    uint32_t *counts;
    unsigned long long *energy;
    mrt_hit_record *records;
    unsigned long long *dev_counters;   // kNumCounters entries
    unsigned long long *chunk_counter;  // next unclaimed ray offset

    TraceParamsF32 f32;           // FP32 copies (see above)
};

// Device counter slots.
enum {
    kCMissed = 0, kCAbsorbed, kCExitReflected, kCExitTransmitted, kCTruncated, kCDetected,
    kCEvents, kCReflections, kCRecords, kCRefined, kNumCounters
};

// One request's share of a serving round: rays [first, first + count) of the
// request whose parameter block is slots[slot], handed to waves `chunk` rays
// at a time.  `start` is the sum of the counts of the items before it (waves
// pick their first item by it, so each item starts with a share of the waves
// proportional to its rays).
struct ServeItem {
    uint64_t first;
    uint64_t count;
    uint64_t start;
    int32_t slot;
    uint32_t chunk;
};

// Kernel of a precision / geometry / mosaic / rocking-curve / records
// combination (nullptr for an unknown kind).
const void *trace_kernel_ptr(int precision, int geometry, int mdf, int irc, bool records);
int launch_zero(void *ptr_u32, size_t n_words, void *stream);
int launch_calibration_map(const uint32_t *counts, const uint64_t *energy, size_t n, double *map,
                           void *stream);
constexpr int kMaxQeNodes = 1024;
// Serving kernel of a precision (ext: the instance with the extended
// inputs): (const TraceParams *slots, const ServeItem *items, uint32_t
// n_items, uint64_t total, unsigned long long *cursors), one zeroed cursor
// per item.
const void *serve_kernel_ptr(int precision, bool ext);
// Kernel of the paper's event model (FP64) for a geometry (nullptr for an
// unknown one): (TraceParams), like the trace kernels.
const void *mwg_kernel_ptr(int geometry, bool records, bool polarised, bool planes);
// Kernel for the extended inputs (an energy-dependent rocking curve,
// polarisations, further plane sets) of a precision / geometry / mosaic /
// rocking-curve / records combination (nullptr for an unknown kind).
const void *ext_kernel_ptr(int precision, int geometry, int mdf, int irc, bool records);
constexpr int kMaxPsiNodes = 2048;

}  // namespace mrt
