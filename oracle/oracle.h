/*
 * Reference (oracle) implementation of the per-ray mosaic-crystal transport
 * of Gawne et al., "HEART: A New X-Ray Tracing Code for Mosaic Crystal
 * Spectrometers" (arXiv 2503.16955).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, scalar FP64 CPU program
 * that exists to check the GPU library.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the GPU library; the two agree only
 * because both follow the same written model:
 *
 *   source (paper sec. 2.1) -> crystal entry (sec. 2.2, FlatCrystal /
 *   CylinderCrystal) -> null-collision depth stepping under Beer-Lambert
 *   absorption (sec. 2.2.3, Eq. AnyEvent and the absorb-or-reflect rule)
 *   -> crystallite tilt drawn from the mosaic distribution (sec. 2.2.2,
 *   Eqs. vMF/MF, SWL, WL) -> deviation from the Bragg angle (Eq. BraggLaw)
 *   -> acceptance by the intrinsic rocking curve (sec. 2.2.1, pseudo-Voigt,
 *   Eqs. Gaussian and Lorentz) -> specular reflection off the crystallite
 *   (sec. 2.2.4, reflection equation) -> pixel detector (sec. 2.3).
 *
 * Units: lengths mm, angles rad, energies keV, lattice spacing Angstrom,
 * attenuation 1/mm.  All arithmetic is IEEE double with glibc libm.
 */
#ifndef MOSAIC_ORACLE_H
#define MOSAIC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_SPEC_UNIFORM = 0, ORC_SPEC_LINES = 1, ORC_SPEC_TABLE = 2 };
enum { ORC_GEOM_FLAT = 0, ORC_GEOM_CYLINDER = 1 };
enum { ORC_MDF_VMF = 0, ORC_MDF_LORENTZ = 1, ORC_MDF_PVOIGT = 2,
       ORC_MDF_WRAPPED_LORENTZ = 3, ORC_MDF_SPHERICAL_WRAPPED_LORENTZ = 4,
       ORC_MDF_GAUSSIAN = 5 };
enum { ORC_IRC_GAUSS = 0, ORC_IRC_PVOIGT = 1, ORC_IRC_TABLE = 2,
       ORC_IRC_LORENTZ = 3, ORC_IRC_BOX = 4 };
enum { ORC_MODEL_STEPPING = 0, ORC_MODEL_MWG = 1 };
enum { ORC_SPOT_POINT = 0, ORC_SPOT_GAUSSIAN = 1, ORC_SPOT_DISK = 2 };
enum { ORC_MISS = 0, ORC_ABSORBED = 1, ORC_EXIT_REFLECTED = 2,
       ORC_EXIT_TRANSMITTED = 3, ORC_TRUNCATED = 4 };

typedef struct orc_source {
    double origin[3];
    double axis[3];          /* cone axis (unit) */
    double b1[3];            /* unit, orthogonal to axis; b2 = axis x b1 */
    double half_angle;       /* cone half-angle */
    int32_t spectrum;        /* ORC_SPEC_* */
    int32_t n_lines;         /* <= 8 */
    double e_min, e_max;     /* flat part / table range */
    double line_e[8], line_sigma[8], line_w[8];
    double background_w;
    int32_t n_bins;          /* table spectrum */
    int32_t spot_kind;       /* ORC_SPOT_*: the source spot (sec. 4.2) */
    const double *bin_w;     /* n_bins weights (host) */
    /* spot plane (orthonormal) and size: Gaussian standard deviations
       along u and v, or the disk radius in spot_sigma[0] */
    double spot_u[3], spot_v[3], spot_sigma[2];
    /* user ray arrays (sec. 2.1), host, row ray_id - user_first, or NULL:
       origins (x, y, z), unit directions, energies; each replaces the
       sampled field (user origins also replace the spot) */
    const double *user_o, *user_k, *user_e;
    uint64_t user_first;
    /* user polarisations (sec. 2.1), host, same rows, or NULL: when given,
       polarisation is tracked through the reflections */
    const double *user_p;
} orc_source;

/* Reflecting planes beyond the main set (sec. 2.2.3, closing paragraphs):
   the antiparallel planes' strength relative to H, and up to three further
   plane sets (higher orders) with their own spacing, peak strength
   relative to the main curve, width scale and shift of the curve. */
typedef struct orc_planes {
    double hbar_ratio;
    int32_t n_extra;
    int32_t pad_;
    double two_d[3], strength[3], width_scale[3], shift[3];
} orc_planes;

typedef struct orc_crystal {
    int32_t geometry;        /* ORC_GEOM_* */
    int32_t max_refl;
    /* flat: surface centre, outward normal, length axis */
    double centre[3], normal[3], e1[3];
    /* cylinder: point on axis, axis direction, azimuth reference (phi = 0) */
    double axis_pt[3], axis_dir[3], ref_dir[3];
    double radius, phi_c, z_c;
    /* shared extents: length (along e1 / axis), width (along e2 / arc
       length at the front radius), thickness */
    double length, width, thickness;
    double two_d;            /* Angstrom */
    double mu0;              /* linear attenuation, 1/mm */
    double mfp;              /* mean path between crystallite encounters, mm */
    const orc_planes *planes;  /* NULL: the main set alone, H and H-bar alike */
} orc_crystal;

typedef struct orc_mosaic {
    int32_t kind;            /* ORC_MDF_* */
    int32_t pad_;
    double fwhm;             /* Gamma */
    double eta;              /* Lorentzian fraction for ORC_MDF_PVOIGT */
} orc_mosaic;

typedef struct orc_irc {
    int32_t kind;            /* ORC_IRC_* */
    int32_t n_table;
    double peak;             /* reflection probability at the curve maximum */
    double shift;            /* Delta_M */
    double fwhm;             /* Lambda (Gaussian, Lorentzian, box) */
    double fwhm_g, fwhm_l;   /* pseudo-Voigt components */
    double x_min, x_max;     /* table range */
    const double *table;     /* n_table values (host) */
    /* n_dep > 0: the curve of a photon of energy E is r((Delta -
       Delta_M(E)) / s(E)), Delta_M and s interpolated linearly (end values
       held) from (dep_kev, dep_shift) and (dep_kev, dep_scale) */
    int32_t n_dep, pad_;
    const double *dep_kev, *dep_shift, *dep_scale;
} orc_irc;

/* n_qe > 0: quantum efficiency table (energies strictly increasing, keV);
   a detected photon adds rint(E QE(E) 1e6) to the energy image. */
typedef struct orc_detector {
    double centre[3], normal[3], u[3], v[3];
    int32_t nx, ny;
    double pitch;
    int32_t n_qe, pad_;
    const double *qe_kev, *qe;
} orc_detector;

/* One record per ray (104 bytes). */
/* Event model.  STEPPING: null-collision stepping with per-encounter
   acceptance.  MWG: the paper's model (sec. 2.2.3-2.2.4): free paths at
   mu0 + gamma0 sigma(alpha), sigma by the psi quadrature of Eq.
   SimpleReflXsection on psi_nodes intervals, reflections with (psi, Delta)
   from burn_in Metropolis-within-Gibbs sweeps. */
typedef struct orc_model {
    int32_t kind;            /* ORC_MODEL_* */
    int32_t burn_in;
    int32_t psi_nodes;
    int32_t irc_off;         /* 1: the IRC disabled, every reflection at Delta_M */
} orc_model;

typedef struct orc_record {
    uint64_t ray_id;
    double energy;
    double entry[3];
    double end[3];
    double dir[3];
    int32_t pix_i, pix_j;
    uint32_t n_events;
    uint16_t n_refl;
    uint8_t status;
    uint8_t detected;
} orc_record;

typedef struct orc_counters {
    uint64_t emitted, missed, absorbed, exit_reflected, exit_transmitted,
             truncated, detected, events, reflections;
} orc_counters;

/* Philox4x32-10 and Philox4x64-10 (Salmon et al., SC'11). */
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Bragg angle (Eq. BraggLaw); returns -1 when hc/E exceeds 2d. */
double orc_bragg_angle(double energy_kev, double two_d);

/* Pseudo-Voigt total width and Lorentzian fraction from the component
   widths (sec. 2.2.1). */
void orc_pvoigt_params(double fwhm_g, double fwhm_l, double *fwhm, double *eta);

/* Rocking-curve reflection probability r(x) at x = Delta - Delta_M. */
double orc_irc_value(const orc_irc *irc, double x);

/* Draw a crystallite normal about frame (N, e1, e2) from uniforms (u2, u3). */
void orc_mdf_sample(const orc_mosaic *m, double u2, double u3,
                    const double N[3], const double e1[3], const double e2[3],
                    double n_out[3]);

/* Source sample for one ray: origin, direction, energy. */
void orc_source_sample(const orc_source *s, uint64_t seed, uint64_t ray_id,
                       double o[3], double k[3], double *energy);

/* Exit distance of a point inside the crystal moving along k. */
double orc_exit_distance(const orc_crystal *c, const double p[3], const double k[3]);

/* Pieces of the paper's event model, for unit pins.  orc_mdf_density: the
   mosaic density per steradian at v = 1 - cos(theta).  orc_psi_integral: the
   psi integral of Eq. SimpleReflXsection on M intervals.  orc_irc_integral:
   int r(x) dx.  orc_irc_width: the sampler's Delta step.  orc_mwg_sample:
   one sampler draw (margin may be NULL).  orc_crystallite: the normal at
   (alpha, b = alpha_B + Delta, psi) about planes of normal N. */
double orc_mdf_density(const orc_mosaic *m, double v);
double orc_psi_integral(const orc_mosaic *m, double alpha, double beta, int M);
double orc_irc_integral(const orc_irc *irc);
double orc_irc_width(const orc_irc *irc);
void orc_mwg_sample(const orc_mosaic *m, const orc_irc *irc, double w_psi, double w_delta,
                    uint64_t seed, uint64_t ray, uint32_t event, int burn_in,
                    double alpha, double ab, double *psi_out, double *delta_out,
                    double *margin);
/* The same with Delta held at Delta_M (the IRC disabled, sec. 2.2.1): the
   sweeps make psi moves only. */
void orc_mwg_sample_psi(const orc_mosaic *m, const orc_irc *irc, double w_psi,
                        uint64_t seed, uint64_t ray, uint32_t event, int burn_in,
                        double alpha, double ab, double *psi_out, double *delta_out,
                        double *margin);
void orc_crystallite(const double N[3], const double k[3], double alpha, double b,
                     double psi, double n[3]);

/* Trace rays [first, first + n).  counts / energy_mev / records / counters /
   margins may each be NULL.  Images are accumulated into (not cleared).
   records and margins are indexed by ray_id - first.  margins[i] is the
   smallest decision margin met by ray i (a diagnostic for tie analysis).
   n_threads <= 0 uses every online core.  Returns 0 or a negative error. */
int orc_trace_model(const orc_source *s, const orc_crystal *c, const orc_mosaic *m,
                    const orc_irc *irc, const orc_detector *d, const orc_model *model,
                    uint64_t first, uint64_t n, uint64_t seed, uint32_t max_events,
                    uint32_t *counts, uint64_t *energy_mev,
                    orc_record *records, orc_counters *counters, double *margins,
                    int n_threads);
int orc_trace_ids_model(const orc_source *s, const orc_crystal *c, const orc_mosaic *m,
                        const orc_irc *irc, const orc_detector *d, const orc_model *model,
                        const uint64_t *ids, uint64_t n, uint64_t seed, uint32_t max_events,
                        orc_record *records, double *margins, int n_threads);
int orc_trace(const orc_source *s, const orc_crystal *c, const orc_mosaic *m,
              const orc_irc *irc, const orc_detector *d,
              uint64_t first, uint64_t n, uint64_t seed, uint32_t max_events,
              uint32_t *counts, uint64_t *energy_mev,
              orc_record *records, orc_counters *counters, double *margins,
              int n_threads);

/* Trace an arbitrary list of ray ids (no images); records[i], margins[i]
   belong to ids[i]. */
int orc_trace_ids(const orc_source *s, const orc_crystal *c, const orc_mosaic *m,
                  const orc_irc *irc, const orc_detector *d,
                  const uint64_t *ids, uint64_t n, uint64_t seed, uint32_t max_events,
                  orc_record *records, double *margins, int n_threads);

/* The polarisation factor G = 1 - (p.k_s)^2 and the polarisation after a
   reflection into k_s (sec. 2.2.3, 2.2.4). */
double orc_polarisation_reflect(const double p[3], const double ks[3], double out[3]);

/* The paper's model with polarisation (sec. 2.2.3): the angle phi of p
   about k for planes of normal N at glancing angle alpha, the psi integral
   of Eq. SimpleReflXsectionPol, and the sampler with target the integrand
   of Eq. ReflXsectionPol. */
double orc_polarisation_angle(const double p[3], const double N[3], const double k[3],
                              double alpha);
double orc_psi_integral_pol(const orc_mosaic *m, double alpha, double beta, double phi, int M);
void orc_mwg_sample_pol(const orc_mosaic *m, const orc_irc *irc, double w_psi, double w_delta,
                        uint64_t seed, uint64_t ray, uint32_t event, int burn_in,
                        double alpha, double ab, double phi, double *psi_out, double *delta_out,
                        double *margin);

int orc_version(void);

#ifdef __cplusplus
}
#endif
#endif
