/* hlc.h -- C ABI of the MI355X (gfx950) positional cross-match library.
 *
 * The operation (paper, section 2.1): given two catalogues A and B of sky
 * positions (right ascension, declination, both in degrees) and a radius r,
 * report every pair (i, j) whose great-circle separation (the angle of
 * eq. (1)) is at most r. The comparison is inclusive, as in eq. (4), and all
 * pairs are reported, not only the nearest one (section 4.3.2 keeps a result
 * for every catalogue pair). The paper's eq. (4) threshold 3*sqrt(r1^2+r2^2)
 * is passed as r by the caller.
 *
 * Semantics shared by every entry point
 *   - Inputs are FP64 degrees read as exact reals: RA in [0, 360] (360 is the
 *     same point as 0), Dec in [-90, 90], finite. Anything else is rejected
 *     with HLC_E_INVAL (detected on the device; the output buffers and the
 *     pair count are then unspecified).
 *   - The result is a set: pair order is unspecified. Each pair carries the
 *     indices into the caller's ORIGINAL arrays and, unless HLC_NO_SEP is
 *     set, the separation in arcsec as FP64 (within 1e-9 arcsec of the exact
 *     value).
 *   - The pair set is exact: a pair is reported iff its exact separation is
 *     <= r_arcsec/3600 degrees, where pairs within a relative 1e-28 of r
 *     (indistinguishable at double-double precision) count as matches.
 *   - r_arcsec must lie in (0, 3600]; 0 <= na, nb <= 2^31 - 2^16 (B's
 *     entries, halo copies included, then stay below 2^32).
 *   - A and B may be the same arrays; they are still two catalogues, so
 *     (i, i) is reported with separation 0, unless HLC_SELF is set.
 *
 * Memory and ownership
 *   - Coordinate and output pointers are DEVICE pointers (hipMalloc'd, or a
 *     torch tensor's data_ptr()) unless a name says _host.
 *   - The caller owns all input and output buffers; the library never keeps
 *     a caller pointer after a call returns.
 *   - The library owns a per-device workspace, grown on demand and released
 *     by hlc_shutdown(), and every hlc_part it hands out.
 *   - A call on a device sizes its staging buffers, and (FP32) chooses how
 *     it lays out B's coordinates for the certification, from what earlier
 *     calls on that device counted; results never depend on this, only the
 *     time does.
 *
 * Errors: every int-returning call returns HLC_OK (0) or a negative
 * hlc_status; no C++ exception crosses this boundary. HIP runtime failures
 * map to HLC_E_DEVICE. Calls are synchronous on opts->stream (they return
 * once the pair count is known) and are not thread-safe with each other.
 */
#ifndef HLC_H_
#define HLC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HLC_OK = 0,
  HLC_E_INVAL = -1,       /* bad argument or coordinate                           */
  HLC_E_NOMEM = -2,       /* device or host allocation failed                     */
  HLC_E_OVERFLOW = -3,    /* more pairs than opts->capacity; *n_pairs = required  */
  HLC_E_DEVICE = -4,      /* HIP runtime error                                    */
  HLC_E_UNSUPPORTED = -5  /* valid request the library does not handle            */
} hlc_status;

/* Filter precision. Both give the same exact pair set; they differ in speed.
 *   HLC_FP32_RECHECK: candidate filter in FP32 on offsets from a centre per
 *     group of 16 A sources (each unit vector stored as its FP32 lattice
 *     corner plus a fixed-point offset of 2^-34 per axis), against a bound
 *     that covers every FP32 rounding; every candidate is then certified in
 *     FP64 (default). The batched form's FP32 filter works on offsets from
 *     each job's frame centre.
 *   HLC_FP64: candidate filter in FP64 on unit vectors.                     */
typedef enum { HLC_FP32_RECHECK = 0, HLC_FP64 = 1 } hlc_precision;

/* Output record: indices into the caller's original A and B arrays. */
typedef struct {
  uint32_t a, b;
} hlc_pair;

/* opts->flags */
#define HLC_NO_SEP 0x1u   /* do not write separations (out_sep may be NULL)    */
#define HLC_PROFILE 0x2u  /* time each stage with HIP events (hlc_last_stats)  */
#define HLC_SORTED 0x4u   /* pairs (and separations) ordered by (a, b); not   *
                           * with hlc_xmatch_stream (HLC_E_UNSUPPORTED)       */
#define HLC_TIME_FILTER 0x10u /* time the filter kernel alone with two HIP   *
                           * events on its stream (hlc_last_stats           *
                           * t_match_ms); much lighter than HLC_PROFILE     */
#define HLC_SELF 0x8u     /* self-match: B is the same arrays as A; each       *
                           * unordered pair is reported once as (i, j), i < j, *
                           * and (i, i) never (the self-match data sets of     *
                           * section 5, Table 2). One partition serves both.   */

/* Optional fixed tuning; zero fields mean "choose automatically". */
typedef struct hlc_tuning {
  double zone_height_arcsec; /* Dec zone height (within 1 deg of a pole the    *
                              * zones are min(this, ~16 r) high); >= 2.0001 r *
                              * is enforced                                    */
  int32_t ra_bins_log2;      /* log2 of RA bins per zone, 1..30 (0 = auto)     */
  int32_t filter_items;       /* work items (four groups of 16 A) per wave of   *
                              * the filter kernel (0 = one)                    */
  double zone_height_factor; /* batched form: scale of each job's density-     *
                              * derived zone height (0 = autotuned and cached)  */
  int32_t fraction_sort;     /* hlc_xmatch, hlc_xmatch_radii: 1 = the          *
                              * partition also sorts the RA sub-bin bits (one  *
                              * more radix pass; narrower windows inside dense *
                              * clumps); 0 = not                               */
  int32_t batch_tile;        /* batched form: sources per partition tile (256, *
                              * 512, 1024 or 2048; 0 = autotuned and cached)   */
  int32_t batch_blocks_per_cu; /* batched form: blocks of the persistent match *
                              * per compute unit (1..8; 0 = autotuned, cached) */
  int32_t reserved[1];
} hlc_tuning;

typedef struct hlc_opts {
  hlc_precision precision;
  void *stream;              /* hipStream_t; NULL = the null stream            */
  int64_t capacity;          /* length of out_pairs / out_sep, in pairs        */
  int64_t *n_pairs;          /* host pointer; out: pairs found (or required)  */
  uint32_t flags;            /* HLC_NO_SEP | HLC_PROFILE | HLC_SELF            */
  const hlc_tuning *tuning;  /* NULL = automatic                               */
} hlc_opts;

/* Statistics of the last call made on the calling thread (each thread keeps *
 * its own record).                                                         */
typedef struct hlc_stats {
  int64_t na, nb;            /* catalogue sizes                               */
  int64_t nb_halo;           /* B entries after Dec-halo duplication          */
  int64_t n_pairs;           /* pairs in the result                            */
  int64_t n_candidates;      /* filter survivors sent to certification        */
  int64_t n_band;            /* candidates re-evaluated from (ra, dec) in FP64 */
  int64_t n_ties;            /* candidates decided in double-double            */
  int32_t n_zones;           /* Dec zones                                      */
  int32_t ra_bits;           /* RA bins = 2^ra_bits                            */
  double zone_height_arcsec;
  /* stage times in milliseconds (HLC_PROFILE only, else 0): t_match_ms is
   * the filter kernel alone; t_certify_ms the candidate certification, the
   * band list and the packing of the output */
  double t_keygen_ms, t_sort_ms, t_layout_ms, t_ranges_ms, t_match_ms, t_certify_ms, t_total_ms;
  /* batched form: the partition tile and the match blocks per compute unit
   * used (zone_height_arcsec then holds the zone-height factor used)       */
  double batch_tile, batch_blocks_per_cu;
  double reserved[6];
} hlc_stats;

/* Cross-match A against B at radius r_arcsec (the paper's section 3.1 kernel
 * module and section 4.2 two-level partition, redesigned for one GPU).
 *   a_ra, a_dec [na], b_ra, b_dec [nb]: device FP64 degrees.
 *   out_pairs [opts->capacity]: device; out_sep [opts->capacity]: device FP64
 *     arcsec, or NULL with HLC_NO_SEP.
 *   *opts->n_pairs receives the pair count. If it exceeds opts->capacity the
 *     call returns HLC_E_OVERFLOW, *n_pairs holds the exact required count
 *     and the buffers' contents are unspecified.
 *   opts may be NULL only when capacity is irrelevant: it is required.       */
int hlc_xmatch(const double *a_ra, const double *a_dec, int64_t na, const double *b_ra,
               const double *b_dec, int64_t nb, double r_arcsec, hlc_pair *out_pairs,
               double *out_sep_arcsec, const hlc_opts *opts);

/* hlc_xmatch for callers that cannot allocate: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. The same pair set and
 * separations as hlc_xmatch, from the same kernels, but the call's workspace
 * and device counters lie in a fixed device array of the library (128 MiB on
 * each device it runs on, held from the library's load until the process
 * ends), so the call allocates nothing (no hipMalloc, hipFree, hipHostMalloc,
 * no stream or event creation). Every kernel runs on opts->stream; the call
 * returns once the pair count is known. Limits: a call whose workspace would
 * not fit the array (roughly beyond 500,000 sources per catalogue, fewer when
 * the pairs or near-threshold candidates are many) returns HLC_E_UNSUPPORTED,
 * as do HLC_SELF, HLC_SORTED, HLC_PROFILE and HLC_TIME_FILTER. Every call on one device
 * shares that device's array and leaves its contents behind: calls that
 * overlap on one device (two host threads, or two streams) race and must be
 * serialised by the caller. Arguments, outputs and other errors as
 * hlc_xmatch.                                                              */
int hlc_xmatch_noalloc(const double *a_ra, const double *a_dec, int64_t na, const double *b_ra,
                       const double *b_dec, int64_t nb, double r_arcsec, hlc_pair *out_pairs,
                       double *out_sep_arcsec, const hlc_opts *opts);

/* Eq. (4) with per-source error radii: report (i, j) iff the separation is
 * at most k_sigma * sqrt(a_err[i]^2 + b_err[j]^2) arcsec (the paper uses
 * k_sigma = 3). a_err [na], b_err [nb]: device FP64 arcsec, finite, >= 0.
 * The largest such radius must not exceed 3600 arcsec. Pairs are certified
 * at their own radius exactly as hlc_xmatch certifies at r. Other arguments,
 * outputs and errors as hlc_xmatch (HLC_SELF is not supported).           */
int hlc_xmatch_radii(const double *a_ra, const double *a_dec, const double *a_err, int64_t na,
                     const double *b_ra, const double *b_dec, const double *b_err, int64_t nb,
                     double k_sigma, hlc_pair *out_pairs, double *out_sep_arcsec,
                     const hlc_opts *opts);

/* The paper's own partition, emulated for comparison (section 3.2,
 * Algorithm 1; section 4.2; Table 4): each record of A and B is indexed by its
 * HEALPix nested pixel at `order` (0..13) and by the pixels of its four
 * positions shifted by +-r in RA and in Dec (the quad-direction strategy;
 * RA wraps, Dec stops at the poles); records are compared only within a
 * shared pixel, with the same exact decision as hlc_xmatch, and each pair is
 * reported once. The result is a subset of hlc_xmatch's: the pairs it lacks
 * are the scheme's completeness loss. na, nb < 2^28. Arguments, outputs and
 * errors otherwise as hlc_xmatch (the filter is FP64; HLC_SELF unsupported). */
int hlc_xmatch_quad(const double *a_ra, const double *a_dec, int64_t na, const double *b_ra,
                    const double *b_dec, int64_t nb, double r_arcsec, int32_t order,
                    hlc_pair *out_pairs, double *out_sep_arcsec, const hlc_opts *opts);

/* Reusable device index of one catalogue (section 4.2's first-level
 * partition: positions grouped by Dec zone, then RA). An index built for
 * radius r can serve as either side of hlc_xmatch_part at any radius <= r
 * built with the same zone height. Free with hlc_part_free.                 */
struct hlc_part;
int hlc_partition(const double *ra_deg, const double *dec_deg, int64_t n, double r_arcsec,
                  const hlc_opts *opts, struct hlc_part **out);
void hlc_part_free(struct hlc_part *part);
int hlc_xmatch_part(const struct hlc_part *A, const struct hlc_part *B, double r_arcsec,
                    hlc_pair *out_pairs, double *out_sep_arcsec, const hlc_opts *opts);

/* Many independent jobs in one call (section 4.3.1's launch geometry applied
 * to thousands of calculation blocks at once). Job j matches
 * A[a_off, a_off+na) against B[b_off, b_off+nb) at radius r_arcsec; job
 * ranges may overlap. Each job is partitioned in a local frame derived from
 * its own sources; all jobs share one sort and one persistent match launch
 * over a cost-ordered work queue. Repeated calls with the same arguments
 * replay a captured HIP graph.
 *   jobs [njobs]: HOST array, 0 <= njobs <= 65536; r_arcsec in (0, 3600].
 *   a_ra..b_dec: device arrays holding all jobs; the sum of na and the sum
 *     of nb must each be below 2^30.
 *   out_pairs / out_sep: device, capacity opts->capacity; pair indices are
 *     GLOBAL (into the packed arrays).
 *   job_pair_count [njobs]: device int64, pairs found per job (may be NULL).
 *   opts->tuning: zone_height_factor, batch_tile and batch_blocks_per_cu;
 *     each one that is 0 (or no tuning) is autotuned on first use for this
 *     batch shape on this device (timed candidate runs, one knob after the
 *     other) and cached in memory, and in the JSON file named by
 *     $HLC_TUNE_CACHE when set (keyed by the device's gfx architecture and
 *     compute-unit count and by the batch's size class).
 * Total pairs go to *opts->n_pairs; overflow behaves as in hlc_xmatch.     */
typedef struct hlc_job {
  int64_t a_off, na, b_off, nb;
  double r_arcsec;
} hlc_job;
int hlc_xmatch_batch(const hlc_job *jobs, int32_t njobs, const double *a_ra, const double *a_dec,
                     const double *b_ra, const double *b_dec, hlc_pair *out_pairs,
                     double *out_sep_arcsec, int64_t *job_pair_count, const hlc_opts *opts);

/* Catalogues in pinned HOST memory (section 4.3.2: page-locked host memory).
 * B is copied to the device once, partitioned once (zones and bins framed by
 * its footprint widened by r) and kept resident; A follows in slabs of
 * consecutive sources, two device buffers deep, each slab's copy on its own
 * stream overlapping the cross-match of the previous slab (section 4.3.1).
 * Pairs are delivered through `sink` in batches from a bounded device ring
 * (indices into the caller's full arrays); `sink` returns 0 to continue,
 * non-zero to abort (the call then returns HLC_E_INVAL). An invalid
 * coordinate also ends the call with HLC_E_INVAL, after the pairs of the
 * slabs before it may already have been delivered. opts->capacity is the
 * ring size in pairs (0 = default); opts->n_pairs receives the total. B must
 * fit in device memory with its working buffers (about 150 B per source).  */
typedef int (*hlc_sink)(const hlc_pair *pairs, const double *sep_arcsec, int64_t n, void *user);
/* The slab size is chosen from the eq. (5) transfer model (measured once per
 * device): with per-slab fixed cost s = alpha_h2d + alpha_d2h + launch
 * overhead and whole-job time W, about sqrt(W / s) slabs balance the fixed
 * costs against the pipeline's fill and drain.                            */
int hlc_xmatch_stream(const double *a_ra_host, const double *a_dec_host, int64_t na,
                      const double *b_ra_host, const double *b_dec_host, int64_t nb,
                      double r_arcsec, hlc_sink sink, void *user, const hlc_opts *opts);

/* Host<->device transfer model of eq. (5): T(d) = alpha + beta * d seconds
 * for d bytes, fitted by least squares to timed pinned-memory copies of 1 B
 * to 64 MiB on the current device (the alpha/beta measurement procedure of
 * section 4.1). The streaming form uses it to size its A slabs.          */
typedef struct hlc_transfer {
  double alpha_h2d, beta_h2d;  /* s, s/byte */
  double alpha_d2h, beta_d2h;
  double r2_h2d, r2_d2h;       /* coefficient of determination of each fit */
} hlc_transfer;
int hlc_transfer_model(hlc_transfer *out);

const char *hlc_strerror(int status);
int hlc_last_stats(hlc_stats *out);
void hlc_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* HLC_H_ */
