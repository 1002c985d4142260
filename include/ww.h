/*
 * ww.h -- C ABI of the MI355X (gfx950) minimum-cost-flow phase unwrapper.
 *
 * The calls follow the problem statement of Section II-A of "A
 * Probabilistic-Cost Algorithm for Large-Scale 2D Phase Unwrapping": a
 * wrapped phase psi in (-pi, pi], a sample coherence per pixel (eq. 3), the
 * number of looks L and a validity mask go in; the integer cycle field K and
 * the unwrapped phase phi = psi + 2 pi K come out.
 *
 * Conventions shared by every call
 *   - Images are row-major, m rows (slow axis i) by n columns (fast axis j),
 *     contiguous, no padding.  1 <= m, n and m*n < 2^31.
 *   - x-edge hx(i,j) joins pixel (i,j) to (i,j+1): array of m*(n-1).
 *     y-edge vy(i,j) joins pixel (i,j) to (i+1,j): array of (m-1)*n.
 *     loop p(i,j) has corners (i,j),(i,j+1),(i+1,j+1),(i+1,j): (m-1)*(n-1).
 *   - Pointers without a _host suffix are DEVICE pointers on the current HIP
 *     device; the caller allocates and owns them.  The library owns only its
 *     internal workspace and its cost-table cache, which it keeps until the
 *     process ends.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it; calls that return a value through a _host
 *     pointer synchronise that stream before returning.
 *   - No exception crosses the ABI.  A non-zero status leaves the outputs
 *     unspecified; ww_last_error() then describes it (per thread).
 *   - Repeated calls with the same inputs produce identical bytes.
 */
#ifndef WW_H
#define WW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ww_status;
#define WW_OK 0
#define WW_E_INVALID_ARG (-1) /* bad shape, NULL pointer or parameter      */
#define WW_E_OOM (-2)         /* device or host allocation failed          */
#define WW_E_INFEASIBLE (-3)  /* a supply can reach no demand              */
#define WW_E_DEVICE (-4)      /* a HIP call failed                         */
#define WW_E_OVERFLOW (-5)    /* an integer range guard tripped            */

/* Message for the calling thread's last non-OK status ("" if none). */
const char *ww_last_error(void);

/* Library version string. */
const char *ww_version(void);

/* Discretisation of the cost table of Section II-B (eqs. 4-7).
 *   n_alpha  slope bins over [-pi, pi] (bin centres -pi + (b+1/2) 2pi/n_alpha)
 *   n_gamma  coherence bins over [0, 1] (bin centres (c+1/2)/n_gamma)
 *   n_eta    phase-noise samples over (-pi, pi] (midpoints)
 *   n_gpanel, n_gnode  composite Gauss-Legendre rule over the true coherence
 *            for the marginalisation of eq. 5 (panels x nodes per panel)
 *   n_aquad  nodes of the slope marginalisation of eq. 7 over
 *            alpha_hat +- sigma_span * sigma_alpha                        */
typedef struct {
    int32_t n_alpha, n_gamma, n_eta, n_gpanel, n_gnode, n_aquad;
    double sigma_span;
} ww_lut_params;

/* Per-edge cost rules of Section II-B.
 *   box_half      half-width h of the (2h+1)^2 slope box filter (>= 0)
 *   steep_rule    1: edges with |wrapped gradient| > steep_thresh_rad cost 0,
 *                 at most floor(steep_cap_pct * valid_edges / 100) of them
 *   ref_i, ref_j  pixel with K = 0 (-1: first valid pixel, row-major)
 *   nodata        phi written at invalid pixels
 *   lut_interp    0 (default): nearest table bin; 1: the table interpolated
 *                 at run time (Section II-B), bilinear between bin centres:
 *                 slope position t16 = floor((S+K P) n_alpha 2^16/(2 K P)) - 2^15,
 *                 coherence position u16 = floor(g n_gamma 2^16) - 2^15 (FP64),
 *                 each split into a cell and a 16-bit fraction and clamped to
 *                 the outermost centres; the int64 blend of the four entries
 *                 is shifted right by 32; the reverse arc uses
 *                 (n_alpha-1) 2^16 - t16.
 *   looks_frac16  0 (default): the table of the integer number of looks;
 *                 f in [1, 65535]: the effective number of looks is
 *                 looks + f / 2^16 (looks <= 63), and the table is the
 *                 blend of the integer tables of looks and looks + 1
 *                 (Section II-B reads its table grid, which includes L, by
 *                 interpolation), see ww_build_cost_lut_q16.             */
typedef struct {
    int32_t box_half;
    int32_t steep_rule;
    double steep_thresh_rad;
    int32_t steep_cap_pct;
    int32_t ref_i, ref_j;
    float nodata;
    int32_t lut_interp;
    int32_t looks_frac16;
} ww_cost_params;

/* Solver counters (all optional outputs). */
typedef struct {
    int64_t passes;          /* multi-source shortest-path passes            */
    int64_t windows;         /* distance windows processed                  */
    int64_t rounds;          /* tile relaxation rounds (kernel launches)    */
    int64_t tile_visits;     /* tiles relaxed, summed over rounds           */
    int64_t augmentations;   /* unit augmenting paths                       */
    int64_t path_arcs;       /* arcs flipped by augmentations               */
    int64_t supplies;        /* initial positive charge incl. the ground    */
    int64_t max_potential;   /* largest node potential at exit              */
    double relax_ms;         /* device time of the relaxation rounds        */
    double solve_ms;         /* wall time of the whole solve                */
    int64_t settled_nodes;   /* nodes settled, summed over passes, and their */
    int64_t arcs_scanned;    /* residual out-arcs: the work of a textbook    */
                             /* search settling the same nodes; counted when */
                             /* the environment sets WW_MCF_COUNT=1 (which  */
                             /* slows the solve), else -1                   */
} ww_mcf_stats;

/* Schedule of the min-cost-flow solve: the shortest-path windows of every
 * pass (Section II-C replaces Dial's unit buckets by windows; any increasing
 * sequence of windows gives the same exact labels, so these only trade
 * relaxation rounds against windows) and when a pass stops searching.  Every
 * schedule reaches an optimum of the same cost.
 *   first_hop_window     hop limit of a pass's first, zero-distance window
 *                        (1 .. 2^29-2; later zero-distance windows grow by
 *                        hop_growth)
 *   first_distance_step  first increment of the distance bound (1 .. 2^30;
 *                        later increments double)
 *   full_passes          number of first passes that search until every
 *                        reachable deficit is settled (0 .. 2^20)
 *   first_deficit_after  0: every later pass stops once half of the
 *                        remaining units have a settled deficit; 1: every
 *                        later pass stops at the first window that settles a
 *                        deficit.  full_passes = 8 with first_deficit_after = 1
 *                        is the paper's schedule of Section II-C (eight full
 *                        multi-source passes, then searches that stop at the
 *                        first deficit).
 *   reverse_below        0: every pass searches from the supplies; n > 0:
 *                        once at most n units are left, passes search from
 *                        the demands instead (the same successive shortest
 *                        paths on the reversed problem: arcs turned round,
 *                        supplies and demands exchanged, potentials negated)
 *   hop_growth           factor by which the hop limit of each later
 *                        zero-distance window grows (2 .. 2^20; the limit is
 *                        at least the hops of the smallest parked candidate)
 *   tile_cols            columns of the loop tiles the relaxation rounds
 *                        work on (16, 32 or 64; a tile holds 1024 loops, so
 *                        64, 32 or 16 rows): the shape of the frontier's
 *                        granule, a speed knob like the windows
 * Process-wide; applies to solves that start after the call. */
typedef struct {
    int32_t first_hop_window;
    int32_t first_distance_step;
    int32_t full_passes;
    int32_t first_deficit_after;
    int32_t reverse_below;
    int32_t hop_growth;
    int32_t tile_cols;
} ww_mcf_params;

/* Defaults: first_hop_window 64, first_distance_step 256, full_passes 0,
 * first_deficit_after 0, reverse_below 0, hop_growth 2, tile_cols 32. */
void ww_default_mcf_params(ww_mcf_params *p);
/* Errors: WW_E_INVALID_ARG (NULL or out of range). */
ww_status ww_set_mcf_params(const ww_mcf_params *p);
void ww_get_mcf_params(ww_mcf_params *p);

/* Counters of the most recent min-cost-flow solve made by this process
 * (through ww_mcf_solve or ww_unwrap).  Writes zeros before the first. */
void ww_last_mcf_stats(ww_mcf_stats *out);

/* Defaults: n_alpha 128, n_gamma 64, n_eta 2048, 64 x 16 Gauss-Legendre
 * nodes, n_aquad 513, sigma_span 8; box_half 2, steep rule on at 1 rad and
 * 3 %, reference = first valid pixel, nodata = NaN. */
void ww_default_lut_params(ww_lut_params *p);
void ww_default_cost_params(ww_cost_params *p);

/* Residues, eq. 1 (Section II-A), and the balancing boundary charges of the
 * outer ring of zero-cost, unbounded arcs (Section II-A).
 *   psi    float32 [m*n] wrapped phase; pixels with valid == 0 are read as 0.
 *   valid  uint8 [m*n] validity mask (non-zero = valid); NULL = all valid.
 *   res    int8 [(m-1)*(n-1)] out: charge of loop p(i,j) in {-1,0,1}, loop
 *          traversed (i,j)->(i,j+1)->(i+1,j+1)->(i+1,j).
 *   perim  int8 [2(n-1)+2(m-1)] out, nullable: one-sided charges of the ring
 *          beside the top x-edges, bottom x-edges, left y-edges, right
 *          y-edges, in that order.
 *   ground_charge_host  int64 out, nullable (synchronises): -(sum of res).
 * Errors: WW_E_INVALID_ARG on m, n < 1 or NULL psi/res; WW_E_DEVICE. */
ww_status ww_residues(const float *psi, const uint8_t *valid, int32_t m, int32_t n,
                      int8_t *res, int8_t *perim, int64_t *ground_charge_host, void *stream);

/* Integer cost table of Section II-B, eqs. 4-7: entry [c][b] is
 * min(32767, floor(100 max{0, -ln(P+/P0)})) at coherence bin c and slope bin
 * b; 32767 where P+ = 0.  Built in FP64 by HIP kernels on the current device
 * and copied to the host buffer.
 *   looks     number of looks L, 2 <= L <= 64.
 *   p         discretisation, NULL = defaults.
 *   lut_host  int16 [n_gamma * n_alpha] out, row = coherence bin.
 * Synchronous.  Errors: WW_E_INVALID_ARG, WW_E_OOM, WW_E_DEVICE. */
ww_status ww_build_cost_lut(int32_t looks, const ww_lut_params *p, int16_t *lut_host);

/* The table at a non-integer number of looks (Section II-B: the table is
 * precomputed on a grid over slope, coherence and L and read by
 * interpolation at run time; the L grid here is the integers).
 *   looks_q16  effective looks in 2^-16 fixed point, 2 <= looks_q16 / 2^16
 *              <= 64; with l0 = looks_q16 >> 16 and f = looks_q16 & 0xffff,
 *              entry [c][b] = floor((T_l0[c][b] (2^16 - f) +
 *              T_l0+1[c][b] f) / 2^16), the integer tables of
 *              ww_build_cost_lut (f = 0: T_l0 itself).
 * Synchronous; the table is cached per device.  Errors as
 * ww_build_cost_lut. */
ww_status ww_build_cost_lut_q16(int32_t looks_q16, const ww_lut_params *p, int16_t *lut_host);

/* Per-edge integer costs of Section II-B.  For every edge e = (u -> v):
 *   cx_pos/cy_pos  cost of the arc that raises the edge's cycle difference by
 *                  one: T[bg][ba], ba = bin of the box-filtered wrapped
 *                  gradient (fixed point 2^-20 rad, clipped window, samples
 *                  with two valid endpoints), bg = bin of min(coh_u, coh_v);
 *   cx_neg/cy_neg  the reverse correction: T[bg][n_alpha-1-ba];
 *   (with cp->lut_interp = 1 both are the interpolated lookups instead)
 * 0 for edges with an invalid endpoint and for the steep edges.
 *   psi, coh  float32 [m*n]; coh is clamped to [0,1], NaN read as 0.
 *   valid     uint8 [m*n], NULL = all valid.
 *   lut       int16 [n_gamma*n_alpha] DEVICE copy of ww_build_cost_lut.
 *   lp        table shape (only n_alpha, n_gamma are read), NULL = defaults.
 *   cp        cost rules, NULL = defaults.
 *   cx_pos, cx_neg  int16 [m*(n-1)] out; cy_pos, cy_neg int16 [(m-1)*n] out.
 * Errors: WW_E_INVALID_ARG, WW_E_OOM, WW_E_DEVICE. */
ww_status ww_edge_costs(const float *psi, const float *coh, const uint8_t *valid, int32_t m,
                        int32_t n, const int16_t *lut, const ww_lut_params *lp,
                        const ww_cost_params *cp, int16_t *cx_pos, int16_t *cx_neg,
                        int16_t *cy_pos, int16_t *cy_neg, void *stream);

/* Minimum-cost flow of eq. 2 (Section II-A) on the loop graph plus one
 * ground node standing for the outer ring, solved exactly by successive
 * shortest paths with potentials (Section II-C): every pass grows a
 * shortest-path forest from all supplies at once over integer reduced costs
 * and augments one unit along vertex-disjoint forest paths.
 *   res      int8 [(m-1)*(n-1)] loop charges (supply +1, demand -1).
 *   costs    the four int16 planes of ww_edge_costs (all >= 0).
 *   dk_x     int8 [m*(n-1)] out: cycle difference of each x-edge in {-1,0,1}.
 *   dk_y     int8 [(m-1)*n] out: same for y-edges.
 *   potentials  int64 [(m-1)*(n-1)+1] out, nullable: optimal node potentials
 *            (ground last); every residual arc has cost - pot(u) + pot(v) >= 0.
 *   total_cost_host  int64 out: sum of the costs of the chosen corrections.
 *   stats_host  ww_mcf_stats out, nullable.
 * Synchronous.  m or n = 1: no loops, zero flow, cost 0.
 * Errors: WW_E_INVALID_ARG, WW_E_OOM, WW_E_INFEASIBLE, WW_E_OVERFLOW,
 * WW_E_DEVICE. */
ww_status ww_mcf_solve(const int8_t *res, int32_t m, int32_t n, const int16_t *cx_pos,
                       const int16_t *cx_neg, const int16_t *cy_pos, const int16_t *cy_neg,
                       int8_t *dk_x, int8_t *dk_y, int64_t *potentials, int64_t *total_cost_host,
                       ww_mcf_stats *stats_host, void *stream);

/* Integration of the corrected gradients (Sections II-A, II-C): K(ref) = 0
 * and K_v - K_u = dk_e - w_e along every edge, w_e the wrap count of psi;
 * phi = (float)((double)psi + 2 pi K) at valid pixels, cp->nodata elsewhere.
 *   psi, valid  as for ww_residues; dk_x, dk_y from ww_mcf_solve.
 *   cp       reference pixel and nodata, NULL = defaults.
 *   K        int32 [m*n] out (written at every pixel); phi float32 [m*n] out.
 * Errors: WW_E_INVALID_ARG, WW_E_DEVICE. */
ww_status ww_integrate(const float *psi, const uint8_t *valid, const int8_t *dk_x,
                       const int8_t *dk_y, int32_t m, int32_t n, const ww_cost_params *cp,
                       int32_t *K, float *phi, void *stream);

/* ww_integrate for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, results and errors as ww_integrate, and WW_E_INVALID_ARG
 * for m > 65536.  Its scratch (the integration state and one int32 per row:
 * 256 B + 256 KiB) is a static device array, one copy per device, held until
 * the process ends; the call allocates nothing.  The first call on a device
 * looks up that copy's address.  Every call on one device shares the array:
 * calls that overlap on one device (other streams or threads) race, so the
 * caller serialises them.  The state is re-initialised by every call. */
ww_status ww_integrate_noalloc(const float *psi, const uint8_t *valid, const int8_t *dk_x,
                               const int8_t *dk_y, int32_t m, int32_t n,
                               const ww_cost_params *cp, int32_t *K, float *phi, void *stream);

/* The whole path: residues -> cost table (cached per L) -> edge costs ->
 * min-cost flow -> integration, on one device with library workspace.
 *   coh    float32 [m*n] sample coherence; looks as ww_build_cost_lut.
 *   cp     NULL = defaults.   K, phi as ww_integrate.
 *   total_cost_host  int64 out, nullable (the call synchronises anyway).
 * Errors: as the five calls above. */
ww_status ww_unwrap(const float *psi, const float *coh, const uint8_t *valid, int32_t m,
                    int32_t n, int32_t looks, const ww_cost_params *cp, int32_t *K, float *phi,
                    int64_t *total_cost_host, void *stream);

/* Connected components of reliably unwrapped pixels (Section II-D).  An
 * edge is reliable when both pixels are valid and changing its cycle
 * difference by +1 or by -1 would each raise its cost by more than
 * `threshold` cost units: dk = 0, c+ > threshold and c- > threshold (an
 * edge with dk = +-1 could be changed back for a refund, so it is never
 * reliable).  Components are grown over reliable edges; those with at
 * least max(1, ceil(min_size_frac * valid pixels)) pixels are numbered
 * 1, 2, ... in row-major order of their first pixel, all other pixels and
 * every invalid pixel get 0.
 *   threshold      >= 0, cost units of ww_edge_costs (default 300)
 *   min_size_frac  in [0, 1] (default 0.001)                            */
typedef struct {
    int32_t threshold;
    double min_size_frac;
} ww_cc_params;

void ww_default_cc_params(ww_cc_params *p);

/*   dk_x, dk_y     the cycle differences of ww_mcf_solve.
 *   cx_*, cy_*     the cost planes of ww_edge_costs.
 *   valid          uint8 [m*n], NULL = all valid.
 *   labels         uint32 [m*n] out.
 *   ncomp_host     int64 out: number of labelled components (synchronises).
 * Errors: WW_E_INVALID_ARG, WW_E_OOM, WW_E_DEVICE. */
ww_status ww_connected_components(const int8_t *dk_x, const int8_t *dk_y, const int16_t *cx_pos,
                                  const int16_t *cx_neg, const int16_t *cy_pos,
                                  const int16_t *cy_neg, const uint8_t *valid, int32_t m,
                                  int32_t n, const ww_cc_params *p, uint32_t *labels,
                                  int64_t *ncomp_host, void *stream);

/* Goldstein adaptive power-spectrum filter (the optional preprocessing of
 * Section II-D).  Unit phasors exp(i psi) at valid pixels, 0 elsewhere and
 * outside the image, in patch x patch windows on a grid of step patch/2
 * whose first window starts patch/2 rows above and columns left of the
 * image (every pixel lies in four windows).  Per window: the 2-D DFT Z is
 * multiplied by (B / max B)^alpha, B the circular smooth x smooth mean of
 * |Z| (an all-zero window contributes 0); the inverse DFT is tapered by
 * w(r) w(c), w(i) = 1 - |2i + 1 - patch| / patch; the filtered phase is the
 * argument of the sum of the tapered windows at each valid pixel, and
 * invalid pixels keep psi.  FP32 arithmetic.
 *   patch   16, 32 or 64 (default 32)
 *   smooth  1, 3 or 5 (default 3)
 *   alpha   exponent in [0, 4] (default 0.5)                            */
typedef struct {
    int32_t patch;
    int32_t smooth;
    float alpha;
} ww_filter_params;

void ww_default_filter_params(ww_filter_params *p);

/*   psi, valid  as ww_residues (device).
 *   p           NULL = defaults.
 *   psi_out     float32 [m*n] out (device), may equal psi.
 * Uses 32 bytes per pixel of library workspace.
 * Errors: WW_E_INVALID_ARG, WW_E_OOM, WW_E_DEVICE. */
ww_status ww_goldstein_filter(const float *psi, const uint8_t *valid, int32_t m, int32_t n,
                              const ww_filter_params *p, float *psi_out, void *stream);

/* Cycle counts found on a filtered copy psi_f moved onto the original phase
 * psi (Section II-D: the modified phase only estimates K).  At a valid pixel
 * K = K_f + k, k the integer that puts psi + 2 pi K within (-pi, pi] of
 * psi_f + 2 pi K_f: k = -([x > pi] - [x <= -pi]), x = psi - psi_f in FP64;
 * at an invalid pixel K = K_f.  With ref_i >= 0 every K is then shifted so
 * that K(ref_i, ref_j) = 0.  phi = (float)((double)psi + 2 pi K) at valid
 * pixels, nodata elsewhere.
 *   K_f    int32 [m*n] (device); K may equal K_f.
 *   K, phi int32 / float32 [m*n] out (device).
 * Errors: WW_E_INVALID_ARG, WW_E_OOM, WW_E_DEVICE. */
ww_status ww_transfer_ambiguity(const float *psi, const uint8_t *valid, const float *psi_f,
                                const int32_t *K_f, int32_t m, int32_t n, int32_t ref_i,
                                int32_t ref_j, float nodata, int32_t *K, float *phi,
                                void *stream);

/* ww_unwrap on the Goldstein-filtered phase, then ww_transfer_ambiguity
 * onto psi with the reference pixel of the integration (K = 0 there).
 * total_cost_host is the optimum of the filtered problem.
 * Errors: as ww_unwrap and ww_goldstein_filter. */
ww_status ww_unwrap_filtered(const float *psi, const float *coh, const uint8_t *valid, int32_t m,
                             int32_t n, int32_t looks, const ww_cost_params *cp,
                             const ww_filter_params *fp, int32_t *K, float *phi,
                             int64_t *total_cost_host, void *stream);

/* Bridging of mask-separated regions (Section II-D post-processing).  The
 * wrapped phase carries no information about the relative cycle levels of
 * regions the mask separates; this call sets them.  Regions are the
 * 4-connected components of valid pixels, numbered 1, 2, ... in row-major
 * order of their first pixel, and ranked by decreasing size (ties by
 * number).  Each region of rank k >= 1 attaches to the region of smaller
 * rank holding the pixel closest to it: the pair (p in the region, q of
 * smaller rank) minimising (|p - q|^2, index p, index q), indices
 * row-major.  With phi = psi + 2 pi K in FP64, the lower medians of phi
 * over the pixels of the same region in the (2 half_window + 1)^2 windows
 * centred on q and on p give d = floor((med_q - med_p) / 2 pi + 1/2); the
 * region's shift is its parent's shift plus d, and the largest region keeps
 * its cycle counts.
 *   half_window  0..32 (default 32: 65 x 65 windows)                      */
typedef struct {
    int32_t half_window;
} ww_bridge_params;

void ww_default_bridge_params(ww_bridge_params *p);

/*   psi, valid   as ww_residues (device); m, n <= 46000.
 *   K_in         int32 [m*n] cycle counts (device), e.g. from ww_unwrap.
 *   K_out, phi   int32 / float32 [m*n] out (device): K_in + shift at valid
 *                pixels, K_in elsewhere; phi = (float)((double)psi +
 *                2 pi K_out), nodata at invalid pixels.  K_out may equal
 *                K_in.
 *   regions      uint32 [m*n] out (device), nullable: region numbers
 *                (0 = invalid).
 *   nregions_host  int64 out: number of regions.
 * Synchronous.  Errors: WW_E_INVALID_ARG, WW_E_OOM, WW_E_DEVICE. */
ww_status ww_bridge(const float *psi, const uint8_t *valid, const int32_t *K_in, int32_t m,
                    int32_t n, const ww_bridge_params *p, float nodata, int32_t *K_out,
                    float *phi, uint32_t *regions, int64_t *nregions_host, void *stream);

/* ---------------------------------------------------------------------
 * Many interferograms: a job server and a batch call.
 *
 * A server runs `slots` workers on the current device.  Each worker owns a
 * HIP stream (default priority) and a private workspace, so jobs on
 * different workers overlap on the GPU.  A submitted job waits in a queue
 * until a worker is free and its device footprint fits the server's HBM
 * budget beside the jobs already running; the first queued job that fits
 * is taken, and a job that has waited longer than one second blocks the
 * jobs behind it until it fits (no job starves).  A job larger than the
 * budget runs alone.  Each job computes exactly what ww_unwrap computes on
 * the same inputs (default cost rules), byte for byte.
 * ------------------------------------------------------------------- */

/* One unwrap request.  The caller fills the inputs and keeps the struct
 * (and its arrays) alive until the server hands it back. */
typedef struct {
    int32_t m, n, looks;
    int32_t host_io;         /* 0: the five arrays are device pointers;
                                1: host pointers (pinned for full copy
                                speed); the worker copies in and out    */
    const float *psi;        /* [m*n] wrapped phase                      */
    const float *coh;        /* [m*n] sample coherence                   */
    const uint8_t *valid;    /* [m*n] mask, NULL = all valid             */
    int32_t *K;              /* [m*n] out                                */
    float *phi;              /* [m*n] out                                */
    int64_t tag;             /* caller's, not touched                    */
    /* outputs */
    ww_status status;
    int64_t total_cost;
    double t_submit, t_start, t_end;  /* seconds on ww_clock()          */
    int64_t footprint_bytes;          /* device bytes reserved for it   */
    char error[160];                  /* message when status != WW_OK  */
    /* input: the job's own solve schedule (used by the server when
     * use_sched = 1; 0 = the process-wide schedule) */
    int32_t use_sched;
    ww_mcf_params sched;
} ww_job;

typedef struct ww_server ww_server;

/* Seconds on the monotonic clock the server stamps jobs with. */
double ww_clock(void);

/* Starts `slots` workers (1..64) on the current device with an HBM budget
 * in bytes (<= 0: 3/4 of the device memory that is free at creation).  A
 * job is admitted when the device bytes held by all workers, counting for
 * each the larger of its (grow-only) workspace and its running job's
 * footprint, stay within the budget; a job's footprint is every device
 * byte that ww_unwrap's workspace requests for its shape, plus device
 * copies of host-side inputs and outputs.
 * Errors: WW_E_INVALID_ARG, WW_E_DEVICE. */
ww_status ww_server_create(int32_t slots, int64_t hbm_budget_bytes, ww_server **out);

/* Queues a job (stamps t_submit).  Errors: WW_E_INVALID_ARG (NULL job or
 * server, stopped server). */
ww_status ww_server_submit(ww_server *s, ww_job *job);

/* Hands back up to max_done finished jobs in completion order, waiting up
 * to wait_ms (< 0: until at least one finishes or nothing is in flight).
 * Returns the number written to done[]. */
int32_t ww_server_poll(ww_server *s, ww_job **done, int32_t max_done, int32_t wait_ms);

/* Jobs submitted but not yet handed back by ww_server_poll. */
int64_t ww_server_in_flight(ww_server *s);

/* Waits for the queued and running jobs, stops the workers and frees the
 * server (finished jobs not yet polled keep their outputs). */
ww_status ww_server_destroy(ww_server *s);

/* Unwraps njobs jobs (a time-series stack of interferograms of any sizes)
 * as a batch on the current device and returns when all have finished.
 * Residues, costs and integration run per job; the min-cost-flow solve
 * runs once for a whole group of jobs: the jobs' loop graphs, each with
 * its own ground node, form one disjoint graph whose flow problem is the
 * sum of the jobs' problems (Section II-A eq. 2), and one run of successive
 * shortest paths (Section II-C) solves it, every relaxation round covering
 * the frontier tiles of all jobs of the group.  Each job's cost equals
 * what ww_unwrap computes on it (default cost rules); its K is an optimum's
 * cycle field, equal to ww_unwrap's wherever the optimum is unique (where
 * several optima exist the shared passes may pick another one; group = 1
 * reproduces ww_unwrap byte for byte).  Repeated calls on the same jobs in
 * the same order give identical bytes.
 *   group  jobs per solve at most (1..256; 0 = 256); consecutive jobs in
 *          the given order form a group, which also stays below 2^31 loops
 *          and 400 Mpixel;
 *   sched  the solve schedule, NULL = the process-wide one.
 * A job that cannot be unwrapped gets its status and message; when a group
 * solve fails, its jobs are solved one by one so that only the failing job
 * fails.  Returns WW_OK if every job succeeded, else the first failure's
 * status.  Uses the library workspace of the current device. */
ww_status ww_unwrap_batch(ww_job *jobs, int32_t njobs, int32_t group, const ww_mcf_params *sched);

/* ---------------------------------------------------------------------
 * Measurement
 * ------------------------------------------------------------------- */

/* Streaming ceiling of the device (not part of the unwrapping path): times
 * `reps` launches of a hand-written grid sweep over `bytes` bytes with
 * 16-byte accesses, after one untimed launch, and returns the average
 * launch time in *ms_host (HIP events on `stream`; synchronises it).
 *   mode 0  copy src -> dst (bytes read + bytes written);
 *   mode 1  read src only; dst receives one 16-byte word per workgroup
 *           (it must hold 32 KiB);
 *   mode 2  copy with non-temporal loads and stores.
 * src and dst are device pointers, 16-byte aligned; bytes a positive
 * multiple of 16; they must not overlap. */
ww_status ww_stream_probe(const void *src, void *dst, int64_t bytes, int32_t mode, int32_t reps,
                          float *ms_host, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* WW_H */
