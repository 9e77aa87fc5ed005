/*
 * mcrt.h -- C ABI of the MI355X (gfx950) Monte Carlo dust radiative-transfer
 * library: the photon-package life cycle and its path-replay adjoint.
 *
 * Method: Camps & Baes, "SKIRT: an advanced dust radiative transfer code with
 * a user-friendly architecture" (arXiv:1410.1629).  Sect. 1 names the
 * techniques (photon packages; peel-off at emission and scattering,
 * Yusef-Zadeh et al. 1984; continuous absorption, Lucy 1999 and Niccolini et
 * al. 2003; forced scattering, Cashwell & Everett 1959).  Sect. 2.2 defines
 * the problem data: a grid of cells with constant density and optical
 * properties (Table 1(d): regular Cartesian grid), sources with a geometry
 * and a luminosity per wavelength (Table 1(a): point and exponential disk),
 * and instruments: frames and SEDs seen by a distant observer (parallel
 * projection) and perspective cameras placed anywhere.  Sect. 2.3 gives the
 * optical properties: kappa (extinction per unit density), albedo
 * kappa_sca/kappa_ext and the asymmetry parameter g of the phase function
 * (Henyey-Greenstein here).  Fig. 4/5 give the instrument parameters and the
 * package count; Fig. 5 the seeded random generator (default seed 4357).
 *
 * Conventions shared by every entry point
 *  - Cell m = i + nx*(j + ny*k), x fastest.  Cells are half-open along each
 *    axis; a point on a wall moving towards lower indices belongs to the
 *    lower cell.
 *  - Densities live on the device.  precision == MCRT_PREC_FP64: double;
 *    precision == MCRT_PREC_FP32: float (the walk's densities, optical
 *    depths and exponentials in FP32; package state, every tally, and the
 *    crossing times of the life-cycle kernel's walks in FP64 -- a segment's
 *    length is a difference of two crossing times, which FP32 would carry
 *    with an error proportional to the distance walked).  FP32 calls on
 *    regular and rectilinear grids take at most 2^24 - 1 cells along each
 *    axis (the FP32 walks count crossed planes in FP32); larger grids fail
 *    with MCRT_EINVAL.
 *  - Images are FP64 flux per pixel (luminosity / distance^2), laid out as
 *    [comp][lambda][frame pixels], where one wavelength's block is the
 *    frames one after another, each [ny][nx] row-major; comp is 2 with
 *    MCRT_SPLIT (0: direct light peeled off at emission, 1: scattered light),
 *    else 1.
 *  - Frame geometry (distant instruments): observer direction
 *    (sin t cos p, sin t sin p, cos t);
 *    image axes e_x = (-sin p, cos p, 0), e_y = (-cos t cos p, -cos t sin p,
 *    sin t), rotated by the position angle; frame [-half_x, half_x] x
 *    [-half_y, half_y] around the origin; pixels half-open.
 *  - Random numbers: Philox4x32-10 with key = seed and counter = (package
 *    index lo, hi, wavelength index, draw index): draw 0 emission position,
 *    draw 1 emission direction and source choice, draw 2+n scattering n.
 *    Any package range [first, first + n) therefore reproduces exactly the
 *    packages of a larger run.
 *  - Every call is asynchronous on `hip_stream` (a hipStream_t, NULL for the
 *    default stream) unless it returns statistics, in which case it waits
 *    for its own work to finish before returning.
 *  - Ownership: the caller owns every buffer; host structs and arrays are
 *    read only during the call.  The library keeps no state between calls.
 *    Each call allocates stream-ordered device memory (hipMallocAsync) for
 *    its tables, a bricked copy of the densities and, where it has one, a
 *    tally in the library's own cell order (the forward's absorbed tally
 *    takes up to twice the cells of the grid per wavelength: its cell units
 *    are padded to a power of two), the adjoint's event scratch and the
 *    peel-ray queue, and frees it on the stream when its work ends.
 *  - Errors: 0 on success; MCRT_EINVAL for invalid arguments (nothing is
 *    launched), MCRT_EOVERFLOW when a segment buffer was too small,
 *    MCRT_EHIP for a HIP runtime error.  mcrt_last_error() returns a message
 *    for the last nonzero return of the calling thread.  No call aborts.
 */
#ifndef MCRT_H
#define MCRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCRT_OK 0
#define MCRT_EINVAL (-1)
#define MCRT_EOVERFLOW (-2)
#define MCRT_EHIP (-3)

#define MCRT_PEEL_EMIT 1u /* peel-off at emission */
#define MCRT_PEEL_SCAT 2u /* peel-off at every scattering */
#define MCRT_ABSORB 4u    /* per-cell absorbed-luminosity tally */
#define MCRT_SPLIT 8u     /* separate direct and scattered images */
#define MCRT_ATTACHED 16u /* backward_density, backward: the attached (pathwise) gradient */

/* Most events (emission and scatterings) a package may have in a call with
 * MCRT_ATTACHED; the bound is that of mcrt_tape_bytes. */
#define MCRT_ATTACHED_MAX_EVENTS 4096

#define MCRT_PREC_FP64 0
#define MCRT_PREC_FP32 1

#define MCRT_SRC_POINT 0
#define MCRT_SRC_EXPDISK 1
#define MCRT_SRC_CELLS 2

#define MCRT_MAX_SOURCES 8
#define MCRT_MAX_DETECTORS 8
#define MCRT_MAX_PACKAGES 20000000000000ULL /* 2e13, the paper's upper bound (Fig. 3) */
#define MCRT_MAX_SCATTER_LIMIT 1000000

/* Cartesian grid of cuboidal cells (Table 1(d)): box and cells per axis.
 * planes NULL: regularly spaced cells (LinCub).  Otherwise a host array of
 * the cell-boundary coordinates -- nx + 1 along x, then ny + 1 along y, then
 * nz + 1 along z -- each run strictly increasing from the box's minimum to
 * its maximum (equal to them exactly): cells spaced by any rule, such as
 * the power-law spacing of PowCub (Table 1(d)).  Cell m = i + nx (j + ny k)
 * either way.
 *
 * tree_nodes > 0 (planes NULL): a tree grid (Table 1(d): k-d tree; an
 * octree is three binary levels per octree level, Sect. 2.4), host arrays
 * of tree_nodes entries.  Node 0 is the box.  Node q with tree_axis[q] in
 * {0, 1, 2} is split along that axis at tree_split[q], strictly inside the
 * node, into the nodes tree_child[q] (the lower side) and tree_child[q] + 1
 * (the upper side), both numbered above q; tree_axis[q] = -1 marks a leaf,
 * and tree_child[q] is then its cell index.  The cells are the leaves:
 * nx * ny * nz of them, each index used by one leaf; every node is reached
 * from node 0 exactly once; depth at most 64.  A point on a split plane
 * belongs to the side the ray moves to (the upper side when it moves
 * parallel to the plane).  brick_shape does not apply.  All arrays are read
 * only during the call. */
typedef struct {
    double xmin, xmax, ymin, ymax, zmin, zmax;
    int32_t nx, ny, nz;
    const double *planes;
    int32_t tree_nodes;
    const int32_t *tree_axis;
    const double *tree_split;
    const int32_t *tree_child;
} mcrt_grid;

/* Optical properties per wavelength (Sect. 2.3); host arrays [n_lambda]:
 * kappa >= 0 (extinction per unit density), 0 <= albedo <= 1, |g| < 1. */
typedef struct {
    int32_t n_lambda;
    const double *kappa, *albedo, *g;
} mcrt_optics;

/* Source (Table 1(a)): MCRT_SRC_POINT at (x, y, z), or MCRT_SRC_EXPDISK
 * centred there with density ~ exp(-R/h_r - |z|/h_z), untruncated.
 * lum: host array [n_lambda] of luminosities >= 0.
 * MCRT_SRC_CELLS: the grid's cells emit (dust emission, Sect. 1 and 2.1):
 * cell_lum is a device array [n_lambda][cell] of luminosities >= 0 (cell m
 * as in mcrt_grid), for instance the output of dust_emission; a package of
 * wavelength l starts in a cell drawn with probability proportional to
 * cell_lum[l][m], at a uniform position inside it, in an isotropic
 * direction; lum and (x, y, z, h_r, h_z) are ignored.  At most one cell
 * source per call; the call then waits for the per-wavelength totals of
 * cell_lum and fails with MCRT_EINVAL if one is negative or not finite. */
typedef struct {
    int32_t kind;
    double x, y, z, h_r, h_z;
    const double *lum;
    const double *cell_lum;
} mcrt_source;

/* Instruments (Sect. 2.2: instruments record the flux received at a
 * viewpoint; Fig. 4/5).  kind:
 *  MCRT_DET_FRAME: a distant observer (parallel projection) at distance > 0
 *    (enters as 1/distance^2) in the direction given by inclination and
 *    azimuth, image rotated by the position angle (degrees); nx x ny pixels
 *    over the half-extents half_x, half_y > 0 of the model's projection.
 *  MCRT_DET_SED: the same distant observer recording only the total flux
 *    per wavelength (the spectral energy distribution): nx = ny = 1, every
 *    package counts whatever its projected position; pa, half_x and
 *    half_y are ignored.
 *  MCRT_DET_PERSPECTIVE: a pinhole camera anywhere, also inside the model:
 *    at eye, looking along w = (target - eye) / |target - eye| (target !=
 *    eye); image axes e_y = up made perpendicular to w and normalised (up
 *    not parallel to w) and e_x = w x e_y; nx x ny pixels over
 *    [-half_x, half_x] x [-half_y, half_y] of the plane through target
 *    perpendicular to w.  A point r with d = r - eye and d.w > 0 is seen at
 *    (x, y) = |target - eye| (d.e_x, d.e_y) / (d.w) in that plane (points
 *    behind or at the eye are not seen); its peel-off travels from r to the
 *    eye (optical depth along that segment only) and counts 1 / |d|^2.
 *    Pixels record flux; for surface brightness divide by the pixel's
 *    solid angle at the eye, F(a2, b2) - F(a1, b2) - F(a2, b1) + F(a1, b1)
 *    with F(a, b) = atan(a b / sqrt(1 + a^2 + b^2)) for the pixel spanning
 *    [a1, a2] x [b1, b2] in units of |target - eye|.  distance and the
 *    angles are ignored.
 * Every kind has nx x ny pixels in the image layout (SED: one). */
#define MCRT_DET_FRAME 0
#define MCRT_DET_SED 1
#define MCRT_DET_PERSPECTIVE 2

typedef struct {
    double distance, incl_deg, azim_deg, pa_deg;
    int32_t nx, ny;
    double half_x, half_y;
    int32_t kind;
    double eye[3], target[3], up[3];
} mcrt_detector;

/* Run options.  n_packages per wavelength in [1, 2e13]; packages
 * [first_package, first_package + n_packages) are run; seed is the Philox
 * key; precision MCRT_PREC_*; a package stops when its weight drops below
 * w_min times its initial weight or after max_scatter scatterings (the rest
 * is tallied as truncated); flags MCRT_*.  launch_blocks, event_batch and
 * brick_shape tune the run without changing its results (0 = library
 * choice): blocks per compute unit of the persistent kernels; how many
 * lanes of a wavefront wait before the wavefront processes events (library
 * choice: 32 in the forward run -- 24 when the densities exceed 256 MiB and
 * are walked from HBM -- and 32 and 48 in the adjoint's two replays of each
 * package; a value set here applies to every launch); and the
 * brick of the library's internal cell layout, MCRT_BRICK(lx, ly, lz) for
 * bricks of 2^lx x 2^ly x 2^lz cells (each log2 in [0, 7], at most 2^10
 * cells).  The default brick fills one 128-byte cache line with the most
 * compact block of cells in physical units.  peel_queue caps the device
 * queue of peel rays, in rays per chunk of packages (at most 2^31): 0 =
 * library choice, -1 = no queue (every peel ray is walked inline by the
 * life-cycle kernel; in the adjoint its deposits go out as global atomics);
 * rays beyond the cap are walked inline.  Queued rays are sorted by frame
 * and image tile, then pixel, and walked for their optical depth by a lean
 * kernel (forward: the contribution goes to its pixel); the adjoint walks
 * them again for their deposits in bundles whose deposits are summed in LDS
 * before they reach the gradient.  The results do not depend on the cap up
 * to the order of FP64 additions -- and, in the FP32 path, up to FP32
 * rounding of the peel walks (walked inline, a ray keeps the life-cycle
 * kernel's FP64 times; queued, the queue kernel's FP32 times).
 * max_chunk caps the packages (work items: packages x wavelengths) of one
 * chunk of the call: 0 = library choice (chunks as large as the peel-ray
 * queue and the adjoint's event scratch allow), else at most that many per
 * chunk; each chunk is a launch of the life-cycle kernel (two in the
 * adjoint) followed by its queue's sort and walks.  Results do not depend on
 * it up to the order of FP64 additions.
 *
 * tape, tape_bytes: the forward run's record for its adjoint (tape NULL:
 * none).  run_photons fills a device tape of mcrt_tape_bytes bytes with,
 * per package (work item) and for each of its events, the optical depth T
 * of the path leg that follows the event and, per frame, the event's
 * peel-off contribution C and image index.  backward_density and backward,
 * called with the same arguments and densities and the filled tape, take T
 * and q = (dL/dI) C from it instead of replaying every package a first
 * time and walking its peel rays for their optical depth: each package is
 * replayed once -- its positions, directions and cells are recomputed from
 * its random numbers, never stored -- and walks only its locate legs, and
 * its peel rays with q != 0 for their deposits.  The tape records a
 * fingerprint of the run's arguments (not of the densities or a cell
 * source's luminosities, which must be the same); an adjoint whose
 * arguments differ fails with MCRT_EINVAL.  An adjoint with a tape waits
 * for its fingerprint (a 256-byte copy), so a forward run on another
 * stream must have finished.  A package with more events than the tape
 * keeps (impossible when mcrt_tape_bytes is nonzero, but checked) and a
 * loss on the absorbed tally (adj_absorbed_dev) make the adjoint replay
 * without the tape.  The forward run ignores tape_bytes and the adjoint
 * rejects a tape smaller than mcrt_tape_bytes. */
typedef struct {
    uint64_t n_packages, first_package, seed;
    int32_t precision;
    double w_min;
    int32_t max_scatter;
    uint32_t flags;
    int32_t launch_blocks, event_batch;
    int32_t brick_shape;
    int64_t peel_queue;
    int64_t max_chunk;
    void *tape;
    uint64_t tape_bytes;
} mcrt_opts;

#define MCRT_TAPE_MAX_EVENTS 64

/* Bytes of the adjoint tape of a run with these optics, frames and options
 * (see mcrt_opts.tape): 256 + items x E x (8 (1 + n_det) + 4 n_det), where
 * items = n_packages x n_lambda and E is the most events (emission and
 * scatterings) a package can have -- a package's weight after n
 * scatterings is at most albedo^n of its initial weight and the package
 * stops once it is below w_min times that, so E = min(max_scatter, 2 +
 * floor(ln w_min / ln a)) + 1 with a the largest albedo (max_scatter + 1
 * when a = 1 or w_min = 0).  Returns 0 when E exceeds MCRT_TAPE_MAX_EVENTS,
 * when there is nothing to record (no peel-off or no frame), or for
 * invalid arguments. */
uint64_t mcrt_tape_bytes(const mcrt_optics *optics, int n_det, const mcrt_opts *opts);

#define MCRT_BRICK(lx, ly, lz) (0x1000 | (lx) | ((ly) << 4) | ((lz) << 8))

/* Run statistics (FP64 luminosities summed over wavelengths; crossing
 * counts of positive-length cell segments: pass-1 paths, pass-2 locate
 * walks, peel-off rays; scattering events; packages; peel-off
 * contributions that landed in a frame; deposits into the per-cell tally:
 * absorbed luminosity forward, gradient in the adjoint).  The adjoint's
 * counts cover all of its walks: both replays of each package (pass B takes
 * what pass A kept and walks only its locate legs and the events beyond the
 * kept ones) and the peel-ray deposit walks; x_queue is the part of x_peel
 * walked by the queue kernels (each queued peel ray's optical-depth walk,
 * and its deposit walk when it has one), d_queue the part of deposits made
 * by those deposit walks, which sum them on chip before they reach the
 * tally.  Durations on the stream from HIP events: kernel_ms all kernels of
 * the call, life_ms the life-cycle kernel, queue_ms the sort and the walks
 * of the peel-ray queue.  life_launches counts the life-cycle kernel's
 * launches (the call runs its packages in chunks; the adjoint launches the
 * kernel twice per chunk).  life_ms is the sum over those launches; queue_ms
 * = sort_ms (the peel-ray sort) + peel_ms (the queue's optical-depth walks)
 * + dep_ms (the adjoint's deposit walks), each summed over the chunks.
 * With MCRT_ATTACHED: x_path counts the forward sweep's path walks and the
 * reverse sweep's leg walks, x_locate the locate walks, x_peel both walks of
 * every peel ray, deposits the gradient deposits; d_queue the crossings of
 * the peel rays' deposit walks (no density loads), x_queue the part of
 * them walked by the queue kernels (the rest, with the queue full, by the
 * attached kernel); life_ms and life_launches the attached kernel (one
 * launch per chunk), queue_ms the sort and walks of the queued deposit
 * walks. */
typedef struct {
    double emitted, absorbed, escaped, truncated;
    uint64_t x_path, x_locate, x_peel, events, packages, peels, deposits;
    double kernel_ms;
    uint64_t x_queue;
    double life_ms, queue_ms;
    uint64_t d_queue;
    uint64_t life_launches;
    double sort_ms, peel_ms, dep_ms;
} mcrt_stats;

/* Photon-package life cycle (Sect. 1 techniques, Sect. 2.2 problem data):
 * for every wavelength and package, emission, peel-off at emission,
 * then repeated traversal with continuous absorption, forced scattering,
 * peel-off at scattering and Henyey-Greenstein redirection, until the
 * weight or scatter limit ends the package.  At a wavelength where the
 * sources emit nothing the packages end unborn (counted, no events).
 *  rho_dev       device densities [ncell] (double or float, see precision)
 *  images_dev    device FP64 [comp][n_lambda][frame pixels], overwritten
 *  absorbed_dev  device FP64 [n_lambda][ncell], overwritten; required with
 *                MCRT_ABSORB, else ignored (may be NULL)
 *  stats_host    host mcrt_stats or NULL (non-NULL makes the call wait)
 * Returns 0 or an MCRT_E* code. */
int run_photons(const mcrt_grid *grid, const void *rho_dev, const mcrt_optics *optics, int n_src,
                const mcrt_source *sources, int n_det, const mcrt_detector *detectors, const mcrt_opts *opts,
                double *images_dev, double *absorbed_dev, mcrt_stats *stats_host, void *hip_stream);

/* Straight-line traversal of the grid (Sect. 2.2: packages move through the
 * cells), for a batch of rays o + t k, t >= 0, up to the grid boundary.
 *  origin_dev, dir_dev  device FP64 [n_rays][3]; directions are unit
 *                        vectors (lengths are in units of t)
 *  tau_dev              device FP64 [n_rays]: kappa * sum(rho_m * l_m)
 *  max_seg, seg_cell_dev (int32 [n_rays][max_seg]), seg_len_dev (FP64
 *    [n_rays][max_seg]), n_seg_dev (int32 [n_rays]): optional segment lists
 *    (pass NULL to skip); rays with more than max_seg segments store the
 *    first max_seg, n_seg gets the true count and the call returns
 *    MCRT_EOVERFLOW after finishing all rays.
 *  crossings_host       host uint64 or NULL: total segment count (waits)
 * precision selects the density type and traversal arithmetic. */
int trace_path(const mcrt_grid *grid, const void *rho_dev, double kappa, int precision, int64_t n_rays,
               const double *origin_dev, const double *dir_dev, double *tau_dev, int32_t max_seg,
               int32_t *seg_cell_dev, double *seg_len_dev, int32_t *n_seg_dev, uint64_t *crossings_host,
               void *hip_stream);

/* trace_path for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments, results and errors as trace_path; the call allocates no
 * device memory (no hipMalloc, hipMallocAsync or hipFree): its counters,
 * the plane or tree tables of a rectilinear or tree grid and the bricked
 * copy of the densities live in a library-owned device array of
 * MCRT_NOALLOC_SCRATCH_BYTES bytes, one per device, which each device that
 * the library runs on holds until the process ends.  A grid whose tables and
 * densities need more (about 4 or 8 bytes per cell, FP32 or FP64, plus 256
 * bytes and the tables) is rejected with MCRT_EINVAL before any device
 * work.  Every call on one device uses that device's array and leaves its
 * contents behind: calls that overlap on one device (several streams or
 * host threads) race, and the caller must serialise them.  The counters are
 * cleared by a fill kernel on hip_stream; the tables of a rectilinear or
 * tree grid are copied from host memory the call owns only until it
 * returns, so a capture into a HIP graph should use a regular grid. */
#define MCRT_NOALLOC_SCRATCH_BYTES (96u << 20)

int trace_path_noalloc(const mcrt_grid *grid, const void *rho_dev, double kappa, int precision, int64_t n_rays,
                       const double *origin_dev, const double *dir_dev, double *tau_dev, int32_t max_seg,
                       int32_t *seg_cell_dev, double *seg_len_dev, int32_t *n_seg_dev, uint64_t *crossings_host,
                       void *hip_stream);

/* Peel-off (Sect. 1, Yusef-Zadeh et al. 1984) of a list of events into
 * frames of one wavelength: for every event e and frame d whose pixel
 * contains the projection of pos_e, images[d][pixel] +=
 *   w_e * phase * exp(-tau(pos_e, k_d)) / distance_d^2,
 * with phase = 1/(4 pi) when dir_in_dev is NULL (isotropic emission), else
 * the HG phase function of cos(dir_in_e . k_d) with parameter g.
 *  pos_dev, dir_in_dev  device FP64 [n_events][3]; w_dev FP64 [n_events]
 *  images_dev           device FP64 [frame pixels], accumulated (+=) */
int peel_off(const mcrt_grid *grid, const void *rho_dev, double kappa, double g, int precision, int64_t n_events,
             const double *pos_dev, const double *dir_in_dev, const double *w_dev, int n_det,
             const mcrt_detector *detectors, double *images_dev, void *hip_stream);

/* Gradient of an image loss L with respect to every cell density, for the
 * run that run_photons performs with the same arguments: paths are
 * re-sampled from the same random numbers (never stored) and the detached
 * score-function derivative is accumulated,
 *   dC/drho_m = C [sum_{i<=e} (delta(m, c_i)/rho_m - kappa l_m(leg_i))
 *                  - kappa l_m(peel ray)],
 * for every peel-off contribution C of event e, with c_i the cell of
 * scattering i and leg_i the path from the previous event to it.
 *  adj_images_dev  device FP64 dL/dI in the image layout of run_photons
 *  grad_rho_dev    device FP64 [ncell], overwritten with dL/drho
 *  stats_host      host mcrt_stats or NULL (waits when non-NULL)
 * The absorbed-luminosity tally has no gradient here; MCRT_ABSORB is
 * ignored. */
int backward_density(const mcrt_grid *grid, const void *rho_dev, const mcrt_optics *optics, int n_src,
                     const mcrt_source *sources, int n_det, const mcrt_detector *detectors, const mcrt_opts *opts,
                     const double *adj_images_dev, double *grad_rho_dev, mcrt_stats *stats_host,
                     void *hip_stream);

/* With MCRT_ATTACHED in opts->flags, backward_density (and backward, with
 * grads->rho alone) computes the attached (pathwise) derivative instead: the
 * random numbers are held fixed and the scattering points move with the
 * densities (Sect. 1, forced scattering: the point of each interaction is
 * where the optical depth from the previous event reaches
 * tau_s = -ln(1 - u (1 - e^-T)), u fixed), while every direction (drawn from
 * the random numbers alone) stays.  Each package runs its life cycle once,
 * keeping its events (position, weight, the leg after it: direction,
 * optical depth to the boundary, tau_s, length, density at the next event),
 * then a reverse sweep from the last event back accumulates, for each
 * peel-off contribution q = (dL/dI) C, -q kappa l along its peel ray and
 * its pull on the event's position, and for each leg the terms of T, tau_s
 * and the leg length.  It is the derivative of the per-package estimator
 * itself, so it omits what changes in steps: a contribution that crosses a
 * pixel edge, a peel ray parallel to a grid plane whose origin crosses that
 * plane, a weight that crosses the termination threshold w_min.  Without
 * those (SED instruments seen along directions that no grid plane
 * contains, termination by max_scatter) it is an unbiased gradient of the
 * expected loss, like the detached one, with another variance.
 * The attached gradient is computed in FP64 arithmetic in both precisions
 * (MCRT_PREC_FP32 reads the FP32 densities and widens them): its derivative
 * amplifies the rounding of a point's position wherever a leg grazes a cell
 * face, which FP32 walks would not follow on rough media.
 * Frames and SED instruments only (a perspective camera: MCRT_EINVAL); no
 * absorbed-tally term and no optics gradients (MCRT_EINVAL); a package may
 * have at most MCRT_ATTACHED_MAX_EVENTS events by the bound of
 * mcrt_tape_bytes (else MCRT_EINVAL: lower max_scatter or raise w_min); the
 * tape is not used.  The library keeps a workspace of 88 bytes per event per
 * package of a chunk, and queues the peel rays' deposit walks like the
 * detached gradient (mcrt_opts.peel_queue; -1: every walk inline).  A package that exceeds the bound anyway (not
 * expected) makes the call return MCRT_EOVERFLOW. */

/* Gradients of the same image loss with respect to the densities and to
 * the optical properties and source luminosities of every wavelength
 * (Sect. 2.3: albedo and g; Sect. 2.2: luminosities), in one replay.  The
 * same detached derivative with paths held fixed: a contribution C after n
 * scatterings scales as albedo^n, so dC/dalbedo = n C / albedo; in g it
 * carries the score of every direction sampled before it and of its peel
 * phase, dC/dg = C [sum_i dln Phi(mu_i)/dg + dln Phi(mu_peel)/dg] with
 * dln Phi/dg = -2g/(1 - g^2) - 3(g - mu)/(1 + g^2 - 2 g mu) for HG; and it
 * scales as the luminosity of its package's source (weight L_total / N
 * times choice probability L_s / L_total), dC/dL_s = C / L_s for packages
 * of source s (a cell source: L_s is its total, the derivative that of a
 * uniform scaling of its cells).  Derivatives at albedo = 0 or at a dark
 * source are reported as 0 (no contribution carries them).  Device FP64
 * outputs, each overwritten, each NULL when not wanted:
 *   rho [ncell], albedo [n_lambda], g [n_lambda], lum [n_src][n_lambda].
 * adj_absorbed_dev (device FP64 [n_lambda][ncell], or NULL) adds a term
 * sum b A to the loss, A the absorbed-luminosity tally of run_photons and b
 * = dL/dA: every path's deposits dep_j = W (1 - albedo) e^-tau_{j-1}
 * (1 - e^-dtau_j) (Sect. 1, continuous absorption) carry, with paths held
 * fixed, the density dependence of their weight W (the legs before the
 * path, as a peel-off contribution of the path's event does) and of their
 * own factor: -kappa l_k for each cell k crossed before them and kappa l_j
 * e^-dtau_j / (1 - e^-dtau_j) for their own cell.  It requires rho; the
 * optics gradients stay those of the image term. */
typedef struct {
    double *rho, *albedo, *g, *lum;
} mcrt_grads;

int backward(const mcrt_grid *grid, const void *rho_dev, const mcrt_optics *optics, int n_src,
             const mcrt_source *sources, int n_det, const mcrt_detector *detectors, const mcrt_opts *opts,
             const double *adj_images_dev, const double *adj_absorbed_dev, const mcrt_grads *grads,
             mcrt_stats *stats_host, void *hip_stream);

/* Dust emission (Sect. 1: absorption and re-emission by the dust; Sect. 2.1:
 * panchromatic simulations): the equilibrium temperature and the emission
 * spectrum of every cell from the luminosity it absorbed.  The grains are
 * modified black bodies: cell m of dust mass M_m = rho_m V_m (V_m its
 * volume) at temperature T emits
 *   E_m(T) = emissivity * M_m * sum_i kappa_abs[i] B(lambda[i], T) dlambda[i],
 *   B(lambda, T) = lambda^-5 / (exp(c2 / (lambda T)) - 1),  c2 = 14387.77 um K,
 * and T_m solves E_m(T_m) = L_m, L_m the cell's absorbed luminosity summed
 * over the n_abs rows of absorbed_dev [n_abs][cell] (the absorbed tally of
 * run_photons); T_m is that root within [1, 1e5] K, held at the nearer end
 * when the root lies outside (L_m = 0 or M_m = 0: T_m = 0 and no emission).
 * emission_dev [n_lambda][cell] receives
 *   L_m * kappa_abs[i] B(lambda[i], T_m) dlambda[i]
 *       / sum_j kappa_abs[j] B(lambda[j], T_m) dlambda[j],
 * so every cell re-emits exactly what it absorbed (nothing where that sum
 * underflows to 0).  lambda (um), dlambda
 * (bin widths, um), kappa_abs (absorption opacity per unit density): host
 * arrays [n_lambda], > 0; emissivity > 0 sets the temperature scale only.
 * rho_dev: densities [cell] (double, or float with MCRT_PREC_FP32);
 * temperature_dev [cell] may be NULL.  Cells are numbered as in
 * mcrt_grid.  Device arrays belong to the caller; the call runs on
 * hip_stream without waiting.  Returns 0, MCRT_EINVAL (with a message)
 * for invalid arguments before any device work, or MCRT_EHIP. */
int dust_emission(const mcrt_grid *grid, const void *rho_dev, int precision, int n_abs, const double *absorbed_dev,
                  int n_lambda, const double *lambda, const double *dlambda, const double *kappa_abs,
                  double emissivity, double *temperature_dev, double *emission_dev, void *hip_stream);

/* Message for the last nonzero return on the calling thread ("" if none). */
const char *mcrt_last_error(void);

/* ABI version of this header. */
int mcrt_abi_version(void);

#define MCRT_ABI_VERSION 18

#ifdef __cplusplus
}
#endif

#endif /* MCRT_H */
