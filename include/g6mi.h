/*
 * g6mi.h -- C ABI of libg6mi, a direct-summation gravitational force library
 * for AMD Instinct MI355X (gfx950).
 *
 * For a block of active "i-particles" (the sinks) the library computes,
 * against all "j-particles" (the sources) held in a j-particle memory that
 * it first predicts to the current time, the Plummer-softened Newtonian
 *   acceleration  a_i = sum_j m_j r_ij / (r_ij^2 + eps^2)^{3/2}
 *   jerk          da_i/dt = sum_j m_j [ w_ij / s^{3/2} - 3 (r_ij.w_ij) r_ij / s^{5/2} ]
 *   potential     phi_i = - sum_j m_j / (r_ij^2 + eps^2)^{1/2}
 * (r_ij = x_j - x_i, w_ij = v_j - v_i, s = r_ij^2 + eps^2, G = 1), the
 * nearest neighbour and the neighbour list of each i-particle.  These are
 * the quantities a 4th-order Hermite integrator with block time steps needs
 * from its force step (Gaburov, Harfst & Portegies Zwart 2009, "SAPPORO",
 * Sec. 2 and 2.1); the integrator itself (i-prediction, corrector, time
 * steps) stays with the caller, as in the paper's CPU/GPU split (Sec. 2.1).
 *
 * The g6_* functions follow the GRAPE-6 calling sequence that the paper's
 * library reproduces so that existing GRAPE-6 clients only relink (Sec. 2.5):
 *   g6_open -> g6_set_j_particle (for every corrected particle) -> g6_set_ti
 *   -> g6calc_firsthalf -> [host work] -> g6calc_lasthalf[2]
 *   -> g6_nearest_neighbour / g6_read_neighbour_list -> g6_get_neighbour_list
 * Each also has a Fortran alias (trailing underscore, arguments by address).
 * The g6mi_* functions are extensions: precision variant, launch-shape
 * control, kernel timing and a device-resident path that takes device
 * pointers and a HIP stream.
 *
 * Conventions shared by every function
 *   - Positions, velocities, times and masses are float64 in the client's
 *     units with G = 1.  Arrays declared `double x[][3]` are C row-major,
 *     three consecutive doubles per particle.
 *   - `id` is a handle ("cluster id" in GRAPE-6 terms) in [0, G6MI_MAX_HANDLES);
 *     each open handle owns one independent j-memory on the GPU.
 *   - The caller owns every host array it passes; the library copies what it
 *     needs before returning, so arrays may be reused at once.  The library
 *     owns all GPU memory it allocates.  In the device-resident calls the
 *     caller owns the device buffers it passes and must keep them alive until
 *     the work enqueued on `stream` has completed.
 *   - Nothing aborts or exits.  Functions returning int return 0 on success,
 *     1 for the documented warnings (non-finite output, neighbour-list
 *     overflow), or a negative G6MI_E* code; g6mi_last_error(id) gives text.
 *   - One host thread per handle.  Different handles may be driven from
 *     different threads.
 */
#ifndef G6MI_H
#define G6MI_H

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ constants */


/* Maximum neighbours stored per i-particle (Sec. 4: fixed at build time,
 * default 256). */
#define G6MI_NB_MAX 256
/* Default i-particles per call reported by g6_npipes() (Sec. 2.5, footnote:
 * 256 pipelines).  Larger blocks are accepted up to G6MI_NI_MAX. */
#define G6MI_NPIPES_DEFAULT 256
#define G6MI_NI_MAX (1 << 24)
#define G6MI_NJ_MAX (1 << 26)
#define G6MI_MAX_HANDLES 1024

/* Precision variants of the pair interaction (Sec. 2.2-2.3). */
#define G6MI_PREC_FP32 0 /* float32 positions and arithmetic                */
#define G6MI_PREC_DS   1 /* double-single positions, separation by Eq. (3),
                            float32 arithmetic (the paper's scheme); default */
#define G6MI_PREC_FP64 2 /* float64 throughout                              */

/* Return codes. */
#define G6MI_OK          0
#define G6MI_WARN        1  /* non-finite output, or neighbour-list overflow */
#define G6MI_EINVAL    (-1) /* bad argument, or arguments of lasthalf differ
                               from those of the matching firsthalf          */
#define G6MI_ESTATE    (-2) /* handle not open, or call out of sequence      */
#define G6MI_EDEVICE   (-3) /* no usable GPU, or a HIP runtime error         */
#define G6MI_ENOMEM    (-4) /* GPU or pinned host allocation failed          */

/* One cluster of a batched calculation (g6mi_batch_calc): an independent
 * system whose j-particles are the slots joff .. joff+nj-1 of the handle's
 * j-memory, predicted to the cluster's own time ti, and whose i-particles
 * are the rows ioff .. ioff+ni-1 of the batch's i-arrays.  Each i-particle
 * interacts only with its own cluster's j-slots, softened by the cluster's
 * eps2.  32 bytes, no padding. */
typedef struct g6mi_cluster {
  int joff;    /* first j-slot                                   */
  int nj;      /* number of j-slots (>= 0)                       */
  int ioff;    /* first row in the i-arrays and output arrays    */
  int ni;      /* number of i-particles (>= 0)                   */
  double ti;   /* prediction time of the cluster's j-particles   */
  double eps2; /* softening squared (finite, >= 0)               */
} g6mi_cluster;

/* ------------------------------------------------- GRAPE-6 calling sequence */

/* Create the state of handle `id` on the current HIP device (or the device
 * named by the environment variable G6MI_DEVICE): stream, j-memory and
 * work buffers.  Returns 0, G6MI_EINVAL for a bad id, G6MI_ESTATE if the
 * handle is already open, G6MI_EDEVICE if no GPU is present, G6MI_ENOMEM. */
int g6_open(int id);

/* Release everything handle `id` holds.  Returns 0 or G6MI_ESTATE. */
int g6_close(int id);

/* Number of i-particles a GRAPE-6 client should pass per call: 256, or the
 * value of the environment variable G6MI_NPIPES (1 .. G6MI_NI_MAX). */
int g6_npipes(void);

/* GRAPE-6 fixed-point scale hints.  Accepted and ignored: the library holds
 * positions and times in floating point. */
void g6_set_tunit(int newtunit);
void g6_set_xunit(int newxunit);

/* Store particle `index` in j-memory slot `address` (0 <= address <
 * G6MI_NJ_MAX; the memory grows as needed).  `tj` is the time of its last
 * correction, `mass` its mass, and `x`, `v`, `a2` = a/2, `j6` = jerk/6 its
 * position, velocity and pre-scaled Taylor coefficients at tj, from which
 * it is predicted by Eq. (1) and (2) of Sec. 2.2.  `dtj` (its time step)
 * and `k18` (GRAPE-6's snap term) are accepted and ignored: the predictor
 * stops at the jerk term.  The record is staged on the host and uploaded by
 * the next g6calc_firsthalf.  Particle indices must be unique among the slots
 * used by a calculation; slot `address` is excluded from the forces on the
 * i-particle with the same index.  Returns 0, G6MI_EINVAL or G6MI_ESTATE. */
int g6_set_j_particle(int id, int address, int index, double tj, double dtj,
                      double mass, const double k18[3], const double j6[3],
                      const double a2[3], const double v[3], const double x[3]);

/* g6_set_j_particle for n records at once: record k goes to slot
 * address[k] with particle index index[k], time tj[k], mass[k] and the
 * row-major [n][3] arrays j6 (= jerk/6), a2 (= a/2), v and x.  dtj may be
 * NULL (it is ignored, as in g6_set_j_particle).  All records are checked
 * before any is stored.  Returns 0, G6MI_EINVAL or G6MI_ESTATE. */
int g6mi_set_j_particles(int id, int n, const int address[], const int index[],
                         const double tj[], const double dtj[],
                         const double mass[], const double j6[][3],
                         const double a2[][3], const double v[][3],
                         const double x[][3]);

/* Set the time t_i to which the next calculation predicts the j-particles
 * (tau_j = t_i - t_j in Eq. (1)-(2)). */
void g6_set_ti(int id, double ti);

/* Start a force calculation: upload staged j-records, predict j-slots
 * 0..nj-1 to t_i and compute the forces on the ni i-particles with
 * particle indices `index`, host-predicted positions `xi` and velocities
 * `vi`, softening eps2 (one value for the whole block, Sec. 2.5) and
 * neighbour radii squared h2[i] (a j-particle is a neighbour when its
 * unsoftened squared distance is strictly below h2[i]).  `aold`, `j6old`
 * and `phiold` are GRAPE-6 scaling hints and are ignored (may be NULL).
 * Work is enqueued on the handle's stream and the call returns without
 * waiting.  Returns 0, G6MI_EINVAL (e.g. nj larger than the slots set, ni
 * outside 0..G6MI_NI_MAX, non-finite eps2), G6MI_ESTATE, G6MI_EDEVICE or
 * G6MI_ENOMEM; the error is also returned by the following lasthalf. */
int g6calc_firsthalf(int id, int nj, int ni, const int index[],
                     const double xi[][3], const double vi[][3],
                     const double aold[][3], const double j6old[][3],
                     const double phiold[], double eps2, const double h2[]);

/* Wait for the calculation started by g6calc_firsthalf and write the
 * accelerations, jerks and potentials of its ni i-particles.  nj, ni,
 * index and eps2 must equal those of the firsthalf (G6MI_EINVAL otherwise);
 * xi, vi and h2 are not read again.  Returns 0, 1 if any output is not
 * finite (e.g. eps2 = 0 with two distinct particles at the same position),
 * or a negative error code. */
int g6calc_lasthalf(int id, int nj, int ni, const int index[],
                    const double xi[][3], const double vi[][3], double eps2,
                    const double h2[], double acc[][3], double jerk[][3],
                    double pot[]);

/* As g6calc_lasthalf, and also write the particle index of each
 * i-particle's nearest neighbour (-1 if there is no other j-particle). */
int g6calc_lasthalf2(int id, int nj, int ni, const int index[],
                     const double xi[][3], const double vi[][3], double eps2,
                     const double h2[], double acc[][3], double jerk[][3],
                     double pot[], int nnbindex[]);

/* Nearest neighbour of each of the ni i-particles of the last completed
 * calculation: particle index and unsoftened squared distance (-1 and
 * +infinity if none).  The nearest neighbour minimises the squared distance
 * as computed in the active precision variant; ties go to the lower slot.
 * Returns 0, G6MI_EINVAL (ni differs from the last calculation) or
 * G6MI_ESTATE. */
int g6_nearest_neighbour(int id, int ni, int nnbindex[], double r2nn[]);

/* Copy the neighbour lists of the last completed calculation to the host.
 * When some i-particle had more than G6MI_NB_MAX neighbours, its list is
 * first rebuilt on the GPU from the G6MI_NB_MAX smallest indices (this reads
 * the calculation's i-block again: after g6mi_calc_device its device buffers
 * must still be valid).  Returns 0, 1 if any list overflowed, or a negative
 * error code. */
int g6_read_neighbour_list(int id);

/* Neighbour list of i-particle `ipipe` (0-based position in the last
 * calculation's i-block): particle indices in ascending order.  Writes
 * *nblen = the true number of neighbours and the first
 * min(*nblen, maxlength, G6MI_NB_MAX) indices to nbl.  A list with more
 * than G6MI_NB_MAX neighbours stores the G6MI_NB_MAX smallest particle
 * indices.  Returns 0, 1 if the list was cut by maxlength or G6MI_NB_MAX, or
 * a negative error code (G6MI_ESTATE if g6_read_neighbour_list was not
 * called after the calculation). */
int g6_get_neighbour_list(int id, int ipipe, int maxlength, int *nblen,
                          int nbl[]);

/* ------------------------------------------------------------ extensions */

/* Text of the last error on handle id (or of the last global error when
 * the id is invalid).  The pointer stays valid until the next call on id. */
const char *g6mi_last_error(int id);

/* G6MI_NB_MAX, for callers that load the library dynamically. */
int g6mi_nb_max(void);

/* Select the precision variant (G6MI_PREC_*) for subsequent calculations.
 * The default is G6MI_PREC_DS, or the environment variable G6MI_PRECISION
 * ("fp32", "ds", "fp64") read at g6_open.  Returns 0, G6MI_EINVAL,
 * G6MI_ESTATE. */
int g6mi_set_precision(int id, int prec);
int g6mi_get_precision(int id);

/* Enable (1, default) or disable (0) neighbour-list construction.  With
 * lists disabled the neighbour-list calls report zero neighbours (the
 * paper's build-time switch, Sec. 4).  The nearest neighbour is always
 * computed.  Returns 0 or a negative code. */
int g6mi_set_neighbour_lists(int id, int on);

/* Spatial ordering of double-single calculations: 0 off, 1 (default) for
 * blocks of at least 65536 i-particles against at least 512 j-slots, 2 for
 * every double-single calculation.  With the ordering on, the j-records and
 * the i-block are sorted along a Morton curve of their positions, so that
 * each tile of 256 j-records and each workgroup's 512 i-particles is
 * compact; tiles farther from the i-particles than their own radius use
 * float32 separations of coordinates relative to the tile centre (within
 * four float32 roundings of the separation, against two for Eq. (3)), the
 * other tiles the double-single separation.  Results stay within the same
 * tolerances; nearest-neighbour ties between different records may resolve
 * differently.  In mode 1 a launch-shape override (g6mi_set_shape with
 * i_per_group > 0) turns the ordering off; in mode 2 the ordering uses 512
 * i-particles per workgroup whatever the override.  Returns 0, G6MI_EINVAL
 * or G6MI_ESTATE. */
int g6mi_set_spatial(int id, int mode);

/* Fused prediction for one-block calls (extension; on by default).  When the
 * i-block of a calculation fits one workgroup of the narrow interaction
 * kernel (at most 256 i-particles) and is not spatially ordered, that kernel
 * predicts each j-tile into LDS from the float64 j-memory itself (Sec. 2.2,
 * Eq. (1)-(2), fused into the tile load) instead of reading records written
 * by a separate predictor launch, so the predicted records never go
 * through HBM.  The arithmetic is the same either way and so are the
 * results, bit for bit.  on = 0 always runs the separate predictor.
 * Returns 0, G6MI_EINVAL or G6MI_ESTATE. */
int g6mi_set_fused_predict(int id, int on);

/* Override the launch shape of the interaction kernel: i-particles per
 * workgroup (a power of two, 1..512; 512 means two i-particles per lane,
 * 256 or fewer one per lane or several lanes per i-particle) and number of
 * j-splits (1..4096).  0 restores the automatic choice.  Returns 0 or
 * G6MI_EINVAL. */
int g6mi_set_shape(int id, int i_per_group, int j_splits);

/* Launch shape used by the last calculation: i per workgroup, j-splits,
 * j per tile, workgroups.  Returns 0 or a negative code. */
int g6mi_get_shape(int id, int shape[4]);

/* Enable (1) or disable (0, default) per-kernel timing with HIP events
 * recorded on the launch stream around the predictor, the interaction
 * kernel and the reduction of each calculation (up to 4096 calculations are
 * recorded; enabling again clears the record).  g6mi_last_timing waits for
 * the last timed calculation and writes its kernel times in milliseconds:
 * ms[0] predictor, ms[1] interaction, ms[2] reduction.  g6mi_timing_totals
 * waits for all recorded calculations, writes the sums of their kernel times
 * and their number, and clears the record.  Returns 0 or a negative code. */
int g6mi_enable_timing(int id, int on);
int g6mi_last_timing(int id, double ms[3]);
int g6mi_timing_totals(int id, double ms[3], int *count);

/* Device-resident path.
 *
 * g6mi_set_j_particles_device copies nj j-records from device memory into
 * slots 0..nj-1 of handle id's j-memory: t[nj], mass[nj], index[nj] and
 * row-major [nj][3] x, v, a2 (= a/2) and j6 (= jerk/6), all float64 except
 * index.  The copy is enqueued on `stream` (a hipStream_t; NULL means the
 * handle's own stream) and the handle's host-side index map is refreshed,
 * which synchronises that stream.  Returns 0 or a negative code.
 *
 * g6mi_calc_device predicts j-slots 0..nj-1 to the time set by g6_set_ti and
 * computes the forces on ni i-particles whose data are in device memory:
 * d_islot[i] is the j-slot that holds i-particle i itself (excluded from its
 * sums) or -1; d_xi, d_vi are [ni][3], d_h2 is [ni].  Outputs d_acc, d_jerk
 * ([ni][3]) and d_pot, d_nnb (particle index of the nearest neighbour or -1)
 * and d_r2nn ([ni]) are written in device memory; d_nnb and d_r2nn may be
 * NULL.  Neighbour lists stay in the handle and are read with
 * g6_read_neighbour_list / g6_get_neighbour_list.  All work is enqueued on
 * `stream` without any host synchronisation.  Returns 0 or a negative code
 * (argument errors are detected before anything is enqueued). */
int g6mi_set_j_particles_device(int id, int nj, const double *d_t,
                                const double *d_mass, const int *d_index,
                                const double *d_x, const double *d_v,
                                const double *d_a2, const double *d_j6,
                                void *stream);

int g6mi_calc_device(int id, int nj, int ni, const int *d_islot,
                     const double *d_xi, const double *d_vi, double eps2,
                     const double *d_h2, double *d_acc, double *d_jerk,
                     double *d_pot, int *d_nnb, double *d_r2nn, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, hosts that forbid allocation during a run):
 * g6mi_calc_device_noalloc is g6mi_calc_device with every work buffer of the
 * calculation (predicted records, split partials, neighbour counters and
 * slots, status words, overflow queue) cut from one static device array of
 * G6MI_NOALLOC_SCRATCH_BYTES per GPU instead of the handle's memory.  It
 * calls no hipMalloc, hipFree or other allocating routine; the caller
 * passes inputs and outputs as for g6mi_calc_device, and the j-memory must
 * already hold slots 0..nj-1 on the device (g6mi_set_j_particles_device, or
 * an earlier calculation after g6_set_j_particle).  Differences: the
 * calculation is never spatially ordered, it is not timed, and its j-split
 * count is lowered until the buffers fit.  Returns 0, G6MI_EINVAL (also
 * when the work buffers do not fit even with one j-split: roughly
 * 48 B x nj (DS; 32 B FP32, 64 B FP64; none for a single block of at most
 * 256 i-particles) plus about 1.1 KB x ni), G6MI_ESTATE (j-particles set on
 * the host not uploaded yet, or fewer than nj slots on the device) or
 * G6MI_EDEVICE.  Every call on one GPU shares that GPU's array, which keeps
 * the last call's contents: the neighbour lists read afterwards with
 * g6_read_neighbour_list are those of the last call on that GPU, and calls
 * on one GPU that overlap in time (other streams, other threads or handles)
 * race on it. */
#define G6MI_NOALLOC_SCRATCH_BYTES (64u << 20)
int g6mi_calc_device_noalloc(int id, int nj, int ni, const int *d_islot,
                             const double *d_xi, const double *d_vi, double eps2,
                             const double *d_h2, double *d_acc, double *d_jerk,
                             double *d_pot, int *d_nnb, double *d_r2nn, void *stream);

/* Device properties used by the launch heuristics: compute units and peak
 * engine clock in MHz.  Returns 0 or a negative code. */
int g6mi_device_info(int id, int info[2]);

/* Status flags of the last calculation on handle id (waits for it): bit 0
 * a non-finite output, bit 1 a neighbour list overflowed G6MI_NB_MAX, bit 2
 * (batched calls) a cluster descriptor was invalid and its cluster skipped.
 * Returns 0, G6MI_ESTATE (no calculation) or a negative code. */
int g6mi_last_status(int id, int *flags);

/* --------------------------------------------- batched multi-cluster calls
 *
 * Many independent clusters (GRAPE-6 "cluster ids") evaluated in one
 * launch: the j-particles of every cluster live in the one j-memory of
 * handle id (set as usual with g6_set_j_particle / g6mi_set_j_particles /
 * g6mi_set_j_particles_device), each cluster at its own slots; the
 * i-particles of all clusters are the rows 0 .. ni_total-1 of one set of
 * device arrays, in the layout of g6mi_calc_device (d_islot[r] is the
 * j-slot holding row r's own particle, or -1; d_xi, d_vi [ni_total][3];
 * d_h2 [ni_total]), and so are the outputs (d_acc, d_jerk [ni_total][3],
 * d_pot, d_nnb, d_r2nn [ni_total]; d_nnb and d_r2nn may be NULL).  Row r of
 * cluster c gets, as a separate g6mi_calc_device on that cluster alone
 * would give (up to the order of the force sums: the batch may cut a block
 * into other i-blocks and j-splits), the forces of
 * c's j-slots predicted to c's ti and softened by c's eps2 (Sec. 2.2-2.3),
 * its nearest neighbour among them, and its neighbour list (read afterwards
 * with g6_read_neighbour_list / g6_get_neighbour_list, ipipe = r).
 *
 * A plan kernel, a persistent kernel and a reduction kernel: work items
 * (cluster, i-block, j-split) are taken from a queue, each predicting its
 * j-tiles in on-chip memory; then each i-block's split partials are added
 * and its rows written.  All work
 * is enqueued on `stream` (NULL: the handle's stream) without host
 * synchronisation.  The caller keeps every device buffer valid until the
 * work has completed (and the i-arrays until g6_read_neighbour_list).
 *
 * g6mi_batch_calc takes the ncl descriptors in host memory; they are checked
 * (ranges inside the slots set from slot 0 and inside 0 .. ni_total-1,
 * finite ti and eps2 >= 0, no two clusters sharing an i-row) and copied.
 * Returns 0, G6MI_EINVAL, G6MI_ESTATE, G6MI_EDEVICE or G6MI_ENOMEM.
 *
 * g6mi_batch_calc_device takes them in device memory (d_cl, read when the
 * work runs, so it may be filled by earlier work on the stream); an invalid
 * descriptor is not an error at the call: its cluster is skipped and bit 2
 * of g6mi_last_status is set.  Clusters must not share i-rows. */
int g6mi_batch_calc(int id, int ncl, const g6mi_cluster *cl, int ni_total,
                    const int *d_islot, const double *d_xi,
                    const double *d_vi, const double *d_h2, double *d_acc,
                    double *d_jerk, double *d_pot, int *d_nnb,
                    double *d_r2nn, void *stream);
int g6mi_batch_calc_device(int id, int ncl, const g6mi_cluster *d_cl,
                           int ni_total, const int *d_islot,
                           const double *d_xi, const double *d_vi,
                           const double *d_h2, double *d_acc, double *d_jerk,
                           double *d_pot, int *d_nnb, double *d_r2nn,
                           void *stream);

/* Graph mode (1) or direct launches (0, default) for batched calls.  In
 * graph mode the plan and persistent kernels are captured once into a HIP
 * graph and the graph is replayed by later batched calls whose arguments
 * (pointers, ncl, ni_total, variant, tuning, stream) are all unchanged;
 * descriptor and particle contents may change between replays.  Any change
 * captures a new graph.  Returns 0 or a negative code. */
int g6mi_batch_use_graph(int id, int on);

/* Launch policy of batched calls.
 *   item_work  work per item, in units of a quarter of one j-tile of 256
 *              records against 512 i-particles (1 .. 1024; default 8); a
 *              block below wide_min is also cut into i-blocks of at most
 *              item_work * 128 particles
 *   wide_min   clusters with at least this many i-particles use two
 *              i-particles per lane (default 512); above ni_total, a batch
 *              runs a kernel without the two-per-lane path, whose
 *              registers allow four workgroups per compute unit
 *   wg_per_cu  persistent workgroups per compute unit (0: the kernel's
 *              occupancy, 3, or 2 for float64, or 4 without the
 *              two-per-lane path; 1 .. 8)
 *   max_split  most j-splits per cluster (1 .. 4096; default 64; lowered
 *              so that the partial sums stay within 4 GiB) */
typedef struct g6mi_batch_tuning {
  int item_work;
  int wide_min;
  int wg_per_cu;
  int max_split;
} g6mi_batch_tuning;

/* Set (t = NULL: the defaults) or read the launch policy.  Returns 0 or a
 * negative code. */
int g6mi_batch_set_tuning(int id, const g6mi_batch_tuning *t);
int g6mi_batch_get_tuning(int id, g6mi_batch_tuning *t);

/* Choose the launch policy for batches like the given one.  The key is the
 * device, the precision variant, neighbour lists on/off, ncl and the log2
 * size classes of the batch's pairs, i-particles and j-slots.  When the
 * key is in this process's table or in the text file cache_path (or the
 * file named by the environment variable G6MI_TUNE_CACHE when cache_path is
 * NULL; lines "g6mi-batch-tune-v2 key item_work wide_min wg_per_cu
 * max_split ms", the last line for a key wins) that policy is applied.
 * Otherwise every combination of item_work 1, 2, 4, 8, 16, 32, 64,
 * wide_min 257, 512, 1024, 2^30 and wg_per_cu 1 .. occupancy is timed on
 * this batch (one
 * untimed and `reps` timed runs each, reps <= 0 meaning 3; the output
 * arrays are overwritten), the fastest is applied and appended to the file.
 * The chosen policy is written to *best when best is not NULL.  Returns 0,
 * 1 if the cache file could not be written (the policy is still applied),
 * or a negative code. */
int g6mi_batch_autotune(int id, int ncl, const g6mi_cluster *cl,
                        int ni_total, const int *d_islot, const double *d_xi,
                        const double *d_vi, const double *d_h2,
                        double *d_acc, double *d_jerk, double *d_pot,
                        int *d_nnb, double *d_r2nn, void *stream,
                        const char *cache_path, int reps,
                        g6mi_batch_tuning *best);


/* ------------------------------------------- device-resident block steps
 *
 * The client side of Sec. 2.1 (i-prediction, Hermite corrector, block time
 * steps) run on the GPU, so that a whole block step is one replayed graph
 * of four kernels with no host round trip.  The particles are j-slots
 * 0 .. n-1 of handle id: their t, mass, x, v and index as last set (all t
 * equal); the integrator then owns those slots and updates them in place
 * (position, velocity, a/2, jerk/6, time) after every step.
 *
 * Scheme (the 4th-order Hermite integrator with block steps that the
 * paper's library serves, Sec. 2): block time t_b = min(t_k + dt_k); the
 * particles with t_k + dt_k = t_b are predicted to t_b (Eq. (1)-(2) with
 * their own a and jerk) and get new forces from the batched kernels with
 * softening eps2 and neighbour radius^2 h2; the Makino-Aarseth corrector
 * gives x, v at t_b; the next step is Aarseth's sqrt(eta (|a||a2| + |j|^2) /
 * (|j||a3| + |a2|^2)) with a2 taken at the end of the step, halved while
 * too long but never below dt_min, and doubled (up to dt_max) only when t_b is a
 * multiple of the doubled step; the first step is eta_s |a| / |j| rounded
 * down to a power of two in [dt_min, dt_max].
 *
 * g6mi_hermite_init computes the first forces and steps.  Returns 0, 1 if a
 * force was not finite, or a negative code (G6MI_EINVAL: n larger than the
 * slots set, unequal times, bad parameters).
 *
 * g6mi_hermite_advance performs block steps while the next block time is at
 * most t_end, at most max_steps of them (blocks past t_end are not taken:
 * with dt_max dividing t_end every particle ends exactly at t_end).  Writes
 * the time of the last block taken to *t_reached and the running totals of
 * block steps and particle steps since init to counts[0], counts[1] (either
 * may be NULL).  Returns 0, 1 if a force was not finite, or a negative code
 * (G6MI_ESTATE if not initialised or the j-memory was reallocated since).
 *
 * g6mi_hermite_state waits for the integrator and copies, for slots
 * 0 .. n-1, position, velocity, acceleration, jerk, potential (from each
 * particle's last force evaluation), time and step to the given host arrays
 * (any may be NULL); it also refreshes the host copy of the j-memory.
 * Returns 0 or a negative code. */
int g6mi_hermite_init(int id, int n, double eps2, double h2, double eta,
                      double eta_s, double dt_max, double dt_min);
int g6mi_hermite_advance(int id, double t_end, long long max_steps,
                         double *t_reached, long long counts[2]);
int g6mi_hermite_state(int id, int n, double x[][3], double v[][3],
                       double acc[][3], double jerk[][3], double pot[],
                       double t[], double dt[]);

/* ------------------------------------------------------ Fortran aliases */
int g6_open_(const int *id);
int g6_close_(const int *id);
int g6_npipes_(void);
void g6_set_tunit_(const int *newtunit);
void g6_set_xunit_(const int *newxunit);
void g6_set_ti_(const int *id, const double *ti);
int g6_set_j_particle_(const int *id, const int *address, const int *index,
                       const double *tj, const double *dtj, const double *mass,
                       const double k18[3], const double j6[3],
                       const double a2[3], const double v[3], const double x[3]);
int g6calc_firsthalf_(const int *id, const int *nj, const int *ni,
                      const int index[], const double xi[][3],
                      const double vi[][3], const double aold[][3],
                      const double j6old[][3], const double phiold[],
                      const double *eps2, const double h2[]);
int g6calc_lasthalf_(const int *id, const int *nj, const int *ni,
                     const int index[], const double xi[][3],
                     const double vi[][3], const double *eps2,
                     const double h2[], double acc[][3], double jerk[][3],
                     double pot[]);
int g6calc_lasthalf2_(const int *id, const int *nj, const int *ni,
                      const int index[], const double xi[][3],
                      const double vi[][3], const double *eps2,
                      const double h2[], double acc[][3], double jerk[][3],
                      double pot[], int nnbindex[]);
int g6_nearest_neighbour_(const int *id, const int *ni, int nnbindex[], double r2nn[]);
int g6_read_neighbour_list_(const int *id);
int g6_get_neighbour_list_(const int *id, const int *ipipe,
                           const int *maxlength, int *nblen, int nbl[]);

#ifdef __cplusplus
}
#endif

#endif /* G6MI_H */
