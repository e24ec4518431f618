/*
 * gothic.h - C ABI of the MI355X (gfx950) block-step tree-gravity library.
 *
 * The library evaluates Plummer-softened gravity on the active i-particles of
 * a hierarchical (block) time step with a Barnes-Hut octree, following
 * Miki & Umemura, "GOTHIC: Gravitational oct-tree code accelerated by
 * hierarchical time step controlling" (arXiv:1610.07279):
 *   - Section 1: the softened force a_i = sum_j m_j (r_j - r_i) /
 *     (|r_j - r_i|^2 + eps^2)^{3/2} (G = 1) that the tree approximates;
 *   - Section 2.1: space-filling-curve keys, key sort, breadth-first octree,
 *     pseudo j-particles (mass, centre of mass, enclosing radius b_J);
 *   - Section 2.2: the opening-angle MAC b_J / d <= theta (Barnes & Hut),
 *     and the acceleration (Springel) and multipole (Warren & Salmon) MACs;
 *   - Section 2.3: groups of i-particles sharing one walk through a pseudo
 *     i-particle (r_I, b_I) with d = lambda r_JI, and a small interaction list
 *     flushed when full; Appendix B: the five enclosing balls of the groups;
 *   - Section 2.4: groups split at a critical separation r_crit, tuned by
 *     Brent's method on the measured time;
 *   - Section 2.5: several lanes per i-particle (ij-parallelisation), chosen
 *     per sub-step class if asked (the per-step S left as future work in
 *     Section 4);
 *   - Section 2.6 and Appendix C: reuse of the tree until the growth models
 *     of the walk time say a rebuild pays;
 *   - Section 2.7: block time steps (only particles due at time t are active);
 *   - Section 3.2: the float64 direct sum the force errors are measured against.
 *
 * Conventions for every call:
 *   - Particle arrays are DEVICE pointers owned by the caller.  The library
 *     owns only the scratch inside a context.
 *   - Work is enqueued on the caller's HIP stream (hipStream_t passed as
 *     void*; NULL = the null stream).  Results are valid once that stream has
 *     synchronised.  Calls that return counts synchronise the stream.
 *   - Errors are negative return codes (gothic_status); the thread-local
 *     message is in gothic_last_error().  Nothing aborts.
 *   - Not thread-safe per context: one context serves one host thread (and
 *     its calls run in stream order).
 *   - Units: G = 1.  Outputs are in the caller's particle order.
 *   - Debugging aid: with the environment variable GOTHIC_POISON_ALLOC set
 *     (to anything but "0") when a context grows its scratch, every new
 *     floating-point scratch buffer is first filled with NaN bytes (and the
 *     device synchronised), so results that depended on memory no kernel
 *     wrote would show it.  Off by default; costs one fill per allocation.
 */
#ifndef GOTHIC_H
#define GOTHIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gothic_ctx gothic_ctx;

typedef enum {
  GOTHIC_OK = 0,
  GOTHIC_EINVAL = -1,     /* bad argument (n, eps, theta, pointer, parameter) */
  GOTHIC_ENOMEM = -2,     /* device allocation failed */
  GOTHIC_EDEVICE = -3,    /* a HIP call failed (message says which) */
  GOTHIC_EOVERFLOW = -4,  /* node or frontier capacity still exceeded after growing */
  GOTHIC_ECAPTURE = -5,   /* scratch would have to grow during stream capture */
  GOTHIC_ENONFINITE = -6  /* NaN or Inf in the positions or masses */
} gothic_status;

typedef enum { GOTHIC_KEY_MORTON = 0, GOTHIC_KEY_PEANO_HILBERT = 1 } gothic_key_kind;

/* Tunables.  Fill with gothic_default_params() and override fields. */
typedef struct {
  int key_kind;       /* GOTHIC_KEY_MORTON (default) or GOTHIC_KEY_PEANO_HILBERT
                         (Appendix A); both give the same cells, in a different
                         order */
  int n_leaf;         /* a node with more than n_leaf particles is split
                         (1..64; default 16) */
  int multipole;      /* 1 = monopole pseudo particles (Section 2.1),
                         2 = monopole + quadrupole node terms (extension) */
  int group_size;     /* G: i-particles per group sharing one walk; a power of
                         two in 1..64 (default 32) */
  int list_depth;     /* per-wave LDS interaction-list budget in 16-byte slots,
                         a multiple of 64 in 64..1024 (default 384): monopole
                         entries take one slot; with quadrupole nodes half the
                         budget holds particles and half holds node entries
                         (three slots each) */
  int compensated;    /* 1: Neumaier-compensated accumulation of the per-flush
                         partial sums; 0: plain FP32 (default 1) */
  int check;          /* 1: every force call synchronises its stream at the end,
                         checks the device error flags, grows scratch and
                         repeats (up to five times) on overflow; 0: fully
                         asynchronous, flags are reported by the next
                         gothic_get_stats() (default 1) */
  int timing;         /* 1: record HIP events around every walk launch on the
                         call's stream; gothic_get_walk_time() sums them
                         (default 0) */
  float r_crit;       /* critical separation of Section 2.4: two consecutive
                         active particles (key order) farther apart than r_crit
                         never share a group; > 0 absolute length, 0 = no split,
                         < 0 a fraction of the key-cube side L of the
                         particle's system (default -1/16, i.e. L/16) */
  int graph;          /* 1: with check = 0, gothic_sim_step replays one captured
                         HIP graph of the whole sub-step (predict, keys, sort,
                         tree, moments, groups, walk, correct) instead of
                         launching some two hundred kernels; it is captured on
                         first use and again after any buffer or parameter
                         change (default 0) */
  int autotune;       /* 1: gothic_sim_step tunes r_crit while it runs, as in
                         Section 2.4: the walk time of each sub-step is
                         minimised over r_crit with Brent's method, searching
                         log2(r_crit / L) in [-12, 0] (r_crit a fraction of each
                         system's key-cube side L), and every finished search
                         is followed by a new one on a narrower bracket about
                         its best point (the perturbation that follows a
                         drifting optimum).  One search per class of
                         sub-steps with the same due levels.  Synchronises on
                         the previous sub-step's walk.  2: as 1, after first
                         picking the group shape (group size and walk width)
                         of each class by timing (gothic_sim_set_group_sizes)
                         (default 0) */
  int rebuild_interval; /* tree reuse (Section 2.6): 1 = build a new tree for
                         every evaluation (default); k > 1 = build one every
                         k evaluations and walk the last one in between, with
                         the current positions (moments, radii, groups and
                         walk are always recomputed, so every evaluation is an
                         exact Barnes-Hut evaluation of its tree); 0 =
                         automatic: rebuild when the paper's growth models of
                         the walk time (linear, power law, parabolic, chosen
                         by reduced chi^2) say the mean cost per step is
                         minimal; synchronises on the previous evaluation's
                         walk.  With k != 1 the caller must pass the same
                         particles (same order) on the same systems between
                         rebuilds; a change of n or of the systems always
                         rebuilds */
  int mac;            /* multipole acceptance criterion (Section 2.2):
                         0 = opening angle b_J <= theta d (default);
                         1 = acceleration MAC: d^4 >= m_J b_J^2 / (mac_delta
                             |a_old|), |a_old| the smallest previous
                             acceleration in the group (needs
                             gothic_tree_forces_ex or the block-step driver);
                         2 = multipole MAC of Warren & Salmon: d >= b_J/2 +
                             sqrt(b_J^2/4 + sqrt(3 B2 / mac_delta)), B2 = sum
                             m |r - r_J|^2.
                         With 1 and 2 theta is not used, and a node of positive
                         size is never accepted when b_J >= d (it may hold a
                         member of the group) */
  float mac_delta;    /* accuracy of mac 1 (dimensionless) and mac 2 (an
                         acceleration); > 0 (default 2^-7) */
  int ball;           /* enclosing ball of each group's pseudo i-particle
                         (Appendix B): 0 GEO, centred on the bounding box
                         (default); 1 SEB, the smallest enclosing ball; 2 EBS,
                         Ritter's sphere; 3 COM, centred on the centre of mass;
                         4 CMP, the smaller of GEO and COM.  The radius is the
                         largest member distance from the centre */
  int64_t node_capacity; /* initial size of the node arrays in nodes; 0 = from
                         n and n_leaf (about n + 8 n / n_leaf).  Trees that do
                         not fit are abandoned on the device, the arrays grow
                         (at least 2x) and the evaluation repeats (check
                         mode). */
  int64_t max_scratch_bytes; /* cap on the device scratch one context holds, in
                         bytes; 0 = no cap.  A call that would grow the scratch
                         past it returns GOTHIC_ENOMEM, and gothic_get_scratch
                         reports the size it needed */
  int spill_per_wave; /* initial capacity of each walk wave's global pending-node
                         stack (Section 2.3 keeps the pending nodes of a walk in
                         small buffers), in entries: 0 = 16384, else 256..2^24.
                         A walk that outgrows it drops the children it cannot
                         hold and sets the frontier-overflow flag; check mode
                         then grows it 4x and repeats the evaluation */
  int walk_width;     /* W: lanes that share one tree traversal (the paper's
                         T_sub, Table 2): 64 = one group per wave64 (default;
                         0 means 64), 16 or 32 = 64 / W groups walked side by
                         side in one wave, each by its own W lanes with its own
                         pending stack and a 1/(64/W) share of the wave's
                         list budget.  group_size must not exceed W; each
                         i-particle gets S = W / group_size lanes */
} gothic_params;

/* Statistics of the last force evaluation (filled by gothic_get_stats). */
typedef struct {
  int64_t n;              /* particles */
  int64_t n_active;       /* active i-particles */
  int64_t n_nodes;        /* tree nodes */
  int64_t n_groups;       /* i-particle groups */
  int64_t n_levels;       /* deepest tree level + 1 */
  int64_t node_entries;   /* sum over groups of accepted node list entries */
  int64_t part_entries;   /* sum over groups of particle list entries */
  int64_t interactions;   /* sum over active i of its list length */
  int64_t node_interactions; /* the part of interactions that are node terms */
  int64_t mac_tests;      /* MAC evaluations over all groups */
  int32_t flags;          /* device error flags (bit 0 non-finite input, bit 1
                             node overflow, bit 2 frontier overflow, bit 3 an
                             internal index check failed) */
  int32_t n_systems;      /* non-empty systems of the evaluation (1 unless
                             batched) */
  int32_t sticky_flags;   /* the flags above ORed over every evaluation of the
                             context since its creation or the last
                             gothic_clear_flags() (repeats after growing in
                             check mode excepted: their first attempt's
                             overflow was handled); with check = 0 this is how
                             an overflow in any but the last evaluation shows */
} gothic_stats;

/* Default tunables (see gothic_params). */
void gothic_default_params(gothic_params *p);

/* Create a context on HIP device `hip_device`.  p = NULL takes the defaults.
 * Returns GOTHIC_OK and *out, or an error (EINVAL for bad parameters,
 * EDEVICE when the device cannot be used). */
int gothic_create(gothic_ctx **out, int hip_device, const gothic_params *p);

/* Release the context and all its device scratch.  NULL is accepted. */
int gothic_destroy(gothic_ctx *c);

/* Replace the tunables of a context (validated as in gothic_create). */
int gothic_set_params(gothic_ctx *c, const gothic_params *p);
int gothic_get_params(const gothic_ctx *c, gothic_params *p);

/*
 * One tree-force evaluation (Sections 2.1-2.3, 2.5).
 *   n        number of particles, 0 <= n < 2^31 (n = 0 does nothing)
 *   xyzm     [n][4] float: x, y, z, m of every j-particle (masses >= 0)
 *   eps      Plummer softening length, finite and > 0
 *   theta    opening angle of the MAC, 0 <= theta < 1 (theta = 0 gives the
 *            direct sum through the tree)
 *   active   [n] uint8: nonzero = this particle is an i-particle of the step;
 *            NULL = all particles are active
 *   acc_pot  [n][4] float out: ax, ay, az, phi for active rows; rows with
 *            active == 0 are not written.  phi excludes the self pair.
 *   stream   hipStream_t or NULL
 * Returns GOTHIC_OK, or EINVAL / ENONFINITE / EOVERFLOW / ENOMEM / EDEVICE
 * (the last three only in check mode, or from gothic_get_stats otherwise).
 * xyzm and acc_pot must not overlap.
 */
int gothic_tree_forces(gothic_ctx *c, int64_t n, const float *xyzm, float eps, float theta,
                       const uint8_t *active, float *acc_pot, void *stream);

/*
 * Many independent systems in one evaluation: every kernel of the pipeline is
 * launched once for all systems (one walk launch over the groups of every
 * system).  System s owns particles [offsets[s], offsets[s+1]) of xyzm,
 * active and acc_pot, with its own softening eps[s] and angle theta[s]; each
 * system gets its own key cube, keys, tree (root = node s of the combined
 * breadth-first numbering, counting non-empty systems only) and groups, and
 * its forces are those of gothic_tree_forces on that system alone.
 *   nsys     1 <= nsys <= 65535
 *   offsets  HOST int64 [nsys + 1]: offsets[0] = 0, non-decreasing, total
 *            below 2^31 (empty systems are allowed and skipped)
 *   eps, theta  HOST float [nsys], each as in gothic_tree_forces
 * Same pointer and error rules as gothic_tree_forces.
 */
int gothic_tree_forces_batched(gothic_ctx *c, int nsys, const int64_t *offsets,
                               const float *xyzm, const float *eps, const float *theta,
                               const uint8_t *active, float *acc_pot, void *stream);

/*
 * The general evaluation: nsys systems as in gothic_tree_forces_batched, plus
 *   acc_old  [n][4] float DEVICE (ax, ay, az, unused) previous accelerations
 *            in the caller's order, read by the acceleration MAC (mac = 1;
 *            may be NULL otherwise), e.g. the acc_pot of the last step
 * Same rules as gothic_tree_forces_batched; EINVAL when mac = 1 and acc_old
 * is NULL.  acc_old may not overlap acc_pot.
 */
int gothic_tree_forces_ex(gothic_ctx *c, int nsys, const int64_t *offsets, const float *xyzm,
                          const float *eps, const float *theta, const uint8_t *active,
                          const float *acc_old, float *acc_pot, void *stream);

/*
 * Scratch-free variant of gothic_tree_forces, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and argument
 * errors as gothic_tree_forces, with these differences:
 *   - no device or pinned memory is allocated or freed by the call: all
 *     scratch lives in one fixed array of 256 MiB per GPU (a file-scope
 *     __device__ array, looked up when a context is created on that GPU and
 *     held until the process ends).  n is limited by it: about 5e5
 *     particles at n_leaf = 16; a larger n returns GOTHIC_ENOMEM and
 *     gothic_get_scratch() reports the bytes it needed.  The context's own
 *     scratch is neither used nor changed.
 *   - never synchronises (params.check is ignored); device errors (non-finite
 *     input, node or pending-stack overflow) are reported by the next
 *     gothic_get_stats(), which returns GOTHIC_ENONFINITE / GOTHIC_EOVERFLOW.
 *     The pending stack holds params.spill_per_wave entries per walk wave
 *     (0: 4096); the node arrays hold params.node_capacity nodes (0: about
 *     n + 8 n / n_leaf).
 *   - always builds a new tree (params.rebuild_interval and autotune do not
 *     apply); the acceleration MAC (mac = 1) returns EINVAL.
 *   - every scratch-free call on one GPU shares the array and leaves its
 *     contents behind (the next call clears what must start at zero): calls
 *     that may overlap in time on one GPU (other streams, other host threads,
 *     other contexts) race and must be ordered by the caller.  The read-back
 *     calls (gothic_get_stats, gothic_get_keys, ...) after a scratch-free call
 *     read that array, valid until the next scratch-free call on the GPU.
 */
int gothic_tree_forces_noalloc(gothic_ctx *c, int64_t n, const float *xyzm, float eps,
                               float theta, const uint8_t *active, float *acc_pot,
                               void *stream);

/* Result of gothic_autotune. */
typedef struct {
  int group_size;         /* chosen G */
  int list_depth;         /* chosen list budget */
  float r_crit;           /* chosen critical separation (< 0: fraction of each
                             system's key-cube side) */
  int evaluations;        /* timed evaluations spent; 0 = taken from the cache */
  double ms;              /* best measured time of one evaluation (ms) */
  int walk_width;         /* chosen W (16, 32 or 64) */
} gothic_tune_result;

/*
 * Softened direct summation in float64 (Section 1: the Plummer-softened
 * acceleration and potential with G = 1, as the tree force approximates
 * them), the reference that the accuracy of the tree force is measured
 * against (Section 3.2, Fig. 3).  Independent of the tree: every pair is summed.
 *   n        particles, 1 <= n < 2^31 (with ni = 0 any n in [0, 2^31))
 *   xyzm     [n][4] float DEVICE: x, y, z, m of every j-particle
 *   eps      Plummer softening length, finite and > 0
 *   ni       targets, 0 <= ni < 2^31
 *   idx      [ni] int64 DEVICE: the particle of each target; NULL = targets
 *            0 .. ni-1 (then ni <= n).  An index outside [0, n) gives a NaN row.
 *   acc_pot  [ni][4] double DEVICE out: ax, ay, az, phi of each target; the
 *            pair j = idx[k] is left out (another particle at the same
 *            position adds no force and -m/eps to phi)
 * Every target costs n pair terms; the j-particles are split into chunks whose
 * float64 partials are added in a fixed order, so the result is the same on
 * every call.  The partials live in context scratch of (chunks x ni) x 32
 * bytes, grown on demand (ECAPTURE when it would grow inside stream capture).
 * Returns GOTHIC_OK, EINVAL, ENOMEM or EDEVICE.
 */
int gothic_direct_forces(gothic_ctx *c, int64_t n, const float *xyzm, float eps, int64_t ni,
                         const int64_t *idx, double *acc_pot, void *stream);

/*
 * Timed search for the fastest tunables of one workload (Section 2.4 tunes
 * r_crit by Brent's method on the measured time; here the group size G, the
 * walk width W and the list budget are searched as well): every shape (G, W)
 * in (8, 64), (16, 64), (32, 64), (64, 64), (4, 16), (8, 16), (8, 32),
 * (16, 32) with every list_depth in {128, 256, 384, 512, 768} at the current
 * r_crit, then Brent's method over log2(r_crit / L) in [-12, 0] at the best
 * triple.  Each
 * candidate is one whole evaluation timed with HIP events (after an untimed
 * one).  The winner is stored in the context's parameters and cached under
 * (batched or not, floor(log2 n), floor(log2(n / n_active)), multipole); a
 * later call in the same bucket costs one evaluation.  Arguments as in
 * gothic_tree_forces_batched (nsys = 1 for one system); acc_pot receives the
 * forces of a final checked evaluation with the chosen tunables.
 * Synchronises.  Returns as gothic_tree_forces, and EINVAL for a NULL out or
 * with the acceleration MAC (mac = 1), which needs previous accelerations.
 */
int gothic_autotune(gothic_ctx *c, int nsys, const int64_t *offsets, const float *xyzm,
                    const float *eps, const float *theta, const uint8_t *active,
                    float *acc_pot, gothic_tune_result *out, void *stream);

/* Sum of the walk-kernel durations recorded since the previous call (timing
 * = 1; up to 4096 launches are kept), in milliseconds, and their number.
 * Synchronises on the recorded events. */
int gothic_get_walk_time(gothic_ctx *c, double *ms_total, int64_t *launches);

/*
 * Block time-step driver (Section 2.7): RK2 predictor for every particle,
 * tree forces for the particles due at the new time, RK2 corrector and new
 * time levels for them, all on the device in float64 (forces in float32).
 * Readings (the paper gives no criterion): dt_i = eta sqrt(eps / |a_i|);
 * steps dt_max / 2^k, k = 0..kmax; dt_fine = largest power of two <= min dt_i
 * at t = 0 and dt_max = dt_fine 2^kmax; a particle takes the coarsest level
 * whose step fits; it may move to any finer level after a correction and one
 * level coarser when the sub-step is a multiple of that coarser step.
 *   pos, vel   [n][3] double DEVICE arrays owned by the caller, updated in
 *              place (each particle holds its state at its last update time)
 *   mass       [n] float DEVICE array (masses >= 0)
 *   shared_step  1: every particle on the finest level every sub-step (the
 *              scheme is then the leap-frog of the paper's shared-step runs)
 * gothic_sim_bind computes the t = 0 forces and levels and synchronises
 * (with the acceleration MAC, whose a_old does not exist yet at t = 0, the
 * t = 0 forces use the opening angle theta; every sub-step then uses each
 * particle's last acceleration).
 * gothic_sim_step advances one finest sub-step and is asynchronous (check
 * mode synchronises inside the force evaluation).  The arrays must stay
 * valid until the next bind or gothic_destroy.  Each sub-step ends by
 * predicting the positions of the next one (the first is predicted by the
 * bind), so a change a caller makes to pos or vel between two calls reaches
 * the forces one sub-step later.
 */
typedef struct {
  int64_t n;
  int64_t substep;             /* finest sub-steps since t = 0 */
  double t, dt_fine, dt_max;
  int64_t steps;               /* sub-steps since bind or the last counter reset */
  int64_t last_active;         /* due particles of the last sub-step */
  int64_t active_total;        /* summed over the counted sub-steps */
  int64_t interactions_total;  /* list entries x i-particles, summed likewise */
  int64_t node_interactions_total;
  int64_t tree_builds;         /* sub-steps that built a new tree, counted likewise
                                  (all of them unless rebuild_interval != 1) */
  int64_t level_count[32];     /* particles per level now */
} gothic_sim_info;

int gothic_sim_bind(gothic_ctx *c, int64_t n, double *pos, double *vel, const float *mass,
                    float eps, float theta, double eta, int kmax, int shared_step, void *stream);
/* nsys independent systems stepped together (arguments as in
 * gothic_tree_forces_batched, no empty systems): each has its own dt_fine and
 * dt_max (from its own minimum step) and advances one of its own finest
 * sub-steps per gothic_sim_step; the forces of a sub-step are one batched
 * evaluation. */
int gothic_sim_bind_batched(gothic_ctx *c, int nsys, const int64_t *offsets, double *pos,
                            double *vel, const float *mass, const float *eps,
                            const float *theta, double eta, int kmax, int shared_step,
                            void *stream);
int gothic_sim_step(gothic_ctx *c, void *stream);
int gothic_sim_reset_counters(gothic_ctx *c, void *stream);
int gothic_sim_get_info(gothic_ctx *c, gothic_sim_info *out);
/* acc_pot [n][4] float (last forces), levels [n] uint8, last [n] int64 (sub-step
 * of each particle's last update): caller DEVICE buffers, NULL skips. */
int gothic_sim_get_state(gothic_ctx *c, float *acc_pot, uint8_t *levels, int64_t *last);
/* dt_fine and dt_max of every bound system: HOST double arrays of nsys
 * entries (gothic_sim_info reports system 0).  Synchronises. */
int gothic_sim_get_steps(gothic_ctx *c, int nsys, double *dt_fine, double *dt_max);
/* Online tuning (params.autotune): for each sub-step class c = 0..nclass-1
 * (class c = sub-steps whose index has its lowest set bit at c, capped at
 * kmax), the best r_crit of the last finished search (0 if none finished
 * yet), the number of finished searches, and the group size and walk width
 * the class walks with now (params.group_size / params.walk_width until a
 * shape is fixed or picked).  HOST arrays; any may be NULL.
 * 0 <= nclass <= 32. */
int gothic_sim_get_tuning(gothic_ctx *c, int nclass, float *r_crit_best, int *searches,
                          int *group_size, int *walk_width);
/* Group shape per sub-step class (Section 4 names choosing the number of
 * threads per i-particle, S, for each step as future work; a group of G
 * i-particles is walked by W lanes with S = W / G lanes each, so this chooses
 * S and the walk width per class).
 * group_size: HOST int [nclass], each 0 (the class follows params.group_size
 * and params.walk_width) or a power of two in 1..64; walk_width: HOST int
 * [nclass], each 16, 32 or 64 (0 = 64) and at least the class's group size,
 * or NULL for 64 throughout.  Classes >= nclass keep their setting.
 * params.autotune = 2 picks the shape of each class whose entry is 0 by
 * timing (G, W) = (8, 64), (16, 64), (32, 64), (64, 64), (4, 16), (8, 16),
 * (8, 32), (16, 32) on its first sub-steps.  The binding of a system
 * (gothic_sim_bind*) clears the table.  Returns EINVAL for a bad entry
 * (nothing is changed). */
int gothic_sim_set_group_sizes(gothic_ctx *c, int nclass, const int *group_size,
                               const int *walk_width);

/* Counts of the last evaluation; synchronises the stream of that call. */
int gothic_get_stats(gothic_ctx *c, gothic_stats *out);

/* Clear the sticky flags (and those of the last evaluation) on `stream`. */
int gothic_clear_flags(gothic_ctx *c, void *stream);

/* Device scratch: *held = bytes the context holds now; *required = bytes a
 * refused call needed (GOTHIC_ECAPTURE under stream capture, or GOTHIC_ENOMEM
 * from params.max_scratch_bytes), 0 after a call that did not need to grow.
 * Either pointer may be NULL.  Host-side only; never synchronises. */
int gothic_get_scratch(gothic_ctx *c, int64_t *held, int64_t *required);

/*
 * Introspection of the last evaluation, for bit-exact tests.  All outputs are
 * caller-owned DEVICE buffers sized from gothic_get_stats; any pointer may be
 * NULL to skip it.  Each call synchronises.
 *   keys_sorted [n] uint64 and perm [n] uint32: the stable key sort
 *     (perm[k] = caller index of the k-th particle in key order; with several
 *     systems the order is by system first, each within its own range)
 *   cube [n_systems][4] double: x_min, y_min, z_min, side L of the key cube
 *     of each non-empty system
 *   tree [n_nodes] arrays in breadth-first order: first particle (in key
 *     order), particle count, first child, number of children, level
 *   nodes: com_m [n_nodes][4] float (centre of mass, mass), b [n_nodes] float
 *     (enclosing radius), quad [n_nodes][6] float second moments about the
 *     centre of mass (xx, yy, zz, xy, xz, yz; zero unless multipole = 2)
 *   groups: alist [n_active] uint32 (key-order indices of the active
 *     particles), gfirst/gcount [n_groups] into alist, ball [n_groups][4]
 *     float (r_I, b_I), entries [n_groups][2] uint32 (node and particle list
 *     entries of the group's walk)
 *   positions: xyzm_sorted [n][4] float, the positions and masses the moments,
 *     groups and walk used, in key order (for a block sub-step the float32
 *     prediction of Section 2.7, masses non-negative)
 */
int gothic_get_keys(gothic_ctx *c, uint64_t *keys_sorted, uint32_t *perm, double *cube);
int gothic_get_tree(gothic_ctx *c, int64_t *n_nodes, uint32_t *first, uint32_t *count,
                    uint32_t *child_first, uint8_t *n_child, uint8_t *level);
int gothic_get_nodes(gothic_ctx *c, float *com_m, float *b, float *quad);
int gothic_get_positions(gothic_ctx *c, float *xyzm_sorted);
int gothic_get_groups(gothic_ctx *c, int64_t *n_active, int64_t *n_groups, uint32_t *alist,
                      uint32_t *gfirst, uint32_t *gcount, float *ball, uint32_t *entries);
/* (n_nodes, n_active, n_groups: HOST int64 out-parameters, NULL skips.) */

/*
 * Interaction lists of chosen groups of the last evaluation (Sections 2.2-2.3:
 * the nodes a group's walk accepted as pseudo j-particles and the leaves it
 * opened into their particles), for checking the walk's decisions.  The walk
 * of each listed group is run again on the stored tree, groups and positions
 * with the same kernel code, so its decisions and forces are those of the
 * evaluation.
 *   ngsel    number of groups, 0..2^20; gsel HOST uint32 [ngsel] group indices
 *            (< n_groups of the last evaluation)
 *   cap      entries kept per group (1..2^26)
 *   entries  DEVICE uint32 [ngsel][cap]: per group, in the order decided, an
 *            accepted node J as J and an opened leaf J as J | 0x80000000
 *            (node indices as in gothic_get_tree); entries past cap are
 *            counted but not stored
 *   counts   DEVICE uint32 [ngsel][2]: accepted nodes, opened leaves
 *   acc_pot  DEVICE float [n][4]: the rows of the listed groups' particles are
 *            written (the same values the evaluation wrote)
 * Not for the scratch-free entry point's evaluations.  Synchronises.  Returns
 * EINVAL for bad arguments or no evaluation, EOVERFLOW when the last
 * evaluation overflowed.
 */
int gothic_get_lists(gothic_ctx *c, int64_t ngsel, const uint32_t *gsel, int64_t cap,
                     uint32_t *entries, uint32_t *counts, float *acc_pot);

/* Message of the last failed call on this host thread ("" if none). */
const char *gothic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GOTHIC_H */
