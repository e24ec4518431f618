// Internal declarations shared by the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/gothic.h"
#include "tune.h"

namespace gothic {

constexpr int kNlev = 21;         // bits per axis of a key (63-bit keys)
constexpr int kMaxLevels = kNlev + 1;
constexpr int kWave = 64;         // gfx950 wavefront width

// Device error flags (Ctl::flags)
constexpr unsigned kFlagNonFinite = 1u;
constexpr unsigned kFlagNodeOverflow = 2u;
constexpr unsigned kFlagSpillOverflow = 4u;
constexpr unsigned kFlagBadIndex = 8u;  // an index failed its range check (a bug)
constexpr unsigned kFlagMask = 15u;

constexpr int kXworkStride = 32;  // unsigned words per claim counter (128 bytes)

// Device-resident control block: every count the pipeline needs lives here so
// no kernel launch depends on a host read-back.
struct Ctl {
  unsigned flags;
  unsigned sticky;                     // flags of earlier evaluations, ORed (kept by resets)
  unsigned n_nodes;
  unsigned n_active;
  unsigned n_groups;
  unsigned lvl_start[kMaxLevels + 2];  // nodes of level l: [lvl_start[l], lvl_start[l+1])
  unsigned nsys;                       // systems of the evaluation (roots 0 .. nsys-1)
  // per-XCD group counters of the persistent walk, each on a 128-byte line
  // of its own (counter x at index kXworkStride x, the first line after the
  // fields above) so that the XCDs' claims neither queue on one line nor
  // share one with the fields every wave reads
  alignas(128) unsigned xwork[8 * kXworkStride];
  unsigned scan_total;                 // scratch: total of the last scan
  unsigned tree_ok;                    // the last build finished without overflow
  unsigned pad1;
  unsigned long long node_entries;     // summed over groups
  unsigned long long part_entries;
  unsigned long long interactions;     // summed over active i
  unsigned long long node_interactions;
  unsigned long long mac_tests;
};

// One independent system of a (batched) evaluation.  Its particles are the
// index range [soff[s], soff[s+1]) both in the caller's order and in key order
// (the sort orders by system first), and its tree root is node s.
struct SysRec {
  double cube[4];               // x_min, y_min, z_min, L of its bounding cube
  float eps2, theta, inv_eps;   // softening^2, opening angle, 1/softening
  float pad;
};

// Largest s with soff[s] <= k (k inside [soff[0], soff[nsys])): binary search
// over the system offsets, which stay in the caches.
__device__ __forceinline__ unsigned sys_of(const uint32_t *__restrict__ soff, unsigned nsys,
                                           uint32_t k) {
  unsigned lo = 0, hi = nsys;  // soff[lo] <= k < soff[hi]
  while (hi - lo > 1) {
    const unsigned mid = (lo + hi) >> 1;
    if (soff[mid] <= k) lo = mid; else hi = mid;
  }
  return lo;
}

struct Buffers {
  // particles (capacity cap_n)
  uint64_t *keyA = nullptr, *keyB = nullptr;
  uint32_t *idxA = nullptr, *idxB = nullptr;
  float4 *pos = nullptr;          // xyzm in key order
  uint32_t *leaf_of = nullptr;    // leaf node of each key-ordered particle
  uint32_t *flag = nullptr;       // active flag of each key-ordered particle (n)
  uint32_t *flag2 = nullptr;      // scan output scratch (n)
  uint32_t *alist = nullptr;      // key-order indices of active particles
  uint32_t *gA = nullptr, *gB = nullptr;  // group-formation scratch (n)
  uint32_t *gfirst = nullptr;     // first active index of each group, [n_groups + 1]
  // nodes (capacity cap_nodes)
  uint32_t *first = nullptr, *count = nullptr, *child_first = nullptr, *parent = nullptr;
  uint8_t *n_child = nullptr, *level = nullptr;
  uint32_t *nch = nullptr;        // per level-node child counts / offsets (n)
  uint32_t *bnd = nullptr;        // per level-node child boundaries, 8 each (8 n)
  float4 *nrec = nullptr;         // walk record, 2 per node: (x,y,z,M), (b_J, a, b, leaf)
  float4 *quad = nullptr;         // 2 per node: (xx,yy,zz,xy), (xz,yz,tr,0)
  float *mcrit = nullptr;         // per node: critical distance of the multipole MAC
  float *amag = nullptr;          // |a_old| of each key-ordered particle (acceleration MAC)
  float *gamin = nullptr;         // smallest |a_old| of each group
  // ancestors (capacity cap_anc particles): anc[l * n + k] is the level-l
  // ancestor of key-ordered particle k, for l < leaflev[k] (its leaf's level)
  uint32_t *anc = nullptr;
  uint8_t *leaflev = nullptr;
  // groups (capacity cap_groups)
  float4 *ball = nullptr;
  uint32_t *gent = nullptr;       // 2 per group: node entries, particle entries
  // sort / scan scratch
  uint32_t *hist = nullptr;       // radix histograms
  uint32_t *part = nullptr;       // scan partials
  float *bbox_part = nullptr;     // bbox partials
  // walk spill area (per wave: the older part of the pending-node stack)
  uint32_t *spill = nullptr;
  // per-group list read-back (gothic_get_lists): work list of groups and
  // the recorded entries; null outside that call
  const uint32_t *gsel = nullptr;
  unsigned ngsel = 0;
  uint32_t *rec = nullptr, *rec_n = nullptr;
  int64_t rec_cap = 0;
  // systems (capacity cap_sys)
  SysRec *sys = nullptr;
  uint32_t *soff = nullptr;       // [nsys + 1] particle offsets
  // control
  Ctl *ctl = nullptr;
  Ctl *ctl_host = nullptr;        // pinned mirror for read-back
  float *rcrit = nullptr;         // r_crit of the evaluation (device, set before each one)
};

// The systems of one evaluation, non-empty ones only (host side).
struct Systems {
  int nsys = 0;
  int64_t n = 0, max_n = 0;
  std::vector<int64_t> off;  // nsys + 1
  std::vector<float> eps, theta;
};

// Block-step driver state on the device (sim.hip)
struct SimCtl {
  long long s;                  // current finest sub-step
  double eta;
  int kmax, shared;
  unsigned long long n_active;  // due particles of the step in progress
  unsigned long long n_next;    // due particles of the next step (counted while predicting it)
  unsigned long long last_active, steps, inter_total, node_inter_total, active_total;
  unsigned long long level_count[32];
};

// Per-system clock of the block-step driver: every system advances one of
// its own finest sub-steps per driver step.
struct SimSys {
  double dt_fine, dt_max, eps;
  unsigned long long min_dt_bits;
};

struct SimState {
  bool bound = false;
  int64_t n = 0, cap = 0;
  int nsys = 0, cap_sys = 0;
  double *pos = nullptr, *vel = nullptr;  // caller-owned, float64 [n][3]
  const float *mass = nullptr;            // caller-owned [n]
  std::vector<int64_t> offsets;           // host copy, nsys + 1
  std::vector<float> eps, theta;          // host copies, nsys
  int64_t host_s = 0;                     // sub-steps enqueued since the bind
  int64_t builds = 0;                     // of them, with a new tree (since the counter reset)
  int kmax = 0;
  float4 *shadow = nullptr, *aold = nullptr, *anew = nullptr;
  int64_t *si = nullptr;
  uint8_t *lev = nullptr, *act = nullptr;
  uint32_t *soff = nullptr;               // device copy of the offsets
  SimSys *ss = nullptr, *ss_host = nullptr;
  SimCtl *sc = nullptr, *sc_host = nullptr;
};

// Captured sub-step of the block-step driver (params.graph), in segments:
// system table, tree construction (skipped when the tree is reused),
// permute + moments + groups, walk, correct + predict the next sub-step
// (the first sub-step is predicted when the system is bound).  The pieces between
// them (control block, r_crit) and the events timing the construction and
// the walk are launched outside.
constexpr int kSegments = 5;
constexpr int kGroupSizes = 7;  // G = 1, 2, 4, ..., 64
constexpr int kWalkWidths = 3;  // W = 16, 32, 64
struct SimGraphs {
  // segments 0 (system table), 1 (tree) and 4 (correct + predict); 2 and 3 (groups, walk)
  // depend on the group shape and live in exec_g[log2 W - 4][log2 G],
  // captured on demand
  hipGraphExec_t exec[kSegments] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  hipGraphExec_t exec_g[kWalkWidths][kGroupSizes][2] = {};
  hipStream_t cap_stream = nullptr;
  uint64_t generation = 0;
  bool valid = false;
};

// The tree of the last build, for reuse between rebuilds (params.rebuild_interval).
struct TreeState {
  bool valid = false;
  int64_t n = 0;
  std::vector<int64_t> off;   // systems it was built for
  int n_leaf = 0, key_kind = 0;
  uint64_t buffers = 0;       // gothic_ctx::buffers when it was built
  int since = 0;              // evaluations on this tree so far
  RebuildModels models;       // rebuild_interval = 0: the paper's growth models
  double ref[32] = {0};       // walk time of each sub-step class on a fresh tree
  bool have_ref[32] = {false};
  bool fresh[32] = {false};   // ref[k] measured since the last rebuild
  hipEvent_t mk0 = nullptr, mk1 = nullptr;  // around the last construction
};

// Tuning state (params.autotune and gothic_autotune).  The online tuner keeps
// one Brent search per active-level class of the block steps: the sub-steps
// whose index has its lowest set bit at position c (all levels >= kmax - c
// are due) are timed against each other only.
constexpr int kTuneClasses = 32;
struct TuneState {
  OnlineTuner cls[kTuneClasses];
  bool ready = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // walk of the last tuned sub-step
  int pending = -1;                          // its class, or -1
  bool pending_rebuilt = false;              // ... whether it built its tree
  bool pending_tuned = false;                // ... whether its r_crit came from cls[]
  bool pending_pick = false;                 // ... whether its G came from pick[]
  GroupPicker pick[kTuneClasses];            // params.autotune = 2: (G, W) per class
  int class_G[kTuneClasses] = {};            // group size per class (0: params.group_size)
  int class_W[kTuneClasses] = {};            // walk width per class (0: params.walk_width)
  bool recording = false;                    // record ev0 / ev1 around the next walk
  // gothic_autotune results by (batched, log2 n, log2 of n / n_active, multipole)
  std::map<std::tuple<int, int, int, int>, gothic_tune_result> cache;
};

}  // namespace gothic

struct gothic_ctx {
  int device = 0;
  int num_cus = 256;
  gothic_params prm{};
  int64_t cap_n = 0, cap_nodes = 0, cap_groups = 0, cap_hist = 0, cap_sys = 0, cap_anc = 0;
  int64_t spill_per_wave = 0;
  int walk_waves = 0;             // persistent walk waves (slots), the most any G launches
  // walk waves per (log2 W - 4, log2 G) for slots_multi / slots_D
  int slots_g[gothic::kWalkWidths][gothic::kGroupSizes] = {};
  int slots_multi = 0, slots_D = 0;
  int cur_G = 32;                 // group size of the evaluation being enqueued
  int cur_W = 64;                 // ... and its walk width
  gothic::Buffers b;
  gothic::Buffers sb;             // buffers of the last scratch-free call (in the static array)
  gothic::Buffers *lb = nullptr;  // buffers of the last evaluation (b or sb)
  int64_t scratch_held = 0;       // device scratch bytes held by b
  int64_t scratch_required = 0;   // bytes a refused call needed (ECAPTURE / ENOMEM), else 0
  uint64_t generation = 1;        // bumped whenever a device buffer or a parameter changes
  uint64_t buffers = 1;           // bumped whenever a device buffer is (re)allocated
  // last evaluation
  int64_t last_n = 0;
  int last_nsys = 0;
  hipStream_t last_stream = nullptr;
  bool have_last = false;
  // walk-kernel timing (params.timing): event pairs recorded around each walk
  std::vector<hipEvent_t> ev_start, ev_stop;
  int ev_used = 0;
  gothic::SimState sim;
  gothic::SimGraphs graphs;
  gothic::TuneState tune;
  gothic::TreeState tree;
  // float64 partials of the direct summation (gothic_direct_forces)
  double4 *direct_part = nullptr;
  int64_t cap_direct = 0;
};

namespace gothic {

// error plumbing (api.hip)
int set_error(int code, const std::string &msg);
int hip_check(hipError_t e, const char *what);

// ---- launchers (one translation unit each) ----
// scan.hip: exclusive scan of in[0..n) -> out, n = *n_dev - (*lo_dev if lo_dev)
// (or n_host when n_dev is null); the total goes to *total_dev.
void scan_exclusive(const uint32_t *in, uint32_t *out, int64_t n_host, const unsigned *n_dev,
                    const unsigned *lo_dev, int64_t n_max, unsigned *total_dev, uint32_t *part,
                    hipStream_t s);
int scan_blocks();

// direct.hip: float64 direct sum for ni targets; part holds nchunk * ni partials
void direct_plan(int64_t n, int64_t ni, int *nchunk, int64_t *chunk);
void launch_direct(int64_t n, const float4 *xyzm, double eps, int64_t ni, const int64_t *idx,
                   double4 *part, double *out, hipStream_t s);

// keys.hip (nsys systems, the largest holding max_n particles)
void launch_bbox_keys(gothic_ctx *c, const float4 *xyzm, int64_t n, int nsys, int64_t max_n,
                      hipStream_t s);
int bbox_partials(int nsys, int64_t max_n);
// sort.hip: (system, key, index) order in keyA / idxA
void launch_radix_sort(gothic_ctx *c, int64_t n, int nsys, hipStream_t s);
bool keys_to_B(int nsys);  // the key kernel writes keyB / idxB (odd pass count)
int64_t radix_hist_entries(int64_t n);
// tree.hip
void launch_permute(gothic_ctx *c, const float4 *xyzm, const uint8_t *active, bool sign_active,
                    const float4 *acc_old, int64_t n, hipStream_t s);
void launch_build(gothic_ctx *c, int64_t n, int nsys, hipStream_t s);
// moments.hip: the ancestor table of a new tree
void launch_ancestors(gothic_ctx *c, int64_t n, hipStream_t s);
// moments.hip
void launch_moments(gothic_ctx *c, int64_t n, int nsys, hipStream_t s);
// groups.hip
void launch_groups(gothic_ctx *c, int64_t n, hipStream_t s);
// walk.hip
void launch_walk(gothic_ctx *c, int64_t n, float4 *acc_pot, hipStream_t s);
int walk_slots(gothic_ctx *c);
// sim.hip
void sim_launch_setup(gothic_ctx *c, hipStream_t s, double eta, int kmax, int shared);
void sim_launch_reset(gothic_ctx *c, hipStream_t s, bool all);
void sim_launch_shadow(gothic_ctx *c, hipStream_t s);
void sim_launch_init(gothic_ctx *c, hipStream_t s);
void sim_launch_predict(gothic_ctx *c, hipStream_t s);
void sim_launch_correct(gothic_ctx *c, hipStream_t s);
void sim_launch_hist(gothic_ctx *c, hipStream_t s);

}  // namespace gothic
