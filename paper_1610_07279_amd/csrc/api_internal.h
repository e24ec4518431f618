// Host-side internals shared by the translation units of the C ABI
// (context.hip, scratch.hip, pipeline.hip, introspect.hip, sim_api.hip,
// tune_api.hip, noalloc.hip).
#pragma once

#include <string>
#include <type_traits>
#include <vector>

#include "common.h"

namespace gothic {

#define GCHECK(call)                    \
  do {                                  \
    int _rc = hip_check((call), #call); \
    if (_rc != GOTHIC_OK) return _rc;   \
  } while (0)

constexpr int kMaxSys = 65535;  // grid y limit of the per-system kernels

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// How an evaluation is run and metered (defaults: a plain evaluation with
// params.group_size and the caller's active flags).
struct EvalOpts {
  int meter_class = 0;       // sub-step class the walk time is booked to
  bool tuned = false;        // r_crit came from the class's Brent search
  bool picked = false;       // the group size came from the class's picker
  int kmax = 0;              // finest level (class weights of the rebuild models)
  int group_G = 0;           // group size; 0 = params.group_size
  int walk_W = 0;            // walk width; 0 = params.walk_width
  bool sign_active = false;  // active flags are the sign bits of the masses in x4
};

// ---- context.hip
int validate_params(const gothic_params *p);
// params.walk_width with 0 read as 64
inline int walk_width_of(const gothic_params &p) { return p.walk_width ? p.walk_width : 64; }

// ---- scratch.hip: device scratch of a context
// capacities every buffer of Buffers is sized from
struct Caps {
  int64_t n = 0;       // particles
  int64_t nodes = 0;   // tree nodes
  int64_t sys = 0;     // systems
  int64_t anc = 0;     // particles covered by the ancestor table
  int64_t spill = 0;   // global pending-stack entries per walk wave
  int64_t waves = 0;   // walk waves holding a spill stack
};
// bytes of every buffer at capacities k (each rounded up to 256 bytes)
int64_t scratch_bytes(const Caps &k);
// carve every buffer of B from the device memory at base (scratch_bytes(k) of it)
void carve_buffers(Buffers &B, const Caps &k, char *base);
// (re)allocate one buffer; fp: a floating-point buffer (filled with NaN bytes
// when GOTHIC_POISON_ALLOC is set)
int dev_alloc_bytes(void **p, size_t bytes, bool fp);
template <class T>
constexpr bool kFloatBuffer =
    std::is_floating_point<T>::value || std::is_same<T, float4>::value ||
    std::is_same<T, float2>::value || std::is_same<T, double4>::value;
template <class T>
inline int dev_alloc(T **p, int64_t count) {
  return dev_alloc_bytes(reinterpret_cast<void **>(p), sizeof(T) * (size_t)(count > 0 ? count : 1),
                         kFloatBuffer<T>);
}
void free_all(gothic_ctx *c);
int64_t nodes_wanted(gothic_ctx *c, int64_t n, int nsys);
// grow every buffer to hold n particles, nsys systems, want_nodes nodes and
// want_spill pending entries per walk wave; never called under capture
int ensure(gothic_ctx *c, int64_t n, int nsys, int64_t want_nodes, int64_t want_spill);
// the scratch that ensure() would hold after growing (bytes), for the
// capture check and params.max_scratch_bytes
int64_t ensure_bytes(gothic_ctx *c, int64_t n, int nsys, int64_t want_nodes,
                     int64_t want_spill);
int64_t default_spill(const gothic_ctx *c);

// ---- pipeline.hip
int make_systems(int nsys, const int64_t *offsets, const float *eps, const float *theta,
                 bool allow_empty, Systems *out);
void enqueue_begin(gothic_ctx *c, bool keep_tree, float r_crit, hipStream_t s, bool fold = true);
void enqueue_upload(gothic_ctx *c, const Systems &sy, hipStream_t s);
void enqueue_make(gothic_ctx *c, const Systems &sy, const float4 *xyzm, hipStream_t s);
void enqueue_post(gothic_ctx *c, const Systems &sy, const float4 *xyzm, const uint8_t *active,
                  const float4 *acc_old, hipStream_t s, bool sign_active = false);
void enqueue_walk(gothic_ctx *c, int64_t n, float4 *out, hipStream_t s, bool timed);
int enqueue_forces(gothic_ctx *c, const Systems &sy, const float4 *xyzm, const uint8_t *active,
                   const float4 *acc_old, float4 *out, hipStream_t s, float r_crit, bool rebuild,
                   bool sign_active = false, bool fold = true);
// forget the flags of the last evaluation (handled by the host)
void enqueue_drop_flags(gothic_ctx *c, hipStream_t s);
void free_events(gothic_ctx *c);
int ensure_events(gothic_ctx *c);
bool must_rebuild(gothic_ctx *c, const Systems &sy);
void tree_used(gothic_ctx *c, const Systems &sy, bool rebuilt);
bool metering(const gothic_ctx *c);
int meter_prepare(gothic_ctx *c);
int meter_collect(gothic_ctx *c, int kmax);
void meter_mark(gothic_ctx *c, int k, bool rebuilt, bool tuned, bool picked);
int run_forces(gothic_ctx *c, const Systems &sy, const float4 *x4, const uint8_t *active,
               const float4 *acc_old, float4 *o4, hipStream_t s, float r_crit,
               const EvalOpts &o = EvalOpts());
// note that the evaluation just enqueued on s used the buffers lb
void mark_last(gothic_ctx *c, const Systems &sy, hipStream_t s, Buffers *lb);

// ---- noalloc.hip: look up this device's copy of the static scratch array
// (device current); called once per context creation
int static_scratch_attach(int dev);

// ---- sim_api.hip
void free_graphs(gothic_ctx *c);
void free_sim(gothic_ctx *c);

}  // namespace gothic
