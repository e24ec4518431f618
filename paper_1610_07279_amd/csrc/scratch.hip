// Device scratch of a context: the buffers every stage of the pipeline works
// in, grown on demand (ensure), counted against params.max_scratch_bytes, or
// carved from one block of device memory (the scratch-free entry point).
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "api_internal.h"

namespace gothic {

// Every buffer of Buffers, by the capacity it scales with.  f(pointer, count)
// is called once per buffer, in a fixed order.
template <class F>
static void visit_fixed(Buffers &B, F &&f) {
  f(B.ctl, 1);
  f(B.part, (int64_t)scan_blocks() + 64);
  f(B.rcrit, 1);
}

template <class F>
static void visit_sys(Buffers &B, int64_t cs, F &&f) {
  f(B.sys, cs);
  f(B.soff, cs + 1);
  // bbox partials: nsys x bbox_partials(nsys, .) <= max(1024, nsys) workgroups
  f(B.bbox_part, 6 * std::max<int64_t>(1024, cs));
}

template <class F>
static void visit_particles(Buffers &B, int64_t cn, F &&f) {
  f(B.keyA, cn);
  f(B.keyB, cn);
  f(B.idxA, cn);
  f(B.idxB, cn);
  f(B.pos, cn);
  f(B.leaf_of, cn);
  f(B.flag, cn);
  f(B.flag2, cn);
  f(B.alist, cn);
  f(B.nch, cn + 1);
  f(B.gA, cn + 1);
  f(B.gB, cn + 1);
  f(B.gfirst, cn + 1);
  f(B.bnd, 8 * cn + 8);
  f(B.ball, cn);
  f(B.gent, 2 * cn);
  f(B.amag, cn);
  f(B.gamin, cn);
  f(B.hist, 2 * radix_hist_entries(cn));
}

template <class F>
static void visit_nodes(Buffers &B, int64_t nn, F &&f) {
  f(B.first, nn);
  f(B.count, nn);
  f(B.child_first, nn);
  f(B.parent, nn);
  f(B.n_child, nn);
  f(B.level, nn);
  f(B.nrec, 2 * nn);
  f(B.quad, 2 * nn);
  f(B.mcrit, nn);
}

template <class F>
static void visit_anc(Buffers &B, int64_t cn, F &&f) {
  f(B.anc, (int64_t)kMaxLevels * cn);
  f(B.leaflev, cn);
}

template <class F>
static void visit_spill(Buffers &B, int64_t waves, int64_t spill, F &&f) {
  f(B.spill, waves * spill);
}

static int64_t round256(int64_t b) { return (b + 255) / 256 * 256; }

// bytes of one group of buffers
template <class V>
static int64_t group_bytes(V &&visit) {
  Buffers tmp;
  int64_t total = 0;
  visit(tmp, [&](auto *&p, int64_t count) {
    (void)p;
    total += round256((int64_t)sizeof(*p) * std::max<int64_t>(count, 1));
  });
  return total;
}

int64_t scratch_bytes(const Caps &k) {
  int64_t t = group_bytes([&](Buffers &B, auto &&f) { visit_fixed(B, f); });
  t += group_bytes([&](Buffers &B, auto &&f) { visit_sys(B, k.sys, f); });
  t += group_bytes([&](Buffers &B, auto &&f) { visit_particles(B, k.n, f); });
  t += group_bytes([&](Buffers &B, auto &&f) { visit_nodes(B, k.nodes, f); });
  t += group_bytes([&](Buffers &B, auto &&f) { visit_anc(B, k.anc, f); });
  t += group_bytes([&](Buffers &B, auto &&f) { visit_spill(B, k.waves, k.spill, f); });
  return t;
}

void carve_buffers(Buffers &B, const Caps &k, char *base) {
  int64_t off = 0;
  auto take = [&](auto *&p, int64_t count) {
    using T = std::remove_reference_t<decltype(*p)>;
    p = reinterpret_cast<T *>(base + off);
    off += round256((int64_t)sizeof(T) * std::max<int64_t>(count, 1));
  };
  visit_fixed(B, take);
  visit_sys(B, k.sys, take);
  visit_particles(B, k.n, take);
  visit_nodes(B, k.nodes, take);
  visit_anc(B, k.anc, take);
  visit_spill(B, k.waves, k.spill, take);
}

// Debugging aid: with the environment variable GOTHIC_POISON_ALLOC set (to
// anything but "0"), every new floating-point buffer starts as all-ones bytes
// (NaN in every lane), so a kernel that reads memory no kernel of the
// evaluation wrote gives visibly wrong results instead of results that depend
// on what the memory held before.  Index buffers are left alone.
static bool poison_alloc() {
  const char *v = getenv("GOTHIC_POISON_ALLOC");
  return v && v[0] && strcmp(v, "0") != 0;
}

int dev_alloc_bytes(void **p, size_t bytes, bool fp) {
  if (*p) {
    (void)hipFree(*p);
    *p = nullptr;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return hip_check(e, "hipMalloc");
  }
  if (fp && poison_alloc()) {
    // synchronous, so no later launch on any stream can overtake it
    if ((e = hipMemset(*p, 0xff, bytes)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess)
      return hip_check(e, "poison fill");
  }
  return GOTHIC_OK;
}

void free_all(gothic_ctx *c) {
  Buffers &B = c->b;
  auto release = [](auto *&p, int64_t) {
    if (p) (void)hipFree(p);
    p = nullptr;
  };
  visit_fixed(B, release);
  visit_sys(B, 0, release);
  visit_particles(B, 0, release);
  visit_nodes(B, 0, release);
  visit_anc(B, 0, release);
  visit_spill(B, 0, 0, release);
  if (B.ctl_host) (void)hipHostFree(B.ctl_host);
  B = Buffers();
  if (c->lb != &c->b) c->lb = nullptr;
  c->cap_n = c->cap_nodes = c->cap_groups = c->cap_hist = c->cap_sys = c->cap_anc = 0;
  c->walk_waves = 0;
  c->spill_per_wave = 0;
  c->scratch_held = 0;
  ++c->generation;
  ++c->buffers;
}

int64_t default_spill(const gothic_ctx *c) {
  return c->prm.spill_per_wave > 0 ? c->prm.spill_per_wave : 16384;
}

int64_t nodes_wanted(gothic_ctx *c, int64_t n, int nsys) {
  // typical trees hold ~0.25 n nodes at n_leaf = 16 and ~2-3 n at n_leaf = 1
  return std::max<int64_t>(c->cap_nodes, c->prm.node_capacity > 0
                                             ? c->prm.node_capacity
                                             : n + 8 * (n / c->prm.n_leaf) + 1024 + nsys);
}

// The capacities ensure() grows to.
static Caps grown_caps(gothic_ctx *c, int64_t n, int nsys, int64_t want_nodes, int64_t want_spill) {
  Caps k;
  k.sys = nsys > c->cap_sys ? std::max<int64_t>(nsys, 64) : c->cap_sys;
  k.n = n > c->cap_n ? std::max<int64_t>(n, 1024) : c->cap_n;
  const int64_t nodes = std::max<int64_t>(want_nodes, 64);
  k.nodes = nodes > c->cap_nodes ? nodes : c->cap_nodes;
  k.anc = k.n;
  k.waves = walk_slots(c);
  k.spill = std::max<int64_t>(want_spill, default_spill(c));
  if (k.waves == c->walk_waves && c->b.spill) k.spill = std::max<int64_t>(k.spill, c->spill_per_wave);
  return k;
}

int64_t ensure_bytes(gothic_ctx *c, int64_t n, int nsys, int64_t want_nodes, int64_t want_spill) {
  return scratch_bytes(grown_caps(c, n, nsys, want_nodes, want_spill));
}

// Make sure every buffer can hold n particles (and the current node / spill
// capacities).  Never called while the stream is being captured.
int ensure(gothic_ctx *c, int64_t n, int nsys, int64_t want_nodes, int64_t want_spill) {
  Buffers &B = c->b;
  const Caps k = grown_caps(c, n, nsys, want_nodes, want_spill);
  const int64_t need = scratch_bytes(k);
  if (c->prm.max_scratch_bytes > 0 && need > c->prm.max_scratch_bytes) {
    c->scratch_required = need;
    return set_error(GOTHIC_ENOMEM, "scratch would grow to " + std::to_string(need) +
                                        " bytes, above max_scratch_bytes " +
                                        std::to_string(c->prm.max_scratch_bytes));
  }
  int rc = GOTHIC_OK;
  auto grow = [&](auto *&p, int64_t count) {
    if (rc == GOTHIC_OK) rc = dev_alloc(&p, count);
  };
  bool changed = false;
  if (!B.ctl) {
    visit_fixed(B, grow);
    if (rc) return rc;
    GCHECK(hipHostMalloc(reinterpret_cast<void **>(&B.ctl_host), sizeof(Ctl), hipHostMallocDefault));
    // the sticky flags survive every reset of the control block: start clean
    GCHECK(hipMemset(B.ctl, 0, sizeof(Ctl)));
    changed = true;
  }
  if (k.sys != c->cap_sys) {
    visit_sys(B, k.sys, grow);
    if (rc) return rc;
    c->cap_sys = k.sys;
    changed = true;
  }
  if (k.n != c->cap_n) {
    visit_particles(B, k.n, grow);
    if (rc) return rc;
    c->cap_n = k.n;
    c->cap_groups = k.n;
    c->cap_hist = 2 * radix_hist_entries(k.n);
    changed = true;
  }
  if (k.nodes != c->cap_nodes) {
    visit_nodes(B, k.nodes, grow);
    if (rc) return rc;
    c->cap_nodes = k.nodes;
    changed = true;
  }
  if (k.anc != c->cap_anc) {
    visit_anc(B, k.anc, grow);
    if (rc) return rc;
    c->cap_anc = k.anc;
    changed = true;
  }
  if (k.waves != c->walk_waves || k.spill != c->spill_per_wave || !B.spill) {
    visit_spill(B, k.waves, k.spill, grow);
    if (rc) return rc;
    c->walk_waves = (int)k.waves;
    c->spill_per_wave = k.spill;
    changed = true;
  }
  if (changed) {
    ++c->generation;
    ++c->buffers;
  }
  c->scratch_held = need;
  c->scratch_required = 0;
  return GOTHIC_OK;
}

}  // namespace gothic
