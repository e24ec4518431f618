"""Host logic of the tuner (Section 2.4: Brent's method on the measured time,
then perturbation), compiled from the library's own header with the host C++
compiler.  Pinned against scipy's bounded Brent minimiser, which implements
the same published algorithm: the sequence of evaluated points must agree."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1610_07279_amd", "csrc")

WRAP = r'''
#include "tune.h"
using gothic::BrentMin;
using gothic::OnlineTuner;
using gothic::RebuildModels;
using gothic::GroupPicker;
extern "C" {
void *gp_new(int rounds) { auto *g = new GroupPicker(); g->init(rounds); return g; }
int gp_current(void *p) { return static_cast<GroupPicker *>(p)->current(); }
int gp_width(void *p) { return static_cast<GroupPicker *>(p)->current_width(); }
int gp_decided(void *p) { return static_cast<GroupPicker *>(p)->decided(); }
void gp_observe(void *p, double t) { static_cast<GroupPicker *>(p)->observe(t); }
void gp_choose(void *p, int G, int W) { static_cast<GroupPicker *>(p)->choose(G, W); }
void *rm_new(double n_max) { auto *r = new RebuildModels(); r->n_max = n_max; return r; }
void rm_rebuilt(void *p, double t) { static_cast<RebuildModels *>(p)->rebuilt(t); }
void rm_sample(void *p, double t) { static_cast<RebuildModels *>(p)->sample(t); }
int rm_due(void *p) { return static_cast<RebuildModels *>(p)->due(); }
// kind -1: the best model; out = p0, p1, p2, chi2nu, n_opt; returns the kind
int rm_fit(void *p, int kind, double *out) {
  auto *r = static_cast<RebuildModels *>(p);
  RebuildModels::Fit f = kind == 0 ? r->fit_linear() : kind == 1 ? r->fit_power()
                       : kind == 2 ? r->fit_parabolic() : r->best();
  out[0] = f.p0; out[1] = f.p1; out[2] = f.p2; out[3] = f.chi2nu; out[4] = f.n_opt;
  return f.kind;
}
void *bm_new() { return new BrentMin(); }
void bm_free(void *p) { delete static_cast<BrentMin *>(p); }
void bm_start(void *p, double a, double b, double tol, int m) {
  static_cast<BrentMin *>(p)->start(a, b, tol, m);
}
double bm_ask(void *p) { return static_cast<BrentMin *>(p)->ask(); }
void bm_tell(void *p, double f) { static_cast<BrentMin *>(p)->tell(f); }
int bm_done(void *p) { return static_cast<BrentMin *>(p)->done(); }
double bm_best(void *p) { return static_cast<BrentMin *>(p)->best(); }
void *ot_new(double lo, double hi, double tol, int m) {
  auto *t = new OnlineTuner();
  t->init(lo, hi, tol, m);
  return t;
}
double ot_current(void *p) { return static_cast<OnlineTuner *>(p)->current(); }
void ot_observe(void *p, double f) { static_cast<OnlineTuner *>(p)->observe(f); }
double ot_best(void *p) { return static_cast<OnlineTuner *>(p)->best; }
int ot_searches(void *p) { return static_cast<OnlineTuner *>(p)->searches; }
}
'''


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("tune")
    src = d / "wrap.cpp"
    src.write_text(WRAP)
    so = d / "libtune.so"
    subprocess.run(["g++", "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-I", CSRC,
                    str(src), "-o", str(so)], check=True)
    L = ctypes.CDLL(str(so))
    P, D, I = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    L.bm_new.restype = P
    L.bm_start.argtypes = [P, D, D, D, I]
    L.bm_ask.argtypes = [P]
    L.bm_ask.restype = D
    L.bm_tell.argtypes = [P, D]
    L.bm_done.argtypes = [P]
    L.bm_best.argtypes = [P]
    L.bm_best.restype = D
    L.bm_free.argtypes = [P]
    L.ot_new.argtypes = [D, D, D, I]
    L.ot_new.restype = P
    L.ot_current.argtypes = [P]
    L.ot_current.restype = D
    L.ot_observe.argtypes = [P, D]
    L.ot_best.argtypes = [P]
    L.ot_best.restype = D
    L.ot_searches.argtypes = [P]
    L.gp_new.argtypes = [I]
    L.gp_new.restype = P
    L.gp_current.argtypes = [P]
    L.gp_decided.argtypes = [P]
    L.gp_observe.argtypes = [P, D]
    L.gp_choose.argtypes = [P, I, I]
    L.gp_width.argtypes = [P]
    L.rm_new.argtypes = [D]
    L.rm_new.restype = P
    L.rm_rebuilt.argtypes = [P, D]
    L.rm_sample.argtypes = [P, D]
    L.rm_due.argtypes = [P]
    L.rm_fit.argtypes = [P, I, P]
    return L


FUNCS = {
    "parabola": (lambda x: (x - 0.3) * (x - 0.3), (-2.0, 3.0)),
    "kink": (lambda x: abs(x - 0.71) * (1.0 + (x - 0.71) * (x - 0.71)), (0.0, 1.0)),
    "quartic": (lambda x: x * x * x * x - 2.0 * x * x + 0.5 * x, (0.0, 2.0)),
    "edge": (lambda x: -x, (-1.0, 4.0)),  # minimum on the boundary
    "flat": (lambda x: 1.0, (-1.0, 1.0)),
}


@pytest.mark.parametrize("name", list(FUNCS))
@pytest.mark.parametrize("xatol", [1e-5, 0.05])
def test_brent_follows_the_published_algorithm(lib, name, xatol):
    from scipy.optimize import minimize_scalar
    f, (lo, hi) = FUNCS[name]
    seen = []

    def g(x):
        seen.append(float(x))
        return f(float(x))
    res = minimize_scalar(g, bounds=(lo, hi), method="bounded", options={"xatol": xatol})
    p = lib.bm_new()
    lib.bm_start(p, lo, hi, xatol, 500)
    mine = []
    while not lib.bm_done(p):
        u = lib.bm_ask(p)
        mine.append(u)
        lib.bm_tell(p, f(u))
    best = lib.bm_best(p)
    lib.bm_free(p)
    assert len(mine) == len(seen)
    assert np.allclose(mine, seen, rtol=0, atol=1e-12 * max(1.0, abs(hi - lo)))
    assert abs(best - res.x) <= 1e-12 * max(1.0, abs(hi - lo))


def test_brent_finds_known_minima(lib):
    # closed forms: parabola vertex, kink location, quartic x^4 - 2x^2 + x/2 root of 4x^3-4x+1/2
    roots = np.roots([4.0, 0.0, -4.0, 0.5])
    quartic_min = max(r.real for r in roots if abs(r.imag) < 1e-12 and 0 < r.real < 2)
    for name, want in (("parabola", 0.3), ("kink", 0.71), ("quartic", quartic_min), ("edge", 4.0)):
        f, (lo, hi) = FUNCS[name]
        p = lib.bm_new()
        lib.bm_start(p, lo, hi, 1e-6, 500)
        while not lib.bm_done(p):
            u = lib.bm_ask(p)
            lib.bm_tell(p, f(u))
        assert abs(lib.bm_best(p) - want) < 1e-4, name
        lib.bm_free(p)


def test_online_tuner_tracks_a_moving_minimum(lib):
    # the optimum jumps from -3 to -6 after 60 measurements; the perturbed
    # searches follow it
    t = lib.ot_new(-12.0, 0.0, 0.25, 30)
    for k in range(400):
        c = -3.0 if k < 60 else -6.0
        u = lib.ot_current(t)
        assert -12.0 <= u <= 0.0
        lib.ot_observe(t, 1.0 + (u - c) ** 2)
    assert lib.ot_searches(t) >= 3
    assert abs(lib.ot_best(t) - (-6.0)) < 0.3


# ---------------------------------------------------------------- rebuild interval
def _models(lib, t_make, tw, n_max=200.0):
    r = lib.rm_new(n_max)
    lib.rm_rebuilt(r, t_make)
    for t in tw:
        lib.rm_sample(r, t)
    return r


def _fit(lib, r, kind):
    out = np.zeros(5)
    k = lib.rm_fit(r, kind, out.ctypes.data_as(ctypes.c_void_p))
    return k, out


def _argmin_mean(t_tot, hi=200.0):
    """The continuous minimiser of t_tot(n) / n, found numerically."""
    from scipy.optimize import minimize_scalar
    return minimize_scalar(lambda n: t_tot(n) / n, bounds=(1.0, hi), method="bounded",
                           options={"xatol": 1e-9}).x


@pytest.mark.parametrize("t_make,t1,dt", [(40.0, 5.0, 0.2), (4.0, 12.0, 0.06)])
def test_linear_growth_model(lib, t_make, t1, dt):
    tw = [t1 + i * dt for i in range(10)]
    r = _models(lib, t_make, tw)
    k, f = _fit(lib, r, 0)
    assert k == 0 and f[0] == pytest.approx(t1, rel=1e-12) and f[1] == pytest.approx(dt, rel=1e-10)
    assert f[3] < 1e-20
    want = _argmin_mean(lambda n: t_make + n * (t1 - dt) + n * (n + 1) / 2 * dt)
    assert f[4] == pytest.approx(want, rel=1e-6)
    assert f[4] == pytest.approx(np.sqrt(2 * t_make / dt), rel=1e-12)


@pytest.mark.parametrize("t_make,t1,ratio", [(40.0, 5.0, 1.03), (10.0, 2.0, 1.2)])
def test_power_law_growth_model(lib, t_make, t1, ratio):
    tw = [t1 * ratio ** i for i in range(12)]
    r = _models(lib, t_make, tw)
    k, f = _fit(lib, r, 1)
    assert k == 1 and f[0] == pytest.approx(t1, rel=1e-10) and f[1] == pytest.approx(ratio, rel=1e-12)
    want = _argmin_mean(lambda n: t_make + (ratio ** n - 1) / (ratio - 1) * t1)
    assert f[4] == pytest.approx(want, rel=1e-6)
    # the power law fits its own data better than the straight line
    kb, fb = _fit(lib, r, -1)
    assert kb == 1


@pytest.mark.parametrize("t_make,t1,b,a", [(40.0, 5.0, 0.05, 0.01), (25.0, 3.0, -0.1, 0.02)])
def test_parabolic_growth_model(lib, t_make, t1, b, a):
    tw = [t1 + i * b + i * i * a for i in range(12)]
    r = _models(lib, t_make, tw)
    k, f = _fit(lib, r, 2)
    assert k == 2
    assert f[0] == pytest.approx(t1, rel=1e-9) and f[1] == pytest.approx(b, rel=1e-7, abs=1e-12)
    assert f[2] == pytest.approx(a, rel=1e-7)
    want = _argmin_mean(lambda n: t_make + n * t1 + n * (n - 1) / 2 * b
                        + n * (n - 1) * (2 * n - 1) / 6 * a)
    assert f[4] == pytest.approx(want, rel=1e-6)
    assert (2 * f[4] - 1) * a + b >= 0  # a minimum, not a maximum


def test_no_growth_means_no_rebuild(lib):
    r = _models(lib, 10.0, [5.0, 5.0, 5.0, 5.0, 5.0], n_max=64.0)
    k, f = _fit(lib, r, -1)
    assert f[4] == 64.0
    assert not lib.rm_due(r)


def test_rebuild_becomes_due_at_the_optimum(lib):
    t_make, t1, dt = 40.0, 5.0, 0.2  # optimum n = 20
    r = lib.rm_new(200.0)
    lib.rm_rebuilt(r, t_make)
    due_at = None
    for i in range(40):
        lib.rm_sample(r, t1 + i * dt)
        if lib.rm_due(r):
            due_at = i + 1
            break
    assert due_at == 20


def test_group_picker_times_candidates_in_turn(lib):
    """Per-class group shape (the per-step S the paper leaves as future work):
    the candidates (G, W) = (8, 64), (16, 64), (32, 64), (64, 64), (4, 16),
    (8, 16), (8, 32), (16, 32) are visited round-robin, `rounds` times each,
    and the smallest mean time wins; a later observation changes nothing."""
    shapes = [(8, 64), (16, 64), (32, 64), (64, 64), (4, 16), (8, 16), (8, 32), (16, 32)]
    cost = {(8, 64): 3.0, (16, 64): 2.0, (32, 64): 2.5, (64, 64): 4.0,
            (4, 16): 3.5, (8, 16): 2.6, (8, 32): 2.2, (16, 32): 2.4}
    g = lib.gp_new(3)
    seen = []
    while not lib.gp_decided(g):
        sh = (lib.gp_current(g), lib.gp_width(g))
        seen.append(sh)
        # an ageing tree: every later walk is slower, by more than the gap
        # between the two best shapes over the whole pick
        lib.gp_observe(g, cost[sh] + 0.01 * len(seen))
    assert seen == shapes * 3
    assert (lib.gp_current(g), lib.gp_width(g)) == (16, 64)
    lib.gp_observe(g, 0.0)
    assert (lib.gp_current(g), lib.gp_width(g)) == (16, 64)
    # noise that reverses one round does not reverse the means
    g2 = lib.gp_new(2)
    times = iter([3.0, 2.9, 2.5, 4.0, 3.3, 3.0, 2.4, 2.6,
                  3.0, 1.0, 2.5, 4.0, 3.3, 3.0, 2.4, 2.6])
    while not lib.gp_decided(g2):
        lib.gp_observe(g2, next(times))
    assert (lib.gp_current(g2), lib.gp_width(g2)) == (16, 64)  # 1.95 against 2.4 for (8, 32)
    # a walk width below 64 can win
    g4 = lib.gp_new(1)
    times = iter([3.0, 2.9, 2.5, 4.0, 3.3, 3.0, 2.0, 2.6])
    while not lib.gp_decided(g4):
        lib.gp_observe(g4, next(times))
    assert (lib.gp_current(g4), lib.gp_width(g4)) == (8, 32)
    # a shape fixed from outside
    g3 = lib.gp_new(2)
    lib.gp_choose(g3, 64, 64)
    assert lib.gp_decided(g3) and lib.gp_current(g3) == 64 and lib.gp_width(g3) == 64
    g5 = lib.gp_new(2)
    lib.gp_choose(g5, 8, 16)
    assert lib.gp_decided(g5) and (lib.gp_current(g5), lib.gp_width(g5)) == (8, 16)
