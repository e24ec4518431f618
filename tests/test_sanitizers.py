"""Address and undefined-behaviour sanitizers on the CPU-side code:

- the float64 oracle (oracle/gothic_oracle.c), every function on small
  inputs, built with gcc -fsanitize=address,undefined;
- the host logic of the tuners (csrc/tune.h: Brent's method, the online
  tuner, the rebuild-interval growth models, the group-size picker), built
  with g++ and the same sanitizers;
- the library's host code (argument checks of the C ABI), built with hipcc
  with the sanitizers on the host side only (-Xarch_host), called on the
  paths that return before any device is touched.

Each driver aborts on the first report (-fno-sanitize-recover), so a clean
exit means no report."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")

ORACLE_DRIVER = r'''
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
void orc_direct(int64_t, const float *, double, int64_t, const int64_t *, double *);
uint64_t orc_morton(uint64_t, uint64_t, uint64_t);
uint64_t orc_ph_encode(int, uint64_t, uint64_t, uint64_t);
void orc_ph_decode(int, uint64_t, uint64_t *, uint64_t *, uint64_t *);
void orc_cube(int64_t, const float *, double[4]);
void orc_keys(int64_t, const float *, int, const double[4], uint64_t *);
void orc_sort(int64_t, const uint64_t *, uint64_t *, uint32_t *);
int64_t orc_build(int64_t, const uint64_t *, int, int64_t, uint32_t *, uint32_t *, uint32_t *,
                  uint8_t *, uint8_t *);
void orc_moments(int64_t, const uint32_t *, const uint32_t *, const double *, double *, double *,
                 double *);
void orc_seb(int, const double *, double[4]);
int64_t orc_groups(int64_t, const uint8_t *, const double *, int, double, uint32_t *, uint32_t *,
                   uint32_t *, double *, int);
void orc_walk(int64_t, const uint32_t *, const uint32_t *, const uint32_t *, const uint8_t *,
              const double *, const double *, const double *, const double *, const uint32_t *,
              int64_t, const uint32_t *, const uint32_t *, const double *, double, double, int,
              double, double, const int64_t *, int64_t, double *, int64_t *, double *, int,
              double, const double *, uint32_t *, int64_t, uint32_t *);
void orc_walk_replay(int64_t, const uint32_t *, const uint32_t *, const uint32_t *,
                     const uint8_t *, const double *, const double *, const double *,
                     const double *, const uint32_t *, const uint32_t *, const uint32_t *,
                     const double *, double, double, int, double, double, int, double,
                     const double *, int64_t, const int64_t *, const uint32_t *, int64_t,
                     const uint32_t *, const uint32_t *, double *, int64_t *, double *);
static uint64_t st = 88172645463325252ull;
static double rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return (st >> 11) * 0x1.0p-53; }
int main(void) {
  const int64_t n = 1500;
  float *x = malloc(16 * n);
  for (int64_t i = 0; i < n; ++i) {
    double r = pow(rnd(), 2.0);  /* centrally concentrated */
    for (int a = 0; a < 3; ++a) x[4 * i + a] = (float)(r * (2 * rnd() - 1));
    x[4 * i + 3] = (float)(0.5 + rnd()) / n;
  }
  for (int i = 0; i < 40; ++i) for (int a = 0; a < 4; ++a) x[4 * (100 + i) + a] = x[4 * 99 + a];
  int64_t *idx = malloc(8 * n); for (int64_t i = 0; i < n; ++i) idx[i] = i;
  double *dir = malloc(32 * n);
  orc_direct(n, x, 0.01, n, idx, dir);
  uint64_t px, py, pz;
  orc_ph_decode(21, orc_ph_encode(21, 12345, 999, 2097151), &px, &py, &pz);
  if (px != 12345 || py != 999 || pz != 2097151 || orc_morton(1, 0, 0) != 4) return 3;
  double cube[4];
  orc_cube(n, x, cube);
  uint64_t *k = malloc(8 * n), *ks = malloc(8 * n);
  uint32_t *perm = malloc(4 * n);
  double *ps = malloc(32 * n);
  for (int kind = 0; kind < 2; ++kind) {
    orc_keys(n, x, kind, cube, k);
    orc_sort(n, k, ks, perm);
    for (int64_t i = 0; i < n; ++i) for (int a = 0; a < 4; ++a) ps[4 * i + a] = x[4 * perm[i] + a];
    for (int nl = 1; nl <= 16; nl += 15) {
      int64_t cap = 4 * n + 64;
      uint32_t *first = malloc(4 * cap), *count = malloc(4 * cap), *cf = malloc(4 * cap);
      uint8_t *nc = malloc(cap), *lv = malloc(cap);
      int64_t nn = orc_build(n, ks, nl, cap, first, count, cf, nc, lv);
      if (nn <= 0) return 4;
      double *com = malloc(32 * nn), *b = malloc(8 * nn), *S = malloc(48 * nn);
      orc_moments(nn, first, count, ps, com, b, S);
      uint8_t *act = malloc(n);
      for (int64_t i = 0; i < n; ++i) act[i] = rnd() < 0.6;
      uint32_t *alist = malloc(4 * n), *gf = malloc(4 * n), *gc = malloc(4 * n);
      double *ball = malloc(32 * n), *amag = malloc(8 * n), *out = malloc(32 * n);
      for (int64_t i = 0; i < n; ++i) amag[i] = 0.1 + rnd();
      for (int bk = 0; bk < 5; ++bk) {
        int64_t ng = orc_groups(n, act, ps, 16, bk == 2 ? 0.05 : 0.0, alist, gf, gc, ball, bk);
        int64_t *cnt = malloc(24 * (ng + 1));
        double *mass = malloc(8 * (ng + 1));
        int64_t gsel[3] = {0, ng / 2, ng - 1};
        int64_t lcap = 4096;
        uint32_t *lists = malloc(4 * 3 * lcap), *lcount = malloc(4 * 6);
        for (int mac = 0; mac < 3; ++mac)
          for (int mp = 1; mp <= 2; ++mp) {
            orc_walk(nn, first, count, cf, nc, com, b, S, ps, alist, ng, gf, gc, ball, 0.01, 0.5,
                     mp, 2e-5, 1e-6, NULL, 0, out, cnt, mass, mac, 1e-3, amag, NULL, 0, lcount);
            orc_walk(nn, first, count, cf, nc, com, b, S, ps, alist, ng, gf, gc, ball, 0.01, 0.5,
                     mp, 2e-5, 1e-6, gsel, 3, out, cnt, mass, mac, 1e-3, amag, lists, lcap, lcount);
            int64_t info[18];
            double rmass[3];
            orc_walk_replay(nn, first, count, cf, nc, com, b, S, ps, alist, gf, gc, ball, 0.01,
                            0.5, mp, 2e-5, 1e-6, mac, 1e-3, amag, 3, gsel, NULL, lcap, lists,
                            lcount, out, info, rmass);
            for (int q = 0; q < 3; ++q) if (info[6 * q + 2] || info[6 * q + 3] || info[6 * q + 4]) return 5;
          }
        free(cnt); free(mass); free(lists); free(lcount);
      }
      free(first); free(count); free(cf); free(nc); free(lv); free(com); free(b); free(S);
      free(act); free(alist); free(gf); free(gc); free(ball); free(amag); free(out);
    }
  }
  double pts[12] = {1, 1, 1, 1, -1, -1, -1, 1, -1, -1, -1, 1}, sb[4];
  orc_seb(4, pts, sb);
  free(x); free(idx); free(dir); free(k); free(ks); free(perm); free(ps);
  puts("oracle driver clean");
  return 0;
}
'''

TUNE_DRIVER = r'''
#include <cmath>
#include <cstdio>
#include "tune.h"
int main() {
  gothic::BrentMin bm;
  bm.start(-12.0, 0.0, 0.25, 16);
  while (!bm.done()) { double u = bm.ask(); bm.tell((u + 3.3) * (u + 3.3) + 1.0); }
  if (std::fabs(bm.best() + 3.3) > 0.5) return 3;
  gothic::OnlineTuner ot;
  ot.init(-12.0, 0.0, 0.25, 20);
  for (int i = 0; i < 200; ++i) { double u = ot.current(); ot.observe(std::fabs(u + 5.0) + 1.0); }
  gothic::RebuildModels rm;
  rm.n_max = 64;
  for (int r = 0; r < 6; ++r) {
    rm.rebuilt(3.0);
    for (int i = 0; i < 40 && !rm.due(); ++i) rm.sample(10.0 + 0.3 * i + 0.01 * i * i);
    (void)rm.fit_linear(); (void)rm.fit_power(); (void)rm.fit_parabolic(); (void)rm.best();
  }
  gothic::GroupPicker gp;
  gp.init(2);
  for (int i = 0; i < 20 && !gp.decided(); ++i) gp.observe(1.0 / gp.current());
  std::puts("tune driver clean");
  return 0;
}
'''

ABI_DRIVER = r'''
#include <stdio.h>
#include "gothic.h"
int main(void) {
  gothic_params p;
  gothic_ctx *c = 0;
  int fails = 0;
  gothic_default_params(&p); p.n_leaf = 0; fails += gothic_create(&c, 0, &p) != GOTHIC_EINVAL;
  gothic_default_params(&p); p.group_size = 3; fails += gothic_create(&c, 0, &p) != GOTHIC_EINVAL;
  gothic_default_params(&p); p.list_depth = 100; fails += gothic_create(&c, 0, &p) != GOTHIC_EINVAL;
  gothic_default_params(&p); p.r_crit = 1.0f / 0.0f; fails += gothic_create(&c, 0, &p) != GOTHIC_EINVAL;
  gothic_default_params(&p); p.mac_delta = -1.0f; fails += gothic_create(&c, 0, &p) != GOTHIC_EINVAL;
  gothic_default_params(&p); p.max_scratch_bytes = -1; fails += gothic_create(&c, 0, &p) != GOTHIC_EINVAL;
  gothic_default_params(&p); p.spill_per_wave = 5; fails += gothic_create(&c, 0, &p) != GOTHIC_EINVAL;
  gothic_default_params(&p); p.ball = 9; fails += gothic_create(&c, 0, &p) != GOTHIC_EINVAL;
  fails += gothic_create(0, 0, &p) != GOTHIC_EINVAL;
  fails += gothic_tree_forces(0, 10, 0, 0.1f, 0.5f, 0, 0, 0) != GOTHIC_EINVAL;
  int64_t off[3] = {0, 5, 3};
  float e[2] = {0.1f, 0.1f}, t[2] = {0.5f, 0.5f};
  fails += gothic_tree_forces_batched(0, 2, off, 0, e, t, 0, 0, 0) != GOTHIC_EINVAL;
  fails += gothic_get_stats(0, 0) != GOTHIC_EINVAL;
  fails += gothic_get_scratch(0, 0, 0) != GOTHIC_EINVAL;
  fails += gothic_get_lists(0, 1, 0, 1, 0, 0, 0) != GOTHIC_EINVAL;
  fails += gothic_sim_step(0, 0) != GOTHIC_EINVAL;
  fails += gothic_destroy(0) != GOTHIC_OK;
  printf("abi driver %s (last error: %s)\n", fails ? "FAILED" : "clean", gothic_last_error());
  return fails;
}
'''


def _run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, env=ENV, **kw)
    assert p.returncode == 0, p.stdout + p.stderr
    return p.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    (tmp_path / "drv.c").write_text(ORACLE_DRIVER)
    exe = tmp_path / "drv"
    _run(["gcc", *SAN, "-std=c11", "-ffp-contract=off", "-fopenmp", "-Wno-unknown-pragmas",
          str(tmp_path / "drv.c"), os.path.join(ROOT, "oracle", "gothic_oracle.c"), "-o", str(exe),
          "-lm"])
    out = _run([str(exe)], timeout=600)
    assert "oracle driver clean" in out


def test_tuner_host_logic_under_asan_ubsan(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    (tmp_path / "drv.cpp").write_text(TUNE_DRIVER)
    exe = tmp_path / "drv"
    _run(["g++", *SAN, "-std=c++17", "-I", os.path.join(ROOT, "paper_1610_07279_amd", "csrc"),
          str(tmp_path / "drv.cpp"), "-o", str(exe)])
    assert "tune driver clean" in _run([str(exe)], timeout=120)


def test_abi_argument_checks_under_asan_ubsan(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("no hipcc")
    csrc = os.path.join(ROOT, "paper_1610_07279_amd", "csrc")
    host_san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"):
        host_san += ["-Xarch_host", f]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", *host_san, "-Xclang",
             "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")]
    srcs = sorted(f for f in os.listdir(csrc) if f.endswith(".hip"))

    def compile_one(f):
        o = str(tmp_path / (f + ".o"))
        _run([hipcc, *flags, "-c", os.path.join(csrc, f), "-o", o])
        return o

    with ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libgothic_san.so")
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *host_san, *objs, "-o", lib])
    (tmp_path / "drv.c").write_text(ABI_DRIVER)
    exe = str(tmp_path / "drv")
    _run([hipcc, *host_san, "-g", "-I", os.path.join(ROOT, "include"), "-x", "c",
          str(tmp_path / "drv.c"), "-x", "none", lib, "-Wl,-rpath," + str(tmp_path), "-o", exe])
    assert "abi driver clean" in _run([exe], timeout=120)
