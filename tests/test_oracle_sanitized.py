"""The FP64 oracle's C code under AddressSanitizer and UndefinedBehavior-
Sanitizer (CPU): a small C driver linked with oracle/bls_oracle.c calls every
entry point on tiny and edge-case inputs (two points, one period, two bins,
all weights zero but two, a single-period grid, runs that wrap, empty
chips) with one OpenMP thread, and must exit cleanly.  It checks memory and
undefined-behaviour errors only; the values are pinned elsewhere."""
import os
import subprocess
import tempfile

import pytest

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")

DRIVER = r'''
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include "bls_oracle.h"

#define CHECK(c) do { if (!(c)) { printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); return 1; } } while (0)

static double urand(unsigned *s) { *s = *s * 1103515245u + 12345u; return ((*s >> 8) & 0xFFFFFF) / 16777216.0; }

int main(void) {
  unsigned seed = 7;
  enum { N = 300, M = 40 };
  double t[N], x[N], w[N], per[M];
  for (int i = 0; i < N; ++i) { t[i] = 100.0 + 30.0 * urand(&seed); x[i] = urand(&seed) - 0.5; w[i] = 0.5 + urand(&seed); }
  for (int p = 0; p < M; ++p) per[p] = 0.3 * exp(p * log(30.0) / (M - 1));
  double sr[M], depth[M]; int32_t js[M], ks[M]; int64_t best; bls_oracle_prep pr;
  int32_t nbins_list[3] = {2, 37, 256};
  for (int b = 0; b < 3; ++b)
    for (int weighted = 0; weighted < 2; ++weighted)
      for (int dip = 0; dip < 2; ++dip)
        CHECK(bls_oracle_search(t, x, weighted ? w : NULL, N, per, M, nbins_list[b], 0.01, 0.6, 1,
                                dip, 1, sr, depth, js, ks, &best, &pr) == BLS_ORACLE_OK);
  /* two points, one period, two bins; then every weight zero but two */
  CHECK(bls_oracle_search(t, x, NULL, 2, per, 1, 2, 0.4, 0.6, 1, 0, 1, sr, depth, js, ks, &best, &pr) == BLS_ORACLE_OK);
  double w2[N];
  for (int i = 0; i < N; ++i) w2[i] = (i == 3 || i == 200) ? 1.0 : 0.0;
  CHECK(bls_oracle_search(t, x, w2, N, per, M, 50, 0.02, 0.5, 1, 0, 1, sr, depth, js, ks, &best, &pr) == BLS_ORACLE_OK);
  /* invalid input is refused without touching memory it should not */
  CHECK(bls_oracle_search(t, x, NULL, 1, per, M, 50, 0.02, 0.5, 1, 0, 1, sr, depth, js, ks, &best, &pr) != BLS_ORACLE_OK);
  int32_t bins[N]; double hw[256], hs[256]; int64_t hn[256];
  CHECK(bls_oracle_bins(t, x, w, N, per[5], 256, bins, hw, hs, hn) == N);
  /* unbinned, with wrapping runs (a wide q range) */
  int32_t fp[M], lp[M];
  CHECK(bls_oracle_unbinned(t, x, NULL, 60, per, M, 0.01, 0.9, 1, 0, 1, sr, depth, fp, lp, &best) == BLS_ORACLE_OK);
  CHECK(bls_oracle_unbinned(t, x, w, 60, per, M, 0.05, 0.3, 2, 1, 1, sr, depth, fp, lp, &best) == BLS_ORACLE_OK);
  CHECK(bls_oracle_unbinned(t, x, NULL, 2, per, 1, 0.1, 0.9, 1, 0, 1, sr, depth, fp, lp, &best) == BLS_ORACLE_OK);
  /* detection: random SR with a few peaks, then all zeros, then one period */
  double srd[M], mean, sd, sde, psr[8], psde[8]; int64_t pidx[8]; int32_t np, cand;
  for (int p = 0; p < M; ++p) srd[p] = urand(&seed);
  srd[10] = 5.0; srd[20] = 4.0;
  CHECK(bls_oracle_detect(srd, per, M, 8, 0.01, 3.0, &mean, &sd, &sde, pidx, psr, psde, &np, &cand) == BLS_ORACLE_OK);
  for (int p = 0; p < M; ++p) srd[p] = 0.0;
  CHECK(bls_oracle_detect(srd, per, M, 8, 0.5, 3.0, &mean, &sd, &sde, pidx, psr, psde, &np, &cand) == BLS_ORACLE_OK);
  CHECK(bls_oracle_detect(srd, per, 1, 8, 0.01, 3.0, &mean, &sd, &sde, pidx, psr, psde, &np, &cand) == BLS_ORACLE_OK);
  /* eclipse window, one and two eclipses required */
  int32_t obs[M];
  CHECK(bls_oracle_eclipse_window(t, w2, N, per, M, 64, 0.05, 1, 1, obs) == BLS_ORACLE_OK);
  CHECK(bls_oracle_eclipse_window(t, NULL, N, per, M, 200, 0.02, 2, 1, obs) == BLS_ORACLE_OK);
  /* variability: three chips, the middle one empty */
  enum { NC = 30 };
  int64_t noff[NC + 1]; double mag[NC], rms[NC]; int32_t vbin[NC], vflag[NC];
  for (int c = 0; c <= NC; ++c) noff[c] = (int64_t)c * 10;
  for (int c = 0; c < NC; ++c) mag[c] = 14.0 + 6.0 * urand(&seed);
  int64_t chip[4] = {0, 15, 15, NC};
  double bm[3 * 12], bs[3 * 12]; int32_t bc[3 * 12];
  CHECK(bls_oracle_variability(x, w, noff, NC, mag, chip, 3, 13.0, 0.5, 12, 3.0, 5, 3.0, 3,
                               rms, vbin, vflag, bm, bs, bc) == BLS_ORACLE_OK);
  /* injection and the recovery rule */
  double base[2 * N], xi[2 * N], pp[2] = {1.3, 4.1}, ph[2] = {0.2, 0.9}, qq[2] = {0.03, 0.1}, dd[2] = {0.01, 0.02};
  for (int i = 0; i < 2 * N; ++i) base[i] = urand(&seed);
  CHECK(bls_oracle_inject(t, w, N, base, 2, pp, ph, qq, dd, xi) == BLS_ORACLE_OK);
  CHECK(bls_oracle_recovered(1.3, 9.0, 1.3, 7.0, 0.01) == 1);
  printf("OK\n");
  return 0;
}
'''


def test_oracle_entry_points_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(src, "w").write(DRIVER)
        cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
               "-ffp-contract=off", "-fopenmp", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", "-I" + ORACLE, src,
               os.path.join(ORACLE, "bls_oracle.c"), "-o", exe, "-lm"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0 and "asan" in (r.stderr or "").lower():
            pytest.skip("no AddressSanitizer runtime: " + r.stderr[-300:])
        assert r.returncode == 0, r.stderr[-2000:]
        env = dict(os.environ, OMP_NUM_THREADS="1",
                   ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
        out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert out.returncode == 0 and out.stdout.strip().endswith("OK"), \
            (out.stdout[-1000:], out.stderr[-3000:])
