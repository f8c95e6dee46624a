"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only, built with gcc): a test program runs every entry point over frames with
edge blocks, both block sizes, ranges 1..7, learned starts at and beyond the
window corners, both DCDS variants and cost surfaces with holes.  Any
out-of-bounds access, leak or undefined operation aborts the test program."""
import os
import shutil
import subprocess

import pytest

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "me_oracle.c")

PROGRAM = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_fs(const uint8_t *, const uint8_t *, int, int, int, int, int, int16_t *, uint32_t *, uint32_t *);
int oracle_dcds(const uint8_t *, const uint8_t *, int, int, int, int, int, const int16_t *, const uint8_t *, int,
                int16_t *, uint32_t *, uint32_t *);
int oracle_dcds_surface(int, const int64_t *, const uint8_t *, int, int, int, int, int, int16_t *, int64_t *,
                        uint32_t *, uint8_t *, uint32_t *, int, int *);
int64_t oracle_block_sad(const uint8_t *, const uint8_t *, int, int, int, int, int, int, int, int);

static uint32_t seed = 12345u;
static uint32_t rnd(void) { seed = seed * 1664525u + 1013904223u; return seed >> 8; }

static int run_frames(int W, int H, int pitch, int B, int R) {
    uint8_t *cur = malloc((size_t)pitch * H), *ref = malloc((size_t)pitch * H);
    int nb = (W / B) * (H / B);
    int16_t *mv = malloc(sizeof(int16_t) * 2 * nb), *st = malloc(sizeof(int16_t) * 2 * nb);
    uint8_t *orient = malloc((size_t)nb);
    uint32_t *sad = malloc(sizeof(uint32_t) * nb), *nsp = malloc(sizeof(uint32_t) * nb);
    for (int i = 0; i < pitch * H; ++i) { cur[i] = (uint8_t)rnd(); ref[i] = (uint8_t)(cur[i] + (rnd() % 9) - 4); }
    int rc = oracle_fs(cur, ref, W, H, pitch, B, R, mv, sad, nsp);
    for (int v = 0; v < 2 && !rc; ++v) {
        rc |= oracle_dcds(cur, ref, W, H, pitch, B, R, NULL, NULL, v, mv, sad, nsp);
        for (int b = 0; b < nb; ++b) {  /* starts inside, on and beyond the window */
            st[2 * b] = (int16_t)((int)(rnd() % (4 * R + 3)) - 2 * R - 1);
            st[2 * b + 1] = (int16_t)((int)(rnd() % (4 * R + 3)) - 2 * R - 1);
            orient[b] = (uint8_t)(rnd() & 1);
        }
        rc |= oracle_dcds(cur, ref, W, H, pitch, B, R, st, orient, v, mv, sad, nsp);
    }
    for (int k = 0; k < 64; ++k)
        (void)oracle_block_sad(cur, ref, W, H, pitch, B, (int)(rnd() % (W / B)) * B, (int)(rnd() % (H / B)) * B,
                               (int)(rnd() % (2 * R + 3)) - R - 1, (int)(rnd() % (2 * R + 3)) - R - 1);
    free(cur); free(ref); free(mv); free(st); free(orient); free(sad); free(nsp);
    return rc;
}

static int run_surface(int R) {
    int n = (2 * R + 1) * (2 * R + 1);
    int64_t *cost = malloc(sizeof(int64_t) * n), bdm = 0;
    uint8_t *valid = malloc((size_t)n), *s_out = malloc((size_t)n);
    uint32_t trace[4096], nsp = 0;
    int16_t mv[2];
    int tn = 0, rc = 0;
    for (int t = 0; t < 50 && !rc; ++t) {
        for (int i = 0; i < n; ++i) { cost[i] = (int64_t)(rnd() % 1000); valid[i] = (uint8_t)((rnd() % 5) != 0); }
        valid[n / 2] = 1;
        int sx = (int)(rnd() % (2 * R + 1)) - R, sy = (int)(rnd() % (2 * R + 1)) - R;
        rc |= oracle_dcds_surface(R, cost, valid, sx, sy, (int)(t & 1), (int)((t >> 1) & 1), (int)((t >> 2) & 1),
                                  mv, &bdm, &nsp, s_out, trace, 4096, &tn);
    }
    free(cost); free(valid); free(s_out);
    return rc;
}

int main(void) {
    static const int cases[][5] = {{48, 32, 48, 16, 7}, {64, 64, 68, 16, 3}, {40, 24, 40, 8, 7}, {24, 16, 28, 8, 1},
                                   {16, 16, 16, 16, 7}, {32, 48, 36, 8, 5}};
    int rc = 0;
    for (unsigned c = 0; c < sizeof(cases) / sizeof(cases[0]); ++c)
        rc |= run_frames(cases[c][0], cases[c][1], cases[c][2], cases[c][3], cases[c][4]);
    for (int R = 1; R <= 7; ++R) rc |= run_surface(R);
    printf("rc %d\n", rc);
    return rc != 0;
}
"""


def build_and_run(tmp_path, source):
    drv = tmp_path / "prog.c"
    drv.write_text(source)
    exe = tmp_path / "prog"
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-o", str(exe), str(drv), ORACLE]
    try:
        subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=120)
    except subprocess.CalledProcessError as e:
        if "asan" in (e.stderr or "").lower() or "libubsan" in (e.stderr or "").lower():
            pytest.skip("sanitizer runtime not available: %s" % e.stderr[-200:])
        raise
    return subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                          env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(tmp_path):
    r = build_and_run(tmp_path, PROGRAM)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "rc 0" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_the_instrumentation_is_live(tmp_path):
    """A one-byte write past a frame buffer, planted in a copy of the program,
    must be reported: the clean run above then means something."""
    planted = PROGRAM.replace("free(cur); free(ref);", "cur[pitch * H] = 1; free(cur); free(ref);")
    assert planted != PROGRAM
    r = build_and_run(tmp_path, planted)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr
