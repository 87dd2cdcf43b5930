"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host code only): a
small driver runs its public entry points (render on one and two threads, records, 16-bit
readout, eq. 9 map, particle displacement, an optical chain, Mie weights) on the tiny BOS scene
at a reduced size, with every sanitizer report fatal, and its Q32.32 image must equal the one the
regular oracle build renders from the same inputs."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1812_05902_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include "ORACLE_C"
#include <stdio.h>

static void *slurp(const char *path, size_t *n)
{
    FILE *f = fopen(path, "rb");
    if (!f) { perror(path); exit(2); }
    fseek(f, 0, SEEK_END);
    long k = ftell(f);
    fseek(f, 0, SEEK_SET);
    void *p = malloc((size_t)k);
    if (fread(p, 1, (size_t)k, f) != (size_t)k) { perror(path); exit(2); }
    fclose(f);
    *n = (size_t)k;
    return p;
}

int main(int argc, char **argv)
{
    size_t ncfg, nrho, nsrc;
    orc_cfg *cfg = (orc_cfg *)slurp(argv[1], &ncfg);
    float *rho = (float *)slurp(argv[2], &nrho);
    float *src = (float *)slurp(argv[3], &nsrc);
    if (ncfg != sizeof(orc_cfg) || nrho != (size_t)cfg->nx * cfg->ny * cfg->nz * 4) return 3;
    const int64_t n_src = (int64_t)(nsrc / 16);
    const int32_t rps = atoi(argv[4]);
    orc_scene *S = orc_create(cfg, rho);
    if (!S) return 4;
    const size_t npx = (size_t)cfg->width * cfg->height;
    uint64_t *q1 = calloc(npx, 8), *q2 = calloc(npx, 8), counts[8] = {0};
    double *f1 = calloc(npx, 8);
    orc_render(S, src, n_src, rps, q1, f1, counts, 1);
    orc_render(S, src, n_src, rps, q2, NULL, NULL, 2);
    for (size_t p = 0; p < npx; ++p) if (q1[p] != q2[p]) return 5;
    FILE *out = fopen(argv[5], "wb");
    fwrite(q1, 8, npx, out);
    fclose(out);
    /* records, readout, field and integration outside the box */
    int64_t ids[7] = {0, 1, 2, rps, rps + 1, n_src * rps - 2, n_src * rps - 1};
    orc_ray rec[7];
    orc_trace_ids(S, src, rps, ids, 7, rec, 1);
    uint16_t *u16 = calloc(npx, 2);
    orc_readout_u16(q1, (int64_t)npx, 0.0, u16);
    orc_readout_u16(q1, (int64_t)npx, 3.0, u16);
    double R[3] = {-1.0, 2.0, 0.5}, T[3] = {0.0, 0.0, 1.0}, fv[4];
    orc_field_eval(S, R, fv);
    orc_rkn_integrate(S, R, T, 1e-4, 5);
    /* eq. 9 map over a small grid */
    double *map = calloc(5 * 4 * 2, 8);
    orc_bos_theory_map(S, -0.01, -0.01, 0.005, 0.005, 5, 4, src[2], 16, map);
    /* particles moved through a 4 x 3 x 2 velocity grid */
    float vel[2 * 3 * 4 * 3];
    for (int k = 0; k < 2 * 3 * 4 * 3; ++k) vel[k] = 0.01f * (float)(k % 7) - 0.03f;
    const double org[3] = {-0.03, -0.03, -0.01}, sp[3] = {0.02, 0.03, 0.02};
    double *moved = calloc((size_t)n_src * 4, 8);
    orc_displace_sources(src, n_src, vel, 4, 3, 2, org, sp, 1e-3, 4, moved);
    /* an optical chain: stop, two refracting surfaces */
    orc_surface ch[3];
    memset(ch, 0, sizeof ch);
    ch[0].type = ORC_SURF_APERTURE; ch[0].z = cfg->z_lens; ch[0].clear = 0.003;
    ch[1].type = ORC_SURF_REFRACT; ch[1].z = cfg->z_lens + 1e-3; ch[1].radius = 0.05; ch[1].clear = 0.01;
    ch[1].n_after = 1.5;
    ch[2].type = ORC_SURF_REFRACT; ch[2].z = cfg->z_lens + 6e-3; ch[2].radius = -0.05; ch[2].clear = 0.01;
    orc_set_chain(S, ch, 3, cfg->z_lens, 0.003);
    memset(q2, 0, npx * 8);
    orc_render(S, src, n_src, rps, q2, NULL, NULL, 1);
    orc_set_chain(S, ch, 0, 0.0, 0.0);
    /* Mie weights from a 33-entry table */
    double tab[33];
    for (int k = 0; k < 33; ++k) tab[k] = 1.0 / (1.0 + k);
    const double laser[3] = {1.0, 0.0, 0.0};
    orc_set_mie(S, tab, 33, laser);
    memset(q2, 0, npx * 8);
    orc_render(S, src, n_src, rps, q2, NULL, NULL, 1);
    orc_destroy(S);
    free(q1); free(q2); free(f1); free(u16); free(map); free(moved); free(cfg); free(rho); free(src);
    printf("deposited %llu steps %llu\n", (unsigned long long)counts[0], (unsigned long long)counts[7]);
    return 0;
}
"""


def _sanitizer_works(tmp_path) -> bool:
    if shutil.which("gcc") is None:
        return False
    c = tmp_path / "probe.c"
    c.write_text("int main(void){return 0;}\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined", str(c), "-o", str(tmp_path / "probe")],
                       capture_output=True)
    return r.returncode == 0


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    if not _sanitizer_works(tmp_path):
        pytest.skip("gcc with libasan/libubsan not available")
    sc = inputs.tiny_bos().replace(nx=12, ny=11, nz=10, n_src=23, rays_per_src=17)
    rho = np.ascontiguousarray(inputs.density(sc), dtype=np.float32)
    src = np.ascontiguousarray(inputs.sources(sc), dtype=np.float32)
    cfg = oracle.cfg_from_scene(sc)
    (tmp_path / "cfg.bin").write_bytes(bytes(cfg))
    (tmp_path / "rho.bin").write_bytes(rho.tobytes())
    (tmp_path / "src.bin").write_bytes(src.tobytes())
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER.replace("ORACLE_C", os.path.join(ROOT, "oracle", "oracle.c")))
    exe = tmp_path / "driver"
    subprocess.check_call(["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", str(drv), "-o", str(exe), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe), str(tmp_path / "cfg.bin"), str(tmp_path / "rho.bin"), str(tmp_path / "src.bin"),
                        str(sc.rays_per_src), str(tmp_path / "img.bin")],
                       capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    img = np.frombuffer((tmp_path / "img.bin").read_bytes(), dtype=np.uint64)
    q, _, _ = oracle.scene_oracle(sc, rho=rho).render(src, sc.rays_per_src, want_float=False)
    assert img.sum() > 0
    assert np.array_equal(img, np.asarray(q).reshape(-1))
