"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): it is rebuilt with -fsanitize=address,undefined into a temporary
directory and a child Python process (with the ASan runtime preloaded) runs
every step on small sets -- brute force, keys, sort, tree, moments, groups,
lists (both opening criteria), same-list force, potential, quadrupole term,
adjoint and the error magnitudes -- and checks them against the regular
build.  Any out-of-bounds access, use after free or undefined behaviour
aborts the child with a sanitizer report."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent("""
    import sys
    import numpy as np
    sys.path.insert(0, {root!r})
    import oracle, synth
    oracle._LIB_PATH = {lib!r}
    oracle._lib = None
    def run(ps, params):
        ot = oracle.OracleTree(ps.x, ps.y, ps.z, ps.m, params)
        w = synth.loss_weights(ps.n, 5)
        out = [ot.force(), ot.potential(), ot.force_quadrupole(), *ot.adjoint(w), ot.force_bound(2.0 ** -24),
               *ot.adjoint_bound(w, 2.0 ** -24)]
        bf = oracle.brute_force(ps.x, ps.y, ps.z, ps.m, 1.0, params.r_cut, params.eps)
        bfa = oracle.brute_force_adjoint(ps.x, ps.y, ps.z, ps.m, w, 1.0, params.r_cut, params.eps)
        return out + [bf, *bfa]
    res = []
    ps = synth.small_clustered(1500, 3, r_cut=0.08, eps=3e-4, theta=0.5, per_halo=300)
    res += run(ps, ps.params)
    res += run(ps, synth.Params(1.0, 0.08, 3e-4, 0.7, 8, 4, 1))
    rng = np.random.default_rng(4)
    co = np.concatenate([np.full((80, 3), 0.25), rng.random((120, 3))])
    pc = synth.ParticleSet(co[:, 0].copy(), co[:, 1].copy(), co[:, 2].copy(), np.full(200, 1 / 200),
                           synth.Params(1.0, 0.1, 1e-3, 0.5, 16, 16))
    res += run(pc, pc.params)
    np.savez({out!r}, *res)
    print("CHILD_OK", flush=True)
""")


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.exists(asan):
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    src = os.path.join(ROOT, "oracle", "srf_oracle.c")
    subprocess.run(["gcc", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-std=c11", "-shared", "-fPIC",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-o", lib, src, "-lm"], check=True)
    out_san = str(tmp_path / "san.npz")
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib, out=out_san)], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "CHILD_OK" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
    # the same computation with the regular build gives the same numbers
    import oracle

    out_ref = str(tmp_path / "ref.npz")
    r2 = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=oracle.build(force=False), out=out_ref)],
                        capture_output=True, text=True, timeout=600, env=dict(os.environ, OMP_NUM_THREADS="2"))
    assert r2.returncode == 0, r2.stderr[-2000:]
    import numpy as np

    a, b = np.load(out_san), np.load(out_ref)
    assert a.files == b.files
    for k in a.files:
        assert np.allclose(a[k], b[k], rtol=1e-12, atol=1e-300), k
