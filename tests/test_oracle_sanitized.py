"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) runs every entry point on ragged double-double and
quad-double shapes, Strassen recursions with odd sizes (the padding paths),
one and two threads, in a child process: no invalid access and no undefined
behaviour stops it, and its results are bit for bit those of the normal
build (both builds keep every rounding as written: no contraction, no fast
math)."""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = textwrap.dedent(r"""
    import sys
    import numpy as np
    sys.path.insert(0, sys.argv[2])
    from oracle import cref
    from paper_1710_01839_amd import inputs

    def run():
        out = {}
        for L, gen in ((2, inputs.dd_uniform), (4, inputs.qd_uniform)):
            for (m, n, l) in ((7, 9, 13), (17, 5, 33), (1, 1, 1)):
                A, B = gen(m, l, 3 * m + L), gen(l, n, 5 * n + L)
                for t in (1, 2):
                    out[f"simple{L}_{m}_{t}"] = np.stack(cref.gemm_simple(A, B, threads=t))
                    out[f"exact{L}_{m}_{t}"] = np.stack(cref.gemm_exact(A, B, out_limbs=3, threads=t))
                out[f"abs{L}_{m}"] = cref.absprod_exact(A, B, threads=2)
                C = cref.gemm_simple(A, B)
                out[f"diff{L}_{m}"] = cref.exact_diff(C, cref.gemm_exact(A, B, out_limbs=L + 1))
                out[f"num{L}_{m}"] = np.stack(cref.num_op("mul", A, A) + cref.num_op("add", A, A))
            for (m, n, l) in ((13, 11, 9), (16, 16, 16)):
                A, B = gen(m, l, 7 + L), gen(l, n, 8 + L)
                for d in (1, 2):
                    for v in ("classic", "winograd"):
                        out[f"str{L}_{m}_{d}_{v}"] = np.stack(cref.gemm_strassen(A, B, d, v, threads=2))
        x = np.linspace(-3.0, 3.0, 101) * 1e-3
        y = np.sqrt(np.abs(x) + 1.0)
        out["eft"] = np.stack(cref.two_sum(x, y) + cref.fast_two_sum(y, x) + cref.two_prod(x, y)
                              + cref.two_prod(x, y, use_fma=True))
        return out

    np.savez(sys.argv[1], **run())
""")


def _sanitized_build(tmp):
    so = os.path.join(tmp, "libmpref_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "mpref.c"), "-o", so,
                           "-lm"])
    return so


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    so = _sanitized_build(str(tmp_path))
    script = tmp_path / "child.py"
    script.write_text(CHILD)
    env = dict(os.environ, LD_PRELOAD=asan, MPREF_LIB=so, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    san = tmp_path / "san.npz"
    r = subprocess.run([sys.executable, str(script), str(san), ROOT], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    # the same script on the normal build
    env_plain = {k: v for k, v in os.environ.items() if k != "MPREF_LIB"}
    ref = tmp_path / "ref.npz"
    r = subprocess.run([sys.executable, str(script), str(ref), ROOT], env=env_plain, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    a, b = np.load(san), np.load(ref)
    assert sorted(a.files) == sorted(b.files)
    for k in a.files:
        assert a[k].shape == b[k].shape and np.array_equal(a[k].view(np.int64), b[k].view(np.int64)), k
