"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The input generator (synth/gen.cpp) and the oracle (oracle/rtbte_oracle.c)
are rebuilt with -fsanitize=address,undefined and their test files run in a
child process that preloads the sanitizer runtimes: any invalid access,
overflow or undefined operation ends that process with an error.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = ["tests/test_synth.py", "tests/test_oracle_rhs.py", "tests/test_oracle_delta.py",
         "tests/test_oracle_integrators.py"]


def _env():
    rt = [subprocess.check_output(["gcc", f"-print-file-name={n}"], text=True).strip()
          for n in ("libasan.so", "libubsan.so")]
    assert all(os.path.isabs(p) and os.path.exists(p) for p in rt), rt
    env = dict(os.environ)
    env.update(RTBTE_HOST_SANITIZE="1", LD_PRELOAD=":".join(rt),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    return env


def test_generator_and_oracle_under_asan_and_ubsan():
    import oracle
    import synth
    synth.build_lib(sanitized=True)
    oracle.build_lib(sanitized=True)
    env = _env()
    # the child loads the sanitized builds, not the plain ones
    probe = ("import synth, oracle; synth._lib(); oracle._lib(); "
             "m = open('/proc/self/maps').read(); "
             "print('libsynth_san.so' in m, 'liboracle_san.so' in m, 'libasan' in m)")
    r = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and r.stdout.split() == ["True", "True", "True"], r.stdout + r.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider"] +
                       FILES, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert " passed" in out and " failed" not in out
