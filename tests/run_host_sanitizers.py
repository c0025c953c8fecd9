"""Host sanitizer tier: builds the library's host code and the oracle with
AddressSanitizer and UndefinedBehaviorSanitizer and runs the CPU tests
(-m "not gpu") against those builds, in a child process that preloads the
sanitizer runtime (Python itself is not instrumented).  Any sanitizer
report ends the run with a failure.

    python tests/run_host_sanitizers.py [extra pytest arguments]
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def main(argv):
    from oracle import build as obuild
    from paper_2212_14201_amd import build as qbuild
    qlib = qbuild.build(sanitize=True)
    olib = obuild.build(sanitize=True)
    rt = subprocess.run([obuild.CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True, check=True).stdout.strip()
    if not os.path.exists(rt):
        raise SystemExit(f"sanitizer runtime not found: {rt}")
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": rt,
        # torch and numpy keep allocations alive until exit: leaks are not checked
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "QVM_LIBRARY": qlib,
        "QVM_ORACLE_LIBRARY": olib,
        "OMP_NUM_THREADS": env.get("OMP_NUM_THREADS", "4"),
    })
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-m", "not gpu", "-q", "-x",
           "-p", "no:cacheprovider"] + argv
    print("sanitized run:", " ".join(cmd), flush=True)
    return subprocess.run(cmd, env=env, cwd=ROOT).returncode


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
