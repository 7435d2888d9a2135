"""CPU sanitizer build: the host-side program compiler (compile.cpp) under a
random-program fuzz, and the oracle (oracle.c) and input generator
(datagen.c) under the CPU tests that drive them, all built with
AddressSanitizer and UndefinedBehaviorSanitizer.  Any report fails."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1806_08384_amd", "csrc")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=undefined"]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                                reason="needs gcc and g++")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    d = tmp_path_factory.mktemp("sanitize")
    fuzz = str(d / "fuzz_compile")
    _run(["g++", "-std=c++17", *SAN, f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
          os.path.join(ROOT, "tests", "sanitize", "fuzz_compile.cpp"),
          os.path.join(CSRC, "compile.cpp"), "-o", fuzz])
    oracle_so = str(d / "liboracle_san.so")
    _run(["gcc", *SAN, "-fPIC", "-shared", "-pthread", os.path.join(ROOT, "oracle", "oracle.c"),
          "-o", oracle_so])
    datagen_so = str(d / "libdatagen_san.so")
    _run(["gcc", *SAN, "-fPIC", "-shared", "-pthread", os.path.join(ROOT, "datagen", "datagen.c"),
          "-lm", "-o", datagen_so])
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    return {"fuzz": fuzz, "oracle": oracle_so, "datagen": datagen_so, "asan": asan}


def test_compiler_fuzz(builds):
    r = _run([builds["fuzz"], "200000"])
    assert "fuzz: 200000 programs" in r.stdout


def test_oracle_and_generator_under_sanitizers(builds):
    """The oracle's pins and the generator's tests, loading the sanitizer
    builds (the runtime preloaded into the interpreter)."""
    if not os.path.isabs(builds["asan"]) or not os.path.exists(builds["asan"]):
        pytest.skip("libasan.so not found")
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": builds["asan"],
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=23",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "SEL_ORACLE_LIB": builds["oracle"],
        "SEL_DATAGEN_LIB": builds["datagen"],
    })
    which = subprocess.run([sys.executable, "-c", "import oracle, datagen; "
                            "print(oracle.load()._name); print(datagen.lib()._name)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert which.stdout.split() == [builds["oracle"], builds["datagen"]], which.stdout + which.stderr
    tests = [os.path.join(ROOT, "tests", f) for f in
             ("test_oracle_pins.py", "test_datagen.py", "test_oracle_spd.py", "test_oracle_estimate.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out
    assert " passed" in r.stdout
