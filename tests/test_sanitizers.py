"""Address and undefined-behaviour sanitizer builds of the host code that
reads untrusted bytes (CPU only):

- the oracle (oracle/pmc_oracle.c): the multi-component loop of Alg. 1 with
  both codecs on ragged fields, Eq. (1) checked per component, and every
  stream decoded again with flipped bits and truncated
  (tests/sanitize/oracle_fuzz.c);
- the library's parser of store blobs and stream headers
  (paper_2308_11759_amd/csrc/format.cpp, which has no HIP dependency),
  fuzzed with mutated blobs built around oracle streams
  (tests/sanitize/blob_fuzz.cpp).

Each driver exits non-zero on a failed check, and the sanitizers abort the
run on the first invalid access or undefined operation."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import driver
from paper_2308_11759_amd import inputs

from helpers import store_blob

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip("%s not installed" % tool)


def _run(cmd, timeout):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=ENV)
    assert r.returncode == 0, "%s failed (%d):\n%s\n%s" % (cmd[0], r.returncode, r.stdout[-4000:], r.stderr[-4000:])
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_fuzz")
    _run(["gcc", "-std=c11", "-ffp-contract=off"] + SAN +
         [os.path.join(ROOT, "oracle", "pmc_oracle.c"), os.path.join(HERE, "sanitize", "oracle_fuzz.c"),
          "-o", exe, "-lm"], 300)
    out = _run([exe, "7", "60"], 300)
    assert "0 failures" in out


def test_blob_parser_under_sanitizers(tmp_path):
    _need("g++")
    exe = str(tmp_path / "blob_fuzz")
    _run(["g++", "-std=c++17", "-I" + os.path.join(ROOT, "include")] + SAN +
         [os.path.join(ROOT, "paper_2308_11759_amd", "csrc", "format.cpp"),
          os.path.join(HERE, "sanitize", "blob_fuzz.cpp"), "-o", exe], 300)
    blobs = []
    cases = [((5, 7, 13), np.float32, None, [0.5, 0.05, 5e-3, 5e-4]),   # partial blocks, 1 chunk
             ((21, 18, 30), np.float64, None, [0.3, 0.01, 1e-4]),       # several chunks
             ((9, 22, 17), np.float32, driver.PredictionCodec(), [0.2, 0.02, 2e-3]),
             ((1, 1, 1), np.float64, driver.PredictionCodec(), [1.0])]
    for i, (shape, dt, codec, taus) in enumerate(cases):
        x = (inputs.spectral_field(shape, seed=900 + i, dtype=dt) if min(shape) > 1
             else np.full(shape, 0.75, dtype=dt))
        comps, meta = driver.compress(x, taus, codec)
        path = tmp_path / ("blob%d.bin" % i)
        path.write_bytes(store_blob(x.shape, x.dtype, comps, meta, codec=0 if codec is None else 1))
        blobs.append(str(path))
    out = _run([exe, "11", "3000"] + blobs, 300)
    assert "0 failures" in out
