"""Every launch-shape environment variable the library reads (stream use,
grids, samples in flight, LDS budgets, bin targets and table sizes) is
result-invariant: a child process under a set of overrides must return
what a child process under the defaults returns, for dense (under each
sample order), binary, sparse, brute-force and MIPS problems."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))

OVERRIDES = {
    "MAD_TABLES_ONE_STREAM": "1",   # the B side and T0 on the caller's stream
    "MAD_SAMPLER_UNROLL": "2",      # unordered dense sampler
    "MAD_SAMPLER_GRID": "64",
    "MAD_SAMPLER_G8": "3",          # k-ordered sampler
    "MAD_PIPE_G8": "8",             # three-pass order
    "MAD_BINARY_BITMAP": "0",       # binary B read from B itself
    "MAD_SMALL_LDS": "4096",        # one small table per block
    "MAD_ACC_TARGET": "1024",       # accumulation bins
    "MAD_ACC_SLOTS": "8192",
    "MAD_BF_GRID": "16",            # brute force
    "MAD_CSR_GRID": "256",          # sparse sampler
    "MAD_CSR_UNROLL": "2",
}


def run_child(extra):
    env = {k: v for k, v in os.environ.items() if k not in OVERRIDES}
    env.update(extra)
    r = subprocess.run([sys.executable, os.path.join(HERE,
                                                     "launch_env_child.py")],
                       env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_launch_shape_overrides_keep_every_result(gpu):
    base = run_child({})
    print("defaults", base, flush=True)
    alt = run_child(OVERRIDES)
    print("overrides", alt, flush=True)
    assert base.keys() == alt.keys()
    for k in base:
        assert base[k] == alt[k], k
