"""Child process of tests/test_gpu_launch_env.py: runs small dense, binary,
sparse, brute-force and MIPS problems on cuda:0 and prints one JSON object
of result digests.  The launch-shape environment variables it runs under
are read once per process, which is why this runs as a process of its
own."""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402
import torch  # noqa: E402

import paper_1506_03872_amd as mad  # noqa: E402
import workloads  # noqa: E402


def digest(*arrays):
    h = hashlib.sha1()
    for a in arrays:
        a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()[:16]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def dense_case(A, B, tag, out):
    for order in (0, 1, 2):
        p = mad.Plan.dense(dev(A), dev(B))
        p.set_option(mad.MAD_OPT_SAMPLER_ORDER, order)
        r = p.topk(t=10, s=300000, t_prime=300, seed=5)
        k, x, F = p.scores()
        out["%s_order%d" % (tag, order)] = digest(r["i"], r["j"], r["c"],
                                                  r["x"], k, x)
        p.close()


def main():
    out = {}
    A, B = workloads.dense_gaussian(600, 500, 40, seed=3)
    dense_case(A, B, "dense", out)
    dense_case((A > 0.7).astype(np.float32), (B > 0.7).astype(np.float32),
               "binary", out)
    a = workloads.powerlaw_csr(3000, 400, 8, seed=1, role=0)
    b = workloads.powerlaw_csr(2500, 400, 8, seed=1, role=1)
    p = mad.Plan.csr(tuple(dev(x) for x in a), tuple(dev(x) for x in b),
                     3000, 2500, 400)
    r = p.topk(t=20, s=400000, t_prime=500, seed=7)
    k, x, F = p.scores()
    out["csr"] = digest(r["i"], r["j"], r["c"], r["x"], k, x)
    p.close()
    for prec in (mad.MAD_FP32, mad.MAD_BF16, mad.MAD_FP8_E4M3):
        r, _ = mad.bruteforce_topk(dev(A), dev(B), 10, precision=prec)
        out["bf%d" % prec] = digest(r["i"], r["j"], r["c"])
    Adb, Q, _ = workloads.mips(3000, 40, 6, seed=2)
    s = np.array([100, 3000, 20000, 700, 0, 5000], np.int64)
    tp = np.array([50, 3000, 20000, 700, 10, 40], np.int64)
    mp = mad.MipsPlan.create(dev(Adb))
    res = mp.batch(dev(Q), s, tp, 5, seed=3)
    out["mips"] = digest(*[v for q in res if q is not None
                           for v in (q["i"], q["c"], q["x"])])
    mp.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
