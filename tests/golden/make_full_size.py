"""Writes tests/golden/full_size.json: the float64 oracle's results on the
full-size workloads (400^3, 64^5 and 1000^3), on the exact bytes that
synth.make_host produces for them.  It calls only synth (data) and oracle/.

For each workload the file holds
  fingerprint : ||X||^2 (float64 sum over the stored values), sum |X|, and
                32 stored values at fixed linear indices, so that a test can
                confirm it regenerated the same tensor before using the
                numbers below;
  oracle      : the relative reconstruction error of rBKI-TK (Alg. 2), the
                per-mode relative eigen-gap (lam_R - lam_{R+1}) / lam_1 of Z,
                the basis widths, and 32 sampled entries of each projector
                U_n U_n^T (independent of factor signs);
  htr         : (64^5 only) the error of rBKI-TK-TR (Alg. 3, TR-SVD branch),
                from the explicit Tucker residual and the explicit residual
                of the TR-SVD of the core;
  htr_als     : (64^5 only) the same with the TR-ALS branch (Gaussian start
                from the sketch stream, Sec. 4 stopping rule), and its sweep
                count.

Run from the repository root:  python tests/golden/make_full_size.py [names]
(about 25 minutes and 45 GB of host memory for all three on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.rbki import rbki_tucker  # noqa: E402
from oracle.tensor import fro  # noqa: E402
from oracle.trsvd import rbki_htr, tr_als, tr_to_full  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size.json")
NAMES = ("tucker400_f32", "ring64x5_f32", "tucker1000_f32")


def projector_samples(U, count=32, seed=54321):
    """Entries (i, j) of U U^T at fixed random positions, the first 8 on the
    diagonal."""
    I = U.shape[0]
    rng = np.random.default_rng(seed)
    ii = rng.integers(0, I, size=count)
    jj = rng.integers(0, I, size=count)
    jj[:8] = ii[:8]
    vals = [float(U[i] @ U[j]) for i, j in zip(ii, jj)]
    return {"i": [int(v) for v in ii], "j": [int(v) for v in jj], "values": vals}


def oracle_record(infos, factors, ranks):
    gaps, widths, proj = [], [], []
    for info, U, R in zip(infos, factors, ranks):
        lam = info["eigenvalues"]
        gaps.append(float((lam[R - 1] - lam[R]) / lam[0]) if lam.size > R else 1.0)
        widths.append([int(v) for v in info["widths"]])
        proj.append(projector_samples(U))
    return {"eig_gap": gaps, "widths": widths, "projector": proj}


def run(name):
    w = synth.WORKLOADS[name]
    t0 = time.time()
    X, Xc = synth.make_host(w)
    del Xc
    rec = {"dims": list(w["dims"]), "ranks": list(w["ranks"]), "p": w["p"], "q": w["q"],
           "seeds": list(w["seeds"]), "dtype": w["dtype"], "fingerprint": synth.fingerprint(X)}
    print(name, "generated in %.1f s" % (time.time() - t0), flush=True)
    t0 = time.time()
    if w["kind"] == "ring":
        _, err, info = rbki_htr(X, w["ranks"], w["p"], w["q"], w["seeds"][1], w["tr_ranks"],
                                explicit_error="core")
        # the Tucker step of Alg. 3 is rBKI-TK itself; its intermediate
        # results come back in info
        nx2 = rec["fingerprint"]["norm2"]
        rec["htr"] = {"tr_ranks": list(w["tr_ranks"]), "rel_err": err,
                      "core_gap2_rel": info["core_gap2"] / nx2, "discarded_rel": info["discarded"] / nx2}
        e_tk, factors, infos = info["tucker_error"], info["factors"], info["tucker_infos"]
        # the TR-ALS branch of Alg. 3 on the same core, from its start of the
        # sketch stream
        als_cores, sweeps = tr_als(info["G"], w["tr_ranks"], seed=w["seeds"][1])
        gap2 = fro(info["G"] - tr_to_full(als_cores)) ** 2
        rec["htr_als"] = {"tr_ranks": list(w["tr_ranks"]), "sweeps": int(sweeps), "max_sweeps": 20,
                          "fit_tol": 1e-3, "core_gap2_rel": gap2 / nx2,
                          "rel_err": float(np.sqrt((e_tk ** 2) + gap2 / nx2))}
    else:
        _, factors, e_tk, infos = rbki_tucker(X, w["ranks"], w["p"], w["q"], w["seeds"][1], return_info=True)
    rec["oracle"] = {"rel_err": e_tk, **oracle_record(infos, factors, w["ranks"])}
    rec["oracle_seconds"] = time.time() - t0
    print(name, "oracle error %.15g in %.1f s" % (e_tk, time.time() - t0), flush=True)
    return rec


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        data[name] = run(name)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or NAMES)
