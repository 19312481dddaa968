"""Writes tests/golden/pointwise_flops.json: the instrumented pointwise flop
counts of the residual and the Jacobian-vector product (oracle.flops), per
physical dimension and convective flux.  Calls only the oracle.

    python tests/golden/make_pointwise_flops.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.flops import pointwise_flops  # noqa: E402


def table():
    return {flux: {str(d): pointwise_flops(d, flux) for d in (2, 3)} for flux in ("roe", "lf")}


if __name__ == "__main__":
    out = {"source": "oracle.flops.pointwise_flops (operation counts of the oracle's pointwise physics "
                     "on a counting number type; per volume point and per face point)",
           "counts": table()}
    with open(os.path.join(HERE, "pointwise_flops.json"), "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
        fh.write("\n")
