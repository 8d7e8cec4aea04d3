"""Write the stored expected values under tests/golden/ from the oracle only.

Inputs come from the seeded generator (``synth``); expected values come from
the oracle (``oracle``); nothing here touches the HIP library.  Re-running it
must reproduce the committed files byte for byte (checked by
tests/test_golden_files.py).

Usage:  python tests/golden/make_golden.py [--large]
        (--large also writes the full-size digests, minutes of CPU time)
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import exact, grng, native, rng  # noqa: E402


def edges_text(E, header):
    lines = ["# " + h for h in header] + ["%d %d" % (u, v) for u, v in np.asarray(E).reshape(-1, 2)]
    return "\n".join(lines) + "\n"


def files():
    out = {}
    W = synth.uniform2d(1000)
    E = rng.rng_edges(exact.to_grid(W.X, W.q))
    out["uniform2d_n1000_rng_edges.txt"] = edges_text(E, [
        "RNG of 1,000 points i.i.d. uniform in [0,1)^2 (synth.uniform2d(1000)),",
        "by the definition (Section 1, RNG equation) with the O(N^3) oracle.",
        "Each line: u v with u < v, sorted."])
    W = synth.clustered(n=3000, d=16, clusters=8, m=60, knn=40)
    E = native.rng_edges(W.X, W.q)
    out["clustered_n3000_d16_rng_edges.txt"] = edges_text(E, [
        "RNG of synth.clustered(n=3000, d=16, clusters=8, m=60, knn=40) points,",
        "by the definition (Section 1, RNG equation) with the C oracle."])
    L = W.layers[0]
    G = grng.grng_edges(exact.to_grid(W.X[L.pivot_ids], W.q), exact.radius_to_grid(L.radii, W.q))
    out["clustered_n3000_d16_m60_grng_edges.txt"] = edges_text(G, [
        "GRNG of the 60 pivots of synth.clustered(n=3000, d=16, clusters=8, m=60, knn=40)",
        "by Definition 1 (Section 2); indices are positions in the pivot list."])
    return out


def edge_digest_text(E, header):
    """Edge count and the sha256 of the canonical int32 (u, v) array, as the
    library returns it (little-endian, u < v, sorted)."""
    import hashlib
    A = np.ascontiguousarray(np.asarray(E, dtype="<i4").reshape(-1, 2))
    lines = ["# " + h for h in header] + ["edges %d" % len(A), "sha256 %s" % hashlib.sha256(A.tobytes()).hexdigest()]
    return "\n".join(lines) + "\n"


def large_files():
    """Digests of full edge sets that take the C oracle minutes (not rerun by the CPU suite)."""
    out = {}
    W = synth.clustered()
    E = native.rng_edges(W.X, W.q)
    out["clustered_n100000_d16_rng_digest.txt"] = edge_digest_text(E, [
        "RNG of synth.clustered() (100,000 points, 16-D, 32 clusters) by the definition",
        "(Section 1, RNG equation) with the C oracle: edge count and sha256 of the",
        "canonical little-endian int32 (u < v, sorted) array."])
    return out


if __name__ == "__main__":
    native.build(force=False)
    todo = dict(files())
    if "--large" in sys.argv:
        todo.update(large_files())
    for name, text in todo.items():
        with open(os.path.join(HERE, name), "w") as f:
            f.write(text)
        print("wrote", name, text.count("\n"), "lines")
