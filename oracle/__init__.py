"""CPU oracle for the exact RNG / GRNG build -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything in this package.  The
product library (``paper_2208_10022_amd``) never does, and the two share no
code: no kernels, headers, helpers, tables or pre/post-processing.

What the oracle computes is the plain definitions, not the paper's staged,
pivot-pruned method (every pruning step of the method is a theorem, so the
method reaches exactly these results):

* RNG: pair (u, v) is linked iff no third point lies strictly inside their
  lune, i.e. no z with max(d(u,z), d(v,z)) < d(u,v)  (Section 1, the RNG
  definition equation; ties keep the edge).
* GRNG of a pivot layer: pivots i, j are linked iff no pivot k lies in the
  generalized lune d(k,i) < d(i,j) - (2 r_i + r_j) and
  d(k,j) < d(i,j) - (r_i + 2 r_j)  (Section 2, Definition of the GRNG).
* Pivot domains: x belongs to D(p, r) iff d(x, p) <= r (Section 1, pivot
  domain equation); a fine pivot belongs to a coarse relative domain iff
  d(p, p') <= r - r' (Section 3).
* The query neighbourhood, the insertion result and the intermediates of the
  staged method (delta_max, mu_max) by their definitions.

Arithmetic: inputs are float32 values on a dyadic grid (k * 2**-q), so every
squared distance is an exact integer in units of 2**-2q.  The oracle works on
those integers (numpy int64, Python int, C int64 / __int128), never on rounded
values, so every decision it takes is the exact real-number decision.

Modules:
  ``exact``   exact grid integers, squared distances, the exact predicate
              "sqrt(a) + c < sqrt(b)", high-precision cross-checks.
  ``rng``     RNG / Gabriel graph / query rows by definition (O(N^3), small N).
  ``grng``    GRNG layer, domains, relative domains, virtual-pivot GRNG,
              delta_max and mu_max by definition (small M).
  ``native``  ctypes loader of the C oracle (``rng_oracle.c``) for large N.
  ``mlp``     float64 forward / backward of the witness-ranking MLP.
"""
