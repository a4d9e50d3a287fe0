"""CPU FP64 oracle for block-based spectral mesh processing (arXiv 1810.02719).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The GPU library never
calls it and shares no code with it; both sides only share the seeded input
generators in ``synth/``.

Each function is a plain, slow, obviously correct restatement of a
definition in the paper (section / equation / algorithm cited in its
docstring), using numpy / scipy / LAPACK as library primitives.  The method
reaches its result exactly only in the converged limit, so the parity target
for the tracked subspace is that limit computed directly: a dense symmetric
eigendecomposition of each block's Laplacian, then projection and
reconstruction.

Modules
-------
laplacian   edge set and Laplacian L = D - C of a submesh (Section 3, Eq. 1-2)
spectral    eigendecomposition, GFT / inverse GFT, principal angles (Section 3, Eq. 3)
metrics     NMSVE and its GL operator (Section 8, Eq. 16), choice of c, the
            residual of Eq. 6
iterations  paper-literal orthogonal iteration (Alg. 1) and dynamic OI (Alg. 2),
            and the exact span of a polynomially filtered subspace iteration
exact       brute-force integer characteristic polynomials, Sturm bisection and
            spanning-tree counts for meshes of <= 10 vertices
merge       degree-weighted merge of overlapped submeshes (Section 6.1, Alg. 3)
codec       uniform quantisation of the feature vectors and the bit rate (Section 8)
"""
