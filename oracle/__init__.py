"""Oracle: a plain, slow, complex-FP64 CPU implementation of the trace estimator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only the tests, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (no kernels, headers, helpers or tables); the two meet only through
the seeded inputs of `synth`.

Contents, each following the paper's definitions (Frommer et al., "Variance
reduction with probing and Multilevel Monte Carlo in Lattice QCD"):

- gamma      DeGrand-Rossi Dirac matrices (the operator's spin structure).
- geometry   site indexing, periodic/antiperiodic neighbours.
- dirac      the Wilson-Dirac matrix D as a dense or sparse matrix (Sec. 1).
- noise      SplitMix64 counter noise, Rademacher and probing vectors with
             spin-colour and time dilution (Sec. 1, Sec. 3, eq. "probing vectors").
- colouring  torus colouring c(x) = sum_j sigma_j x_j mod n_c, its exhaustive
             search and a brute-force distance check (Sec. 3, eq. coloring-formula).
- solve      dense LU and a textbook BiCGStab (D x = eta, Sec. 1).
- estimator  Hutchinson / probing estimators, exact traces, the Rademacher
             variance formula and its probing generalisation (Sec. 1, Sec. 3, Sec. 4).
- force      derivatives of eta^dag D^-1 eta with respect to m0 and the links.

Parity status: every function here is pinned by a `-m "not gpu"` test against
a closed form, brute force or an exact identity, except where a docstring
says "parity unpinned".
"""
