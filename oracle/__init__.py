"""Plain, slow FP64 CPU oracle for the Wigner-Eckart factorized collision operator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2605_28475_amd``) never imports, links or calls anything here, and the
two share no code: the oracle evaluates special functions through scipy, builds
its Gaunt table by exact sphere quadrature and its radial core by an exact
Gauss rule in a frame aligned with the relative velocity; the product computes
3j symbols in closed form, uses its own recurrences and quadrature rules, and
integrates the core in a frame aligned with the centre-of-mass velocity.

Modules
-------
basis      Laguerre x real-spherical-harmonic basis (Section 2.2).
gaunt      Real Gaunt table, channel list, COO routing table (Section 4.1-4.2).
weakform   Brute-force 8-D exact quadrature of the weak-form tensor (Section 2.3).
core       Exact reduced radial core R and its invariant zeroing (Sections 3, 4.4).
apply      The factorized discrete sum for Q, evaluated literally (Section 4.5); the
           bilinear form Q(f, g) and the Jacobian-vector product.
rk         Explicit Runge-Kutta integration of dc/dt = Q(c) (Section 5).
"""
