"""CPU oracle for the Burgers-Hopf characteristic-function PDE in TT format.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` do.

The oracle is a plain, slow, obviously-correct restatement of what the
method computes, in complex float64 (numpy / scipy), written from the paper
(Rodgers & Venturi, "Tensor approximation of functional differential
equations"):

* ``galerkin``     - Fourier basis, the Galerkin coefficients B and D
                     (Sec. 3 eq. (coefficients), Sec. 5 eq. (eqn:BHfde)).
* ``fd``           - the tensor-product grid and 1-D finite-difference
                     operators (Sec. 4 eq. (tt)/(eqn:ode), Sec. 5).
* ``fullgrid``     - the semi-discrete operator on the full grid, classical
                     RK4, and step-truncation with full-grid TT-SVD
                     (Sec. 4.1 eq. (eqn:discrete-flow-trunc-intro)).
* ``cdf``          - the CDF equation of the stochastic Burgers equation
                     with reaction (Sec. 5, eq. (eqn:cdf-burgers)) on the
                     full grid, and its closed-form pins.
* ``closed_forms`` - exact solutions used as pins (viscous-only transport,
                     per-axis matrix exponential, deterministic initial state).
* ``tt_ref``       - TT format arithmetic written from App. A.1
                     (iterated matrix product, sum by concatenation,
                     orthogonalisation and truncation, Alg. 1 / Alg. 2),
                     plus pointwise evaluation of the operator applied to a
                     TT, usable at any dimension.

It shares no code, header, table or constant with the HIP path.  Inputs
(initial-condition parameters, random TT cores, sample points) are passed
in as arrays; the oracle draws no random numbers itself.

Parity status per function is stated in each module header.  Every function
here is pinned by a ``-m "not gpu"`` test in ``tests/test_oracle_*.py``,
directly or through the pinned function that calls it (helpers such as the
one-axis propagator or the shifted solve), against a closed form, an
invariant, a hand-derived value or a brute-force computation.  What the
pins cannot fix is where the truncated steps place their truncations:
that is a reading of Sec. 4.1 shared with the device path (each
truncation's arithmetic is pinned: a step without truncation is the
classical scheme, and a truncation is the full-grid TT-SVD, which equals
the TT rounding).
"""
