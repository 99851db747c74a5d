"""CPU FP64 oracle for the diagrammatic Monte Carlo hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the bench's CPU-baseline leg may import anything from this
package.  The library (C ABI, HIP kernels, Python binding) never calls it and shares no code
with it: the two sides meet only in the seeded input generators of the `synth` package and
in data conventions (sample layout, diagram labelling and routing rule) that each side
implements separately.

Modules, and what pins each (tests/test_oracle_*.py, tests/test_library_cpu.py):
  physics     free propagator, Yukawa interaction, Fock closed forms (Secs. II.A, VI.A).  Pinned: G0
              antiperiodicity, jump and Matsubara transform, d G0/d mu = -G0*G0, the Fock integral against
              its T -> 0 closed forms.
  diagrams    brute-force enumeration, canonical labelling, routing (eq. sigma_integration).  Pinned: the
              Dyson count identity, the relabelling count, momentum conservation.
  integrand   naive diagram-by-diagram FP64 integrand, forward-mode derivatives, the FP32 tolerance,
              uniform map.  Pinned: the order-1 Fock closed forms, the rainbow time integral, central
              differences for the derivatives, an FP32 emulation for the tolerance.
  quadrature  deterministic order-2 results: the static Lindhard function (the bubble's closed loop, spin
              factor and loop sign), the expanded Fock term (the rainbow), Im Sigma^(2) < 0 (the phase).
              Pinned: the T -> 0 Lindhard closed form and dn/dmu of the free gas.
  mc          plain and importance Monte Carlo, and the oracle's own VEGAS (eq. nf_mcmc_estimator_qft_final_
              revised at alpha = 1).  Pinned: the importance sampler against the rainbow quadrature and the
              sign of Im Sigma^(2); the VEGAS estimator composes the pinned map and refinement with the pinned
              C integrand.
  sampler     Philox4x32-10, VEGAS map, inverse map and refinement.  Pinned: Philox known answers, map
              identities, the Jacobian against a numerical determinant.
  flow        affine-coupling flow in FP64 (optional BF16 emulation), its gradient, Adam, mixtures.  Pinned:
              brute-force Jacobians, torch autograd, central differences, unbiased mixtures.
  nsf         rational-quadratic spline flow (Appendix A).  Pinned: brute-force Jacobians, autograd.
  mcmc        Markov chains with independent proposals and the ratio estimator (Sec. IV).  Pinned: closed-
              form integrals, the planted-bias checks.
  taylor      truncated Taylor series in (mu, lambda) with a k tangent (Secs. III.B, VI.A).  Pinned:
              closed forms of n_F, G0 and V series, finite differences.
  renorm      counterterm recursion, xi series and the effective mass (Secs. III.B, VI.A).  Pinned: the
              tree-function (Lagrange inversion) and hand-expanded cases.
  blocks      building-block variables of each diagram by the Dyson-Schwinger and parquet decomposition (Sec.
              II.C).  Pinned: same topology and a unit-Jacobian change of variables against the canonical routing,
              the Dyson count of bare-vertex diagrams, the envelope as the first irreducible block.
  construct   the bottom-up construction of the diagram set from the same equations, with the fully irreducible
              vertices from an orderly generation.  Pinned: the brute-force set, each topology once, at orders 1-6.
  cevaluate   the same integrand in C (evaluate.c, OpenMP) for orders 4-6.  Pinned per sample to
              integrand.py at orders 1-5.
  enumerate.c (built by build.py) the brute-force diagram enumeration in C, for orders 5-6.  Pinned to
              diagrams.py at orders 1-4 and the order-5 golden list.

Parity unpinned: the integrals at orders >= 3 have no closed form; they rest on the per-line rules and
conventions pinned at orders 1-2, the brute-force diagram set, per-sample parity at orders 1-6 and the
integral checks of the GPU tests (independent estimates by the family rule, and same-sample sums).
"""
