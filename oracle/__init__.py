"""CPU FP64 oracle for the diagrammatic Monte Carlo hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the bench's CPU-baseline leg may import anything from this
package.  The library (C ABI, HIP kernels, Python binding) never calls it and shares no code
with it: the two sides meet only in the seeded input generators of the `synth` package and
in data conventions (sample layout, diagram labelling and routing rule) that each side
implements separately.

Modules:
  physics    free propagator, Yukawa interaction, Fock closed forms (Secs. II.A, VI.A)
  diagrams   brute-force enumeration, canonical labelling, routing (eq. sigma_integration)
  integrand  naive diagram-by-diagram FP64 integrand, forward-mode derivatives, uniform map
  mc         plain Monte Carlo (eq. nf_mcmc_estimator_qft_final_revised at alpha = 1)
  sampler    Philox4x32-10, VEGAS map, inverse map and refinement
  flow       affine-coupling flow in FP64 (optional BF16 emulation), its gradient, Adam, mixtures
  mcmc       Markov chains with independent proposals and the ratio estimator (Sec. IV)
  taylor     truncated Taylor series in (mu, lambda) with a k tangent (Secs. III.B, VI.A)
  renorm     counterterm recursion, xi series and the effective mass (Secs. III.B, VI.A)
  enumerate.c (built by build.py) the brute-force diagram enumeration in C, for orders 5-6

Parity status: orders 1-2 are pinned to closed forms (Fock integral, rainbow time integral,
G0 identities); the diagram set at every order is pinned by the Dyson count identity and
the relabelling count.  The per-sample values of orders >= 3 rest on the same line rules
(parity pinned through the order-1/2 checks of every rule they use) -- there is no closed
form for their integrals (integral parity unpinned at orders >= 3).
"""
