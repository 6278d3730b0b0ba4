"""FP64 CPU oracle of the IEWPF ensemble forecast + analysis (arXiv:1910.01031).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link this
package: only the tests, the smoke check and the benchmark's CPU-baseline leg use it.

It is a plain NumPy (float64) statement of what the paper computes, written from the
paper's equations and in the order of its steps, sharing no code with the HIP library:

  philox        counter-based Philox4x64-10 + Box-Muller normals (random streams)
  swe           rotating shallow-water central-upwind scheme, SSP-RK2 (Section
                "The simplified ocean model", eq. swe_full, eq. swecfl)
  model_error   SOAR on the coarse random grid, bicubic interpolation, geostrophic
                balance (Section "Small scale model errors")
  observe       observation operator, eta-compensated innovations, mooring and
                drifter observations (Section "Synthetic truth and observations")
  iewpf         S, the optimal-proposal pull, perpendicular random vectors, beta,
                alpha (Lambert W), local P^{1/2} and the posterior update (Section
                "Efficient implementation of the IEWPF scheme", Appendix A)
  lambertw      principal-branch Lambert W for the alpha equation
  drifters      passive drifter advection
  resample      SIR weights and residual resampling (Section "Standard particle filter")

Functions whose result no independent pin reaches are marked "parity unpinned" in
their docstrings.
"""
