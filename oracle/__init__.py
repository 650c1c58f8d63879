"""FP64 CPU oracle for the pseudo-spectral beta-plane QG time step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
helpers with the HIP library; the two meet only through the seeded input
generators, which hold none of the method's arithmetic.

Contents
--------
fft      -- its own radix-2 Stockham FFT (decimation in time, self-sorting),
            the half-spectrum real transforms built on it.
qg       -- grid, masks D (2/3 rule) and T (test filter), the right-hand side
            of the QG vorticity equation with the four eddy-viscosity closures,
            RK4, the Lie-Trotter penalization/sponge sub-step, one full step,
            diagnostics.
adjoint  -- the exact discrete adjoint of one step (static closures), and the
            gradient of the a-posteriori vorticity loss.
ab2cn    -- the paper's own time scheme: AB2CN for the penalized equations,
            then the AB2 sponge (Sec. II-E, Eq. 4).
les      -- the filter H_full from the fully-resolved grid to the LES grid
            (Sec. III) and the pattern correlation PCC (Sec. IV).

Every floating-point operation is in float64.  Each function cites the
passage of the paper it follows: the QG vorticity equation (Sec. II-A,
Eq. 1), Brinkman penalization (Sec. II-B, Eq. 2), the Fourier pseudo-spectral
discretisation with 2/3 de-aliasing (Sec. II-C), the sponge and the inflow
gauge (Sec. II-D, Eq. 3), the splitting of the time step (Sec. II-E, Eq. 4),
and the closures (Sec. III-A, Eqs. 9-13).

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against brute-force DFTs, closed forms, conservation laws, exact per-step
amplification factors or finite differences.  The nonlinear step with a
closure has no closed form as a whole; it is pinned term by term: the
closure terms by the enstrophy identity and their static coefficient
formulas, the dynamic coefficient by its invariances and a semi-closed form,
the time stepping by exact single-shell amplification and exact decays,
the Jacobian by a two-mode closed form and its conservation laws; and
``tests/test_oracle_mutations.py`` checks that a planted mistake in any of
these terms fails one of the pins.
"""
