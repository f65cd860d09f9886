"""Self-check of the pins: plant one plausible mistake at a time in the oracle
(on the CPU) and require that at least one pin fails.  The mistakes exist only in
the separate mutant build liboracle_mut.so (-DORC_MUTANTS); oracle.set_mutant()
switches to it and back.

Mutants (see MUT(k) in oracle/hydro_oracle.c):
 1 S_T^tau sign, 2 sign of the pi u~^tau/tau term, 3 sign of I^{mu nu},
 4 missing u~^tau/tau extra in nabla~_eta u~^eta, 5 Delta_eta = deta (no tau),
 6 sign of the u b term, 7 wrong trace coefficient in sigma, 8 local speed
 without the sound speed, 9 sign of the right-state reconstruction,
 10 transposed gradient in D~u~, 11 wrong velocity normalisation in the root
 solve, 12 EoS T interpolation off by one node, 13 no ideal first-step
 estimate, 14 stage-2 T flux with pi' instead of pi^{n+1}, 15 tau_pi = 3 eta/(sT),
 17 sign of the lambda_1 term, 18 projected pi pi without its trace part,
 19 tau_pi coefficient fixed at 5 (ignoring the configured one), 20 pi pi
 contracted without the metric; freeze-out surface: 21 flipped face difference
 (S pointing into the hot region), 22 a dropped term of the two-hot-vertex
 tetrahedron fraction, 23 edge crossings measured from the wrong end, 24 the
 one-hot-vertex fraction missing a factor; spectra: 25 delta f with (1 + sigma f)
 instead of (1 - sigma f), 26 p^eta dSigma_eta without the 1/tau of the tilde
 component, 27 the sign of p^x u^x in p.u; bulk and baryon: 28 the sign of
 zeta theta in S_Pi, 29 S_Pi without its Pi u~^tau/tau term, 30 Pi left out of
 T's density and flux, 31 the root solve without Pi, 32 S_n dropped; shear
 regulator: 33 a third regulation after the root solve with e^{n+1} (the
 stored pi~ then no longer matches T~ and (e, u~)), 34 the corrector regulated
 with e^n instead of e', 35 the sign of the tau-i terms of pi~:pi~, 36 the sign
 of the i-j off-diagonal terms, 37 |pi~:pi~| without the absolute value, 38 the
 shear factor applied to Pi and n too.
Mutant 16 (u* = u^n instead of 2u^n - u^{n-1}) alters only the predicted pi'
at O(h) and the step at O(h^2), the scheme's own order, so no pin is expected
to separate it; the GPU-oracle parity tests cover that code path.
"""
import warnings

import numpy as np
import pytest

import oracle as O

from . import pins

CAUGHT = list(range(1, 16)) + list(range(17, 39))


@pytest.mark.parametrize("k", CAUGHT)
def test_planted_mistake_is_caught(k):
    failed = []
    O.set_mutant(k)
    try:
        with warnings.catch_warnings(), np.errstate(all="ignore"):
            warnings.simplefilter("ignore")
            for name, fn in pins.ALL_PINS.items():
                try:
                    ok, _ = fn()
                except Exception:
                    ok = False
                if not ok:
                    failed.append(name)
                    break
    finally:
        O.set_mutant(0)
    assert failed, f"planted mistake {k} passed every pin"
