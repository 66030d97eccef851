"""FP64 CPU oracle of the 2D HA-NsDLCT (CM-CC-CM-CC / CC-CM-CC-CM).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test suite, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` use it.  It shares
no code, constants or tables with the HIP library; the only common module is
``synth`` (seeded input generators, which hold none of the method's
arithmetic).

Everything is plain numpy in complex128 / float64, written step by step in the
order and notation of Pei & Huang, "Two-dimensional nonseparable discrete
linear canonical transform based on CM-CC-CM-CC decomposition":

* ``symplectic`` -- the ABCD constraints (Sec. 1, eqs. Intro12/Intro16),
  inverse (Sec. 4.3, eq. CCCMCCCM20).
* ``ops``        -- the basic discrete operations of Sec. 2: CM (eq.
  BasicCM12), DFT / IDFT (eqs. BasicDFT16/20) as dense matrices, CC
  (eq. BasicCC20).
* ``gauge``      -- the CM-CC-CM-CC and CC-CM-CC-CM decompositions (Secs.
  4.2, 4.3), the ratio function gamma (eq. HA16), the HA gauge problem
  (eq. HA24) solved by brute force, the trace rule (eq. Reversible08).
* ``chain``      -- the HA-NsDLCT chains (eqs. HA28, CCCMCCCM40), the inverse
  (eq. CCCMCCCM30), chains at injected stage matrices.
* ``dense``      -- the N^2 x N^2 operator of Sec. 6.2 (eq. self12) built
  from literal Kronecker DFT matrices.
* ``direct``     -- the direct method (eq. Intro32) and the closed-form
  continuous NsLCT (eq. Intro08) of a Gaussian.
* ``sampling``   -- the phase-space growth predicate (eqs. HA12-HA20).
* ``fast``       -- the reduced decompositions: CM-CC-CM for symmetric B
  (Sec. 4.1, eq. Bsym12) and the LC-NsDLCT with a rank-one gauge (Sec.
  4.2.2, eqs. LC04-LC12).
* ``route``      -- the decomposition (-B, A; -D, C)(0, -I; I, 0) of Sec.
  4.2.2 for a12 = a21 = 0 (IDFT, then CM-CC-CM), its overall constant from
  the closed-form propagation of a Gaussian through the factors.

Pins (checked by ``tests/test_oracle_*.py``) tie every function to something
other than itself; see the test docstrings.
"""
from . import symplectic, ops, gauge, chain, dense, direct, sampling, fast, route  # noqa: F401
from . import plan  # noqa: F401
from .plan import Plan, plan_from_stages  # noqa: F401
