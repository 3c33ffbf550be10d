"""Binary64 CPU oracle for the BPFA Gibbs sweep: TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct statement of what the GPU path computes,
written from the paper's BPFA section and the BPFA model of the works it cites.
It shares no code with the HIP library and neither imports the other; only the
seeded input generators (package ``synth``) feed both.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run anything in this package.  The product path
never does, and fails loudly when its HIP library is missing.

Pinned by the ``-m "not gpu"`` tests (see tests/test_oracle_*.py) against
independent facts: Philox known-answer vectors, scipy distributions,
quadrature, dense Gaussian algebra, brute-force enumeration of all 2^K
configurations, Geweke's joint-distribution test and closed-form coverage.
"""
from . import acquire, bpfa, gamma, patches, philox  # noqa: F401
