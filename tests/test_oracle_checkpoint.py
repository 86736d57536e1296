"""Checkpoint and resume on the oracle: a scene's state after n steps is its
bodies' (c, A, v, w) (Algorithm 1 carries nothing else from step to step for
scenes without augmented, driven or slider bonds), so re-creating the scene
from that state and stepping m more times reproduces n + m uninterrupted steps
exactly."""
import numpy as np

import oracle
from paper_2609_02675_amd import scenes as S


def _resume_equals_uninterrupted(sc, n, m):
    full = oracle.Oracle(sc)
    full.step(n + m)
    first = oracle.Oracle(sc)
    first.step(n)
    c, A, v, w = first.state()
    rest = oracle.Oracle(sc.with_state(c, A, v, w, t0=sc.t0 + n * sc.h))
    rest.step(m)
    for x, y in zip(rest.state(), full.state()):
        assert np.array_equal(x, y)


def test_chain_resumes_exactly():
    _resume_equals_uninterrupted(S.chain(12, tilt_deg=30.0, precision=S.PREC_FP64), 9, 7)


def test_contact_pile_resumes_exactly():
    _resume_equals_uninterrupted(S.box_drop(n_side=3, layers=2, seed=3, precision=S.PREC_FP64), 45, 15)
