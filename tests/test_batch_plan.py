"""The batched call's planner (kp_batch_plan: host logic, no device call).

A plan must be valid (every problem on exactly one team, teams disjoint and
inside the grid), deterministic, and balanced: its predicted makespan lies
between the trivial lower bound (all work spread evenly over the grid, no
problem faster than on its best team) and a small multiple of it.
"""
import pytest

import workloads as W
import paper_2410_14917_amd as kp


def _plan(probs, m_max=48, n_wg=256):
    return kp.batch_plan([q.op for q in probs], [q.p for q in probs], [q.h for q in probs],
                         m_max=m_max, n_wg=n_wg)


def _check_valid(top, teams, n_wg, nprob):
    assert len(top) == nprob
    used = set()
    for w0, g in teams:
        assert g >= 1 and g & (g - 1) == 0           # power-of-two team sizes
        span = set(range(w0, w0 + g))
        assert not (span & used) and max(span) < n_wg
        used |= span
    assert all(0 <= t < len(teams) for t in top)


def test_uneven_batch_plan_is_valid_and_balanced():
    probs = W.config4()
    top, teams, makespan, work = _plan(probs)
    _check_valid(top, teams, 256, len(probs))
    assert makespan >= work / 256 * (1 - 1e-12)
    assert makespan <= 1.25 * work / 256
    # teams of more than one workgroup exist (the heavy problems need them)
    # and the heaviest problem sits on one of the largest teams
    sizes = [g for _, g in teams]
    assert max(sizes) > 1
    heavy = max(range(len(probs)), key=lambda i: probs[i].op.n * probs[i].op.nu)
    assert teams[top[heavy]][1] == max(sizes)


def test_plan_is_deterministic():
    probs = W.config4(nprob=96)
    assert _plan(probs) == _plan(probs)


def test_small_problems_get_single_workgroups():
    probs = [W.Problem(op=W.adr(32, 32, nu=1e-3), B=None, h=0.05, p=3, m_max=48, tol=1e-8,
                       seed=0, name="t") for _ in range(600)]
    top, teams, makespan, work = _plan(probs)
    _check_valid(top, teams, 256, 600)
    assert {g for _, g in teams} == {1}
    assert makespan <= 1.5 * work / 256


def test_one_heavy_problem_gets_a_large_team():
    probs = [W.Problem(op=W.adr(512, 512, nu=0.1), B=None, h=0.05, p=3, m_max=48, tol=1e-8,
                       seed=0, name="big")]
    probs += [W.Problem(op=W.adr(64, 64, nu=1e-3), B=None, h=0.05, p=3, m_max=48, tol=1e-8,
                        seed=0, name="small") for _ in range(40)]
    top, teams, makespan, work = _plan(probs)
    _check_valid(top, teams, 256, len(probs))
    assert teams[top[0]][1] >= 16
    assert all(teams[top[i]][1] < teams[top[0]][1] for i in range(1, len(probs)))


def test_plan_rejects_bad_input():
    op = W.adr(16, 16)
    with pytest.raises(RuntimeError, match=r"\[-1\]"):
        kp.batch_plan([op], [kp._lib.KP_PMAX + 1], [0.1])
    with pytest.raises(RuntimeError, match=r"\[-1\]"):
        kp.batch_plan([op], [2], [0.1], m_max=0)
    with pytest.raises(RuntimeError, match=r"\[-1\]"):
        kp.batch_plan([op], [2], [float("nan")])
