"""Pins for the literal step-synchronous variant of CLUSTER (Algorithm 1 with
PartialGrowth taken literally: synchronous Delta-growing steps, the strict
distance tie rule, the per-step half-coverage stop, Delta doubled one step at
a time, an optional cap on the steps of a PartialGrowth call).

The C oracle (implicit Contract, frontier of updated nodes) must equal the
brute force that builds every contracted graph with Procedure Contract and in
every step lets every node with d_u < Delta offer over all its light edges:
same clusters, distance bounds, stages, Delta, PartialGrowth calls, steps
(rounds), node updates and messages.  The brute force counts messages on its
own, over the original graph's arcs, from the explicit state of each step."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import brute

from test_oracle_pins import FAMILIES, _edges


def _same(dec, ref, name):
    assert dec.cluster.tolist() == [int(c) for c in ref["cluster"]], name
    assert dec.D.tolist() == [int(d) for d in ref["D"]], name
    assert (dec.stages, dec.delta_end, dec.num_clusters, dec.radius, dec.levels) == \
        (ref["stages"], ref["delta_end"], ref["num_clusters"], int(ref["radius"]), ref["levels"]), name
    assert dec.work["rounds"] == ref["rounds"], name
    assert dec.work["updates"] == ref["updates"], name
    assert dec.work["messages"] == ref["messages"], name


@pytest.mark.parametrize("name,g", FAMILIES, ids=[f for f, _ in FAMILIES])
@pytest.mark.parametrize("tau,seed", [(1, 1), (2, 5)])
def test_steps_equal_explicit_contract(name, g, tau, seed):
    dec = oracle.decompose_steps(g, tau, seed)
    ref = brute.cluster_steps(g.n, _edges(g), tau, seed)
    _same(dec, ref, name)


@pytest.mark.parametrize("name,g", FAMILIES[::4], ids=[f for f, _ in FAMILIES[::4]])
@pytest.mark.parametrize("cap", [1, 2, 5])
def test_step_cap_equals_explicit_contract(name, g, cap):
    dec = oracle.decompose_steps(g, 1, 7, step_cap=cap)
    ref = brute.cluster_steps(g.n, _edges(g), 1, 7, step_cap=cap)
    _same(dec, ref, name)


@pytest.mark.parametrize("delta0", [1, 3, 10**6])
def test_steps_explicit_initial_delta(delta0):
    for name, g in FAMILIES[:6]:
        dec = oracle.decompose_steps(g, 1, 13, delta0=delta0)
        ref = brute.cluster_steps(g.n, _edges(g), 1, 13, delta0=delta0)
        _same(dec, ref, name)


def test_steps_exercise_the_stop_rules():
    """The families must make the per-step half stop cut growth short (so the
    literal variant really differs from growth to the fixpoint), double Delta
    and run several stages."""
    differs = 0
    for name, g in FAMILIES:
        a = oracle.decompose_steps(g, 1, 1)
        b = oracle.decompose(g, 1, 1)
        differs += not np.array_equal(a.cluster, b.cluster)
        assert a.work["rounds"] >= a.levels
    assert differs >= 3
    assert max(oracle.decompose_steps(g, 1, 1).stages for _, g in FAMILIES) >= 2


@pytest.mark.parametrize("name,g", FAMILIES[::2], ids=[f for f, _ in FAMILIES[::2]])
def test_message_invariants(name, g):
    """Every update comes from one accepted message; a step's messages are at
    most the arcs of its active rows, so at most rounds x m; the row reads
    counted are the active-set sizes."""
    dec = oracle.decompose_steps(g, 1, 21)
    wk = dec.work
    assert wk["updates"] <= wk["messages"] <= wk["rounds"] * max(g.m, 1)
    assert wk["sum_arcs"] == wk["messages"]
    deg_max = int(np.diff(g.row_ptr).max()) if g.n else 0
    assert wk["messages"] <= wk["sum_acting"] * deg_max


def test_no_step_without_stages():
    """ceil(8 tau log2 n) > n: no stage, no step, every node a singleton."""
    g = graphgen.grid(5, 5, 10, 1)
    dec = oracle.decompose_steps(g, 1, 1)
    assert dec.stages == 0 and dec.work["rounds"] == 0 and dec.work["messages"] == 0
    assert dec.cluster.tolist() == list(range(g.n))


def test_path_closed_form():
    """Unit-weight path with Delta0 above its total weight: no doubling ever
    happens (one PartialGrowth call per stage), and every step except the
    last one of a call updates at least one node."""
    n = 200
    g = graphgen.csr_from_edges_np(n, range(n - 1), range(1, n), [1] * (n - 1))
    dec = oracle.decompose_steps(g, 1, 4, delta0=10**6)
    assert dec.levels == dec.stages          # Delta0 covers everything: no doubling
    assert dec.delta_end == 10**6
    assert dec.work["updates"] >= dec.work["rounds"] - dec.stages
