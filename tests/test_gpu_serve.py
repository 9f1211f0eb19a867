"""GPU tests of the serving engine (continuous batching, admission by HBM
footprint)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import paper_2006_15512_amd as W
import wmc_workloads as wl

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def frac(v):
    return Fraction(0) if v.mantissa == 0.0 else Fraction(v.mantissa) * Fraction(2) ** v.exp2


def rel(a, b):
    return 0.0 if a == b else float(abs(a - b) / max(abs(a), abs(b)))


STRUCTS = [0, 1, 2, 3, 4, 5]  # the rank <= 19 serving structures (6, 7 reach rank 23-24)


@pytest.fixture(scope="module")
def structures():
    return [wl.serve_structure(s) for s in STRUCTS]


def make_server(structures, precision="fp64", **kw):
    srv = W.Server(precision=precision, **kw)
    plans = [W.Plan(W.Network.from_formula(f), seed=0, precision=precision) for f in structures]
    ids = [srv.register(p) for p in plans]
    return srv, plans, ids


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_serve_results_vs_oracle(structures, precision, tol):
    """Requests over 6 structures with their own weight vectors, all queued at
    once, against the oracle."""
    srv, plans, ids = make_server(structures, precision, max_slots=16, buffer_bytes=1 << 29)
    rng = np.random.default_rng(1)
    reqs = []
    for q in range(24):
        s = int(rng.integers(0, len(structures)))
        w = rng.uniform(0.1, 0.9, size=structures[s].n)
        Wt = np.stack([1 - w, w], axis=1)
        reqs.append((s, Wt))
        srv.submit(ids[s], Wt, q)
    say(f"serve {precision}: submitted")
    got = {r.request_id: r for r in srv.drain()}
    assert len(got) == len(reqs)
    for q, (s, Wt) in enumerate(reqs):
        m, e = oracle.bucket(structures[s].with_weights(Wt))
        ref = Fraction(m) * Fraction(2) ** e
        assert got[q].status == 0
        assert rel(frac(got[q].value), ref) <= tol, q


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_serve_alone_equals_in_mix(structures, precision, tol):
    """Each result in a mix equals the same request served alone, bit for bit
    (both precisions: a request's arithmetic is its plan's, whatever shares
    its launches), and wmc_contract on the same plan: bit for bit in FP64;
    in scaled FP32 within the FP32 tolerance (the solo executor may run a
    node on another kernel family, which rounds at other points)."""
    srv, plans, ids = make_server(structures, precision, max_slots=32, buffer_bytes=1 << 29)
    rng = np.random.default_rng(2)
    reqs = []
    for q in range(40):
        s = int(rng.integers(0, len(structures)))
        w = rng.uniform(0.1, 0.9, size=structures[s].n)
        reqs.append((s, np.stack([1 - w, w], axis=1)))
    # staggered submission: requests join while others are mid-flight
    mix = {}
    it = iter(enumerate(reqs))
    pending = True
    while pending or srv.stats()["n_active"]:
        for _ in range(3):
            nxt = next(it, None)
            if nxt is None:
                pending = False
                break
            q, (s, Wt) = nxt
            srv.submit(ids[s], Wt, q)
        srv.step()
        for r in srv.poll():
            mix[r.request_id] = r.value
    assert len(mix) == len(reqs)
    assert srv.stats()["peak_active"] > 4
    say(f"mix done ({precision})")
    for q, (s, Wt) in enumerate(reqs):
        alone = W.Server(precision=precision, max_slots=1, buffer_bytes=1 << 27)
        sid = alone.register(plans[s])
        alone.submit(sid, Wt, 0)
        (r,) = alone.drain()
        assert (r.value.mantissa, r.value.exp2) == (mix[q].mantissa, mix[q].exp2), q
        solo = W.wmc_contract(plans[s], Wt)
        if precision == "fp64":
            assert (solo.mantissa, solo.exp2) == (mix[q].mantissa, mix[q].exp2), q
        else:
            assert rel(frac(solo), frac(mix[q])) <= tol, q


def test_serve_admission_respects_budget(structures):
    """A budget that fits only a few footprints: requests wait in the queue,
    the peak of used region bytes stays within the budget, all complete."""
    plans = [W.Plan(W.Network.from_formula(f), seed=0) for f in structures]
    fp = max(p.stats()["arena_bytes"] for p in plans)
    budget = int(3.5 * fp) + (1 << 20)
    srv = W.Server(precision="fp64", max_slots=64, hbm_budget_bytes=budget, buffer_bytes=1 << 29)
    ids = [srv.register(p) for p in plans]
    rng = np.random.default_rng(3)
    for q in range(30):
        s = int(rng.integers(0, len(structures)))
        w = rng.uniform(0.1, 0.9, size=structures[s].n)
        srv.submit(ids[s], np.stack([1 - w, w], axis=1), q)
    out = srv.drain()
    st = srv.stats()
    assert len(out) == 30
    assert st["peak_used_bytes"] <= st["region_bytes"] <= budget + 256
    assert st["peak_active"] < 30


def test_serve_queue_full_is_busy(structures):
    srv, plans, ids = make_server(structures[:1], max_slots=2, max_queue=3, buffer_bytes=1 << 27)
    w = np.full((structures[0].n, 2), 0.5)
    for q in range(3):
        srv.submit(ids[0], w, q)
    with pytest.raises(W.WmcError) as e:
        srv.submit(ids[0], w, 99)
    assert e.value.status == 5
    assert len(srv.drain()) == 3


def test_serve_trace_replay(structures):
    """Timed Poisson arrivals replayed by the native loop: every request
    completes once, after it arrived, with its oracle value."""
    srv, plans, ids = make_server(structures, max_slots=32, buffer_bytes=1 << 29)
    n = 60
    arr, st_, w = wl.serve_queries(n, rate=2000.0, seed=5, n_structures=len(structures))
    out = srv.run(arr, [ids[s] for s in st_], list(w))
    assert sorted(r.request_id for r in out) == list(range(n))
    for r in out:
        assert r.t_done >= r.t_admit >= r.t_arrive - 1e-9
    for r in out[:12]:
        f = structures[int(st_[r.request_id])].with_weights(w[r.request_id])
        m, e = oracle.bucket(f)
        assert rel(frac(r.value), Fraction(m) * Fraction(2) ** e) <= 1e-12


def test_serve_long_clause_structures():
    """Structures with factored long clauses: each request's 2n weights are
    expanded with the auxiliary variables' (1, 1)."""
    fs = [wl.random_long(s) for s in range(4)]
    srv = W.Server(precision="fp64", max_slots=8, buffer_bytes=1 << 27)
    ids = [srv.register(W.Plan(W.Network.from_formula(f), seed=0)) for f in fs]
    rng = np.random.default_rng(4)
    reqs = []
    for q in range(16):
        s = q % len(fs)
        w = rng.uniform(0.1, 0.9, size=fs[s].n)
        Wt = np.stack([1 - w, w], axis=1)
        reqs.append((s, Wt))
        srv.submit(ids[s], Wt, q)
    got = {r.request_id: r for r in srv.drain()}
    for q, (s, Wt) in enumerate(reqs):
        ref = Fraction(oracle.brute(fs[s].with_weights(Wt)))
        assert rel(frac(got[q].value), ref) <= 1e-12, q


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_serve_big_structures_vs_oracle(precision, tol):
    """Serving structures 6 and 7 (storage rank 23-24) mixed with small ones,
    against the oracle, and each equal to wmc_contract (bit for bit in FP64,
    within the tolerance in scaled FP32)."""
    fs = [wl.serve_structure(s) for s in (6, 7, 0)]
    plans = [W.Plan(W.Network.from_formula(f), seed=0, precision=precision) for f in fs]
    srv = W.Server(precision=precision, max_slots=8, buffer_bytes=1 << 31)
    ids = [srv.register(p) for p in plans]
    rng = np.random.default_rng(9)
    reqs = []
    for q in range(6):
        s = q % 3
        w = rng.uniform(0.1, 0.9, size=fs[s].n)
        Wt = np.stack([1 - w, w], axis=1)
        reqs.append((s, Wt))
        srv.submit(ids[s], Wt, q)
    got = {r.request_id: r for r in srv.drain()}
    for q, (s, Wt) in enumerate(reqs):
        solo = W.wmc_contract(plans[s], Wt)
        if precision == "fp64":
            assert (solo.mantissa, solo.exp2) == (got[q].value.mantissa, got[q].value.exp2), q
        else:
            assert rel(frac(solo), frac(got[q].value)) <= tol, q
        m, e = oracle.bucket(fs[s].with_weights(Wt))
        assert rel(frac(got[q].value), Fraction(m) * Fraction(2) ** e) <= tol, q


def test_serve_cancel_queued_and_running(structures):
    """A cancelled request ends with CANCELLED (at once when queued, after
    the step in flight when running), its slot and region come back, and
    every other request still matches the oracle."""
    srv, plans, ids = make_server(structures, max_slots=4, buffer_bytes=1 << 28)
    rng = np.random.default_rng(21)
    reqs = []
    for q in range(10):
        s = int(rng.integers(0, len(structures)))
        w = rng.uniform(0.1, 0.9, size=structures[s].n)
        Wt = np.stack([1 - w, w], axis=1)
        reqs.append((s, Wt))
        srv.submit(ids[s], Wt, q)
    srv.cancel(9)                # still queued (4 slots)
    srv.step()
    srv.step()
    srv.cancel(0)                # running
    with pytest.raises(W.WmcError):
        srv.cancel(12345)        # unknown
    got = {r.request_id: r for r in srv.drain()}
    assert sorted(got) == list(range(10))
    assert got[9].status == W.CANCELLED and got[0].status == W.CANCELLED
    for q in range(1, 9):
        s, Wt = reqs[q]
        m, e = oracle.bucket(structures[s].with_weights(Wt))
        assert got[q].status == 0 and rel(frac(got[q].value), Fraction(m) * Fraction(2) ** e) <= 1e-12, q
    st = srv.stats()
    assert st["n_active"] == 0 and st["used_bytes"] == 0


def test_serve_deadlines_and_wait(structures):
    """Requests past their deadline end with CANCELLED; ones with room to
    spare complete; wait() steps the server until a response is ready."""
    srv, plans, ids = make_server(structures, max_slots=2, buffer_bytes=1 << 28)
    rng = np.random.default_rng(22)
    w = [np.stack([1 - x, x], axis=1) for x in (rng.uniform(0.1, 0.9, size=f.n) for f in structures)]
    srv.submit_deadline(ids[0], w[0], 0, 60.0)
    srv.submit_deadline(ids[1], w[1], 1, 60.0)
    for q in range(2, 8):        # queued behind two slots, deadlines that pass at once
        srv.submit_deadline(ids[q % len(ids)], w[q % len(ids)], q, 1e-9)
    out = []
    while len(out) < 8:
        got = srv.wait(10.0)
        assert got, "wait returned nothing"
        out += got
    by = {r.request_id: r for r in out}
    assert by[0].status == 0 and by[1].status == 0
    assert all(by[q].status == W.CANCELLED for q in range(2, 8))
    m, e = oracle.bucket(structures[0].with_weights(w[0]))
    assert rel(frac(by[0].value), Fraction(m) * Fraction(2) ** e) <= 1e-12


def _sliced_structure(precision):
    """A banded formula whose plan (rank 12) is sliced to rank 11: 8 slices."""
    f = wl.banded_3cnf(80, 280, 16, seed=2)
    p = W.Plan(W.Network.from_formula(f), seed=0, rank_cap=11, precision=precision)
    assert p.stats()["n_slices"] >= 4
    return f, p


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_serve_sliced_structure_in_a_mix(structures, precision, tol):
    """Requests on a sliced structure run as one part per slice among
    requests on unsliced ones: each answers once, equal to wmc_contract on
    the same plan (bit for bit in FP64) and to the oracle, and the same
    served alone."""
    f, sp = _sliced_structure(precision)
    srv, plans, ids = make_server(structures, precision, max_slots=12, buffer_bytes=1 << 29)
    sid = srv.register(sp)
    rng = np.random.default_rng(31)
    reqs = []
    for q in range(16):
        if q % 3 == 0:
            w = rng.uniform(0.1, 0.9, size=f.n)
            reqs.append((None, np.stack([1 - w, w], axis=1)))
            srv.submit(sid, reqs[-1][1], q)
        else:
            s = int(rng.integers(0, len(structures)))
            w = rng.uniform(0.1, 0.9, size=structures[s].n)
            reqs.append((s, np.stack([1 - w, w], axis=1)))
            srv.submit(ids[s], reqs[-1][1], q)
    say(f"sliced serve {precision}: submitted")
    out = srv.drain()
    assert sorted(r.request_id for r in out) == list(range(16))  # one answer per request
    got = {r.request_id: r for r in out}
    for q, (s, Wt) in enumerate(reqs):
        assert got[q].status == 0, q
        form = f if s is None else structures[s]
        m, e = oracle.bucket(form.with_weights(Wt))
        assert rel(frac(got[q].value), Fraction(m) * Fraction(2) ** e) <= tol, q
        if s is None:
            solo = W.wmc_contract(sp, Wt)
            if precision == "fp64":
                assert (solo.mantissa, solo.exp2) == (got[q].value.mantissa, got[q].value.exp2), q
            else:
                assert rel(frac(solo), frac(got[q].value)) <= tol, q
            alone = W.Server(precision=precision, max_slots=2, buffer_bytes=1 << 27)
            aid = alone.register(sp)
            alone.submit(aid, Wt, 0)
            (r,) = alone.drain()
            assert (r.value.mantissa, r.value.exp2) == (got[q].value.mantissa, got[q].value.exp2), q
    st = srv.stats()
    assert st["n_active"] == 0 and st["used_bytes"] == 0


def test_serve_sliced_cancel_and_deadline(structures):
    """Cancelling a sliced request while some parts run and others wait, or
    letting its deadline pass, gives exactly one CANCELLED answer; regions
    and slots come back and the other requests are untouched."""
    f, sp = _sliced_structure("fp64")
    srv, plans, ids = make_server(structures, max_slots=3, buffer_bytes=1 << 28)
    sid = srv.register(sp)
    rng = np.random.default_rng(32)
    w = rng.uniform(0.1, 0.9, size=f.n)
    Wt = np.stack([1 - w, w], axis=1)
    srv.submit(sid, Wt, 0)                       # parts beyond 3 slots wait
    srv.submit_deadline(sid, Wt, 1, 1e-9)        # passes at once
    srv.submit(sid, Wt, 2)
    x = rng.uniform(0.1, 0.9, size=structures[0].n)
    W3 = np.stack([1 - x, x], axis=1)
    srv.submit(ids[0], W3, 3)
    srv.step()
    srv.step()
    srv.cancel(0)                                # some parts running, some queued
    out = srv.drain()
    assert sorted(r.request_id for r in out) == [0, 1, 2, 3]
    got = {r.request_id: r for r in out}
    assert got[0].status == W.CANCELLED and got[1].status == W.CANCELLED
    m, e = oracle.bucket(f.with_weights(Wt))
    assert got[2].status == 0 and rel(frac(got[2].value), Fraction(m) * Fraction(2) ** e) <= 1e-12
    m, e = oracle.bucket(structures[0].with_weights(W3))
    assert got[3].status == 0 and rel(frac(got[3].value), Fraction(m) * Fraction(2) ** e) <= 1e-12
    st = srv.stats()
    assert st["n_active"] == 0 and st["n_queued"] == 0 and st["used_bytes"] == 0
