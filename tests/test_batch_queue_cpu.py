"""Host-side checks of the persistent batched step's work queue (no GPU):
the queue covers every tile of every phase exactly once, lists every item
after the items it waits for, and a model of the kernel's control logic --
workgroups taking tickets in order, the step index and the exit from the
ticket arithmetic, waits on monotonic per-problem counters with targets
t * tiles -- completes several steps for any number of workgroups."""
import heapq
import math

import numpy as np
import pytest

import synth

IT_PF_MOVE, IT_GMM_REWEIGHT, IT_FINAL, IT_RESAMPLE, IT_GMM_STEP, IT_MONITOR = range(6)


@pytest.fixture(scope="module")
def L():
    from paper_1306_5583_amd import _lib
    _lib.load()
    return _lib


def _problems(L, shapes):
    """smc_batch_problem structs from (kind, n, K, n_data) shapes; only the
    configurations matter to the queue."""
    out = []
    for i, (kind, n, K, nd) in enumerate(shapes):
        bp = L.smc_batch_problem()
        if kind == "pf":
            bp.cfg = L.make_config(L.SMC_MODEL_CV_TRACK, n, seed=i + 1, problem_id=i, n_obs=8)
        else:
            bp.cfg = L.make_config(L.SMC_MODEL_GMM_TEMPERED, n, seed=i + 1, problem_id=i, K=K,
                                   n_data=nd, move_kind=L.SMC_MOVE_MALA)
        out.append(bp)
    return out


def _shapes_small():
    return [("pf", 1000, 0, 0), ("gmm", 2048, 3, 90), ("pf", 5120, 0, 0), ("gmm", 1500, 1, 60),
            ("gmm", 3333, 5, 130), ("pf", 3001, 0, 0), ("gmm", 700, 2, 45)]


def _shapes_batched_benchmark():
    # the 128-filter / 32-sampler workload's shapes
    return [(q.kind, q.n_particles, q.K, q.n_data) for q in synth.batched_problems()]


def _deps(items, shapes):
    """Per item: (counter kind, problem, target per step) it waits for, or None."""
    tiles = [math.ceil(n / 1024) for _, n, _, _ in shapes]
    out = []
    for kind, p, _, cnt in items:
        if kind == IT_FINAL:
            out.append(("a", p, tiles[p]))
        elif kind == IT_RESAMPLE:
            out.append(("f", p, 1))
        elif kind == IT_GMM_STEP:
            out.append(("r", p, tiles[p]))
        elif kind == IT_MONITOR:
            out.append(("m", p, cnt))
        else:
            out.append(None)
    return out


def _releases(items, shapes):
    """Per item: (counter kind, problem, amount) it adds when done, or None
    (a Metropolis item adds its 64-particle tiles)."""
    out = []
    for kind, p, _, cnt in items:
        if kind in (IT_PF_MOVE, IT_GMM_REWEIGHT):
            out.append(("a", p, 1))
        elif kind == IT_FINAL:
            out.append(("f", p, 1))
        elif kind == IT_RESAMPLE and shapes[p][0] == "gmm":
            out.append(("r", p, 1))
        elif kind == IT_GMM_STEP:
            out.append(("m", p, cnt))
        else:
            out.append(None)
    return out


def _full(shapes):
    """Units of each counter one step of a problem completes."""
    out = {}
    for p, (kind, n, _, _) in enumerate(shapes):
        out[("a", p)] = out[("r", p)] = math.ceil(n / 1024)
        out[("f", p)] = 1
        out[("m", p)] = math.ceil(n / 64)
    return out


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("per_item", [1, 2])
@pytest.mark.parametrize("which", ["small", "benchmark"])
def test_queue_covers_every_tile_once_in_dependency_order(L, order, per_item, which):
    shapes = _shapes_small() if which == "small" else _shapes_batched_benchmark()
    items = L.smc_batch_plan_queue(_problems(L, shapes), order, per_item)
    seen = {}
    for kind, p, tile, cnt in items:
        seen.setdefault((kind, p), []).append((tile, cnt))
    for p, (kind, n, K, nd) in enumerate(shapes):
        nt = math.ceil(n / 1024)
        a = IT_PF_MOVE if kind == "pf" else IT_GMM_REWEIGHT
        assert sorted(t for t, _ in seen[(a, p)]) == list(range(nt))
        assert seen[(IT_FINAL, p)] == [(0, 1)]
        assert sorted(t for t, _ in seen[(IT_RESAMPLE, p)]) == list(range(nt))
        if kind == "gmm":
            covered = sorted(t + q for t, c in seen[(IT_GMM_STEP, p)] for q in range(c))
            assert covered == list(range(math.ceil(n / 64)))
            assert all(1 <= c <= per_item for _, c in seen[(IT_GMM_STEP, p)])
            # the monitor waits for the step's 64-particle tiles, whatever the item size
            assert seen[(IT_MONITOR, p)] == [(0, math.ceil(n / 64))]
        else:
            assert (IT_GMM_STEP, p) not in seen and (IT_MONITOR, p) not in seen
    # every item after everything it waits for
    pos = {}
    for k, (kind, p, tile, cnt) in enumerate(items):
        pos.setdefault((kind, p), []).append(k)
    for k, (kind, p, tile, cnt) in enumerate(items):
        if kind == IT_FINAL:
            a = IT_PF_MOVE if shapes[p][0] == "pf" else IT_GMM_REWEIGHT
            assert max(pos[(a, p)]) < k
        elif kind == IT_RESAMPLE:
            assert pos[(IT_FINAL, p)][0] < k
        elif kind == IT_GMM_STEP:
            assert max(pos[(IT_RESAMPLE, p)]) < k
        elif kind == IT_MONITOR:
            assert max(pos[(IT_GMM_STEP, p)]) < k


def _simulate(items, shapes, G, steps, seed, first_step=1, ctr=None, ticket=0):
    """Event-driven model of the step kernel: G workgroups, each taking the
    next ticket when free; ticket -> (step, item) as in the kernel; an item
    waits until its counter reaches step * target; random durations.  Each
    item that starts is also checked against what has really finished: every
    unit of the step it depends on (so a counter target that does not match
    the releases fails here).  Returns the counters and the next ticket."""
    rng = np.random.default_rng(seed)
    deps, rel = _deps(items, shapes), _releases(items, shapes)
    full = _full(shapes)
    per_step = len(items) + G
    ctr = dict(ctr or {})
    for step in range(first_step, first_step + steps):
        # one launch: every workgroup loops until it draws a ticket past the items
        done = {}                                     # units finished in this step
        clock = 0.0
        ready = [(0.0, w) for w in range(G)]          # (time free, workgroup)
        heapq.heapify(ready)
        waiting = []                                  # (workgroup, item index)
        running = []                                  # (finish time, workgroup, item)
        exited = 0
        while exited < G:
            progressed = False
            # start free workgroups on new tickets
            while ready:
                tfree, w = heapq.heappop(ready)
                tk = ticket
                ticket += 1
                k, t = tk % per_step, tk // per_step + 1
                assert t == step, "a ticket of another step was drawn"
                progressed = True
                if k >= len(items):
                    exited += 1
                    continue
                waiting.append((w, k))
            # items whose dependency is met start running
            still = []
            for w, k in waiting:
                d = deps[k]
                if d is None or ctr.get((d[0], d[1]), 0) >= step * d[2]:
                    if d is not None:
                        assert done.get((d[0], d[1]), 0) == full[(d[0], d[1])], \
                            ("started before its dependency finished", step, items[k])
                    running.append((clock + rng.exponential(1.0), w, k))
                    progressed = True
                else:
                    still.append((w, k))
            waiting = still
            if running:
                running.sort()
                fin, w, k = running.pop(0)
                clock = max(clock, fin)
                if rel[k] is not None:
                    c, p, amount = rel[k]
                    ctr[(c, p)] = ctr.get((c, p), 0) + amount
                    done[(c, p)] = done.get((c, p), 0) + amount
                heapq.heappush(ready, (clock, w))
                progressed = True
            assert progressed, "deadlock: every workgroup waits"
        assert not waiting and not running
        assert ticket % per_step == 0
    return ctr, ticket


@pytest.mark.parametrize("G", [1, 2, 7, 64, 600])
@pytest.mark.parametrize("order", [0, 1])
def test_step_model_completes_for_any_grid(L, G, order):
    shapes = _shapes_small()
    items = L.smc_batch_plan_queue(_problems(L, shapes), order, 2)
    steps = 3
    ctr, _ = _simulate([tuple(r) for r in items], shapes, G, steps, seed=G)
    for p, (kind, n, K, nd) in enumerate(shapes):
        nt = math.ceil(n / 1024)
        assert ctr[("a", p)] == steps * nt and ctr[("f", p)] == steps
        if kind == "gmm":
            assert ctr[("r", p)] == steps * nt
            assert ctr[("m", p)] == steps * math.ceil(n / 64)


def test_schedule_change_between_steps(L):
    # two steps on one schedule, then another queue order, item size and
    # grid: the ticket counter is rebased to steps * new tickets per step
    # (as the library does) and every wait still follows its dependency
    shapes = _shapes_small()
    probs = _problems(L, shapes)
    qa = [tuple(int(x) for x in r) for r in L.smc_batch_plan_queue(probs, 0, 1)]
    qb = [tuple(int(x) for x in r) for r in L.smc_batch_plan_queue(probs, 1, 2)]
    ga, gb = 7, 3
    ctr, ticket = _simulate(qa, shapes, ga, 2, seed=5)
    ticket = ticket // (len(qa) + ga) * (len(qb) + gb)
    ctr, ticket = _simulate(qb, shapes, gb, 2, seed=6, first_step=3, ctr=ctr, ticket=ticket)
    for p, (kind, n, K, nd) in enumerate(shapes):
        if kind == "gmm":
            assert ctr[("m", p)] == 4 * math.ceil(n / 64)


def test_unsupported_shapes_are_refused(L):
    shapes = _shapes_small()
    probs = _problems(L, shapes)
    probs[1].cfg.K = 9                       # beyond the step kernel's mixtures
    with pytest.raises(L.SmcError) as e:
        L.smc_batch_plan_queue(probs, 0, 1)
    assert e.value.status == L.SMC_ERR_UNSUPPORTED
    probs = _problems(L, shapes)
    probs[0].cfg.scheme = L.SCHEMES["multinomial"]
    with pytest.raises(L.SmcError) as e:
        L.smc_batch_table_size(probs)
    assert e.value.status == L.SMC_ERR_UNSUPPORTED
    with pytest.raises(L.SmcError):
        L.smc_batch_plan_queue(_problems(L, shapes), 2, 1)      # unknown order
    with pytest.raises(L.SmcError):
        L.smc_batch_plan_queue(_problems(L, shapes), 0, 3)      # tiles per item


def test_model_detects_an_item_before_its_dependency(L):
    # the model has teeth: a normalisation moved ahead of its tiles stalls a
    # single workgroup forever
    shapes = _shapes_small()
    items = [tuple(int(x) for x in r) for r in L.smc_batch_plan_queue(_problems(L, shapes), 0, 1)]
    k = next(i for i, it in enumerate(items) if it[0] == IT_FINAL)
    bad = [items[k]] + items[:k] + items[k + 1:]
    with pytest.raises(AssertionError, match="deadlock"):
        _simulate(bad, shapes, 1, 1, seed=0)
