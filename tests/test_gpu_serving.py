"""Serving loop (gcdf_submit / gcdf_poll) on the GPU, through the C ABI.

Each request's tiles run in the same per-tile code as gcdf_query, so results
must be bitwise equal to the one-shot call, alone or mixed with other requests.
"""
import time

import numpy as np
import pytest

from paper_2601_18548_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GiB = 1 << 30


@pytest.fixture(scope="module")
def gcdf():
    import paper_2601_18548_amd as g

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g.library()
    return g


class Req:
    def __init__(self, K, Np, seed, outputs=("d", "J", "min", "jmin")):
        self.k = torch.from_numpy(wl.knots(K, seed)).cuda()
        self.p = torch.from_numpy(wl.points_patches(Np, seed + 1)).cuda()
        self.d = torch.full((K, Np), float("nan"), device="cuda") if "d" in outputs else None
        self.J = torch.full((K, Np, 9), float("nan"), device="cuda") if "J" in outputs else None
        self.dmin = torch.full((K,), float("nan"), device="cuda") if "min" in outputs else None
        self.am = torch.full((K,), -7, dtype=torch.int32, device="cuda") if "min" in outputs else None
        self.Jm = torch.full((K, 9), float("nan"), device="cuda") if "jmin" in outputs else None

    def submit(self, ctx):
        return ctx.submit(self.k, self.p, self.d, self.J, self.dmin, self.am, self.Jm)

    def arrays(self):
        return [None if t is None else t.cpu().numpy() for t in (self.d, self.J, self.dmin, self.am, self.Jm)]


def wait_all(ctx, tickets, timeout=60.0):
    t0 = time.time()
    pending = set(tickets)
    while pending:
        for t in list(pending):
            if ctx.poll(t):
                pending.discard(t)
        assert time.time() - t0 < timeout, "serving did not finish"
        time.sleep(0.0005)


def reference(ctx_q, r):
    """The one-shot calls' d, J, dmin, argmin and Jmin (gcdf_knot_min's)."""
    d, J = ctx_q.eval_grad(r.k, r.p)
    dmin, am, Jm = ctx_q.knot_min(r.k, r.p, with_jacobian=True)
    torch.cuda.synchronize()
    return [d.cpu().numpy(), J.cpu().numpy(), dmin.cpu().numpy(), am.cpu().numpy(), Jm.cpu().numpy()]


@pytest.fixture(scope="module")
def weights():
    return wl.weights(256, seed=21)


def test_single_request_matches_one_shot_bitwise(gcdf, weights):
    srv = gcdf.Context(weights.to_blob(), 256, "bf16x2", serve_mem_budget=4 * GiB, serve_slots=8)
    one = gcdf.Context(weights.to_blob(), 256, "bf16x2")
    r = Req(20, 1000, 3)
    wait_all(srv, [r.submit(srv)])
    got = r.arrays()
    ref = reference(one, r)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    srv.close()


def test_alone_and_in_the_mix_are_identical(gcdf, weights):
    srv = gcdf.Context(weights.to_blob(), 256, "bf16x2", serve_mem_budget=8 * GiB, serve_slots=16)
    probe = Req(33, 2500, 5)
    wait_all(srv, [probe.submit(srv)])
    alone = probe.arrays()
    # the same request again, submitted in the middle of a burst of uneven requests
    rng = np.random.default_rng(1)
    others = [Req(int(rng.integers(16, 80)), int(rng.integers(512, 6000)), 100 + i) for i in range(12)]
    probe2 = Req(33, 2500, 5)
    tickets = [o.submit(srv) for o in others[:6]] + [probe2.submit(srv)] + [o.submit(srv) for o in others[6:]]
    wait_all(srv, tickets)
    for a, b in zip(alone, probe2.arrays()):
        assert np.array_equal(a, b)
    one = gcdf.Context(weights.to_blob(), 256, "bf16x2")
    for o in others[::3]:
        for a, b in zip(o.arrays(), reference(one, o)):
            assert np.array_equal(a, b)
    srv.close()


def test_results_match_oracle_on_samples(gcdf, oracle_mod, weights):
    srv = gcdf.Context(weights.to_blob(), 256, "bf16x2", serve_mem_budget=4 * GiB, serve_slots=8)
    r = Req(17, 777, 9)
    wait_all(srv, [r.submit(srv)])
    d, J, dmin, am, Jm = r.arrays()
    k, p = r.k.cpu().numpy(), r.p.cpu().numpy()
    ki = np.arange(17).repeat(8)
    pi = np.random.default_rng(2).integers(0, 777, len(ki))
    dr, Jr = oracle_mod.eval_pairs(weights.to_blob(), k, p, ki, pi)
    assert np.abs(d[ki, pi] - dr).max() <= 1e-3
    nr = np.linalg.norm(Jr, axis=1)
    assert (np.linalg.norm(J[ki, pi] - Jr, axis=1) / np.maximum(nr, 1e-3 * np.median(nr))).max() <= 1e-2
    assert np.array_equal(dmin, d.min(axis=1)) and np.array_equal(am, d.argmin(axis=1))
    # J at the argmin against the oracle's J of the same pairs
    dm_r, Jm_r = oracle_mod.eval_pairs(weights.to_blob(), k, p, np.arange(17), am)
    assert np.abs(dmin - dm_r).max() <= 1e-3
    nm = np.linalg.norm(Jm_r, axis=1)
    assert (np.linalg.norm(Jm - Jm_r, axis=1) / np.maximum(nm, 1e-3 * np.median(nr))).max() <= 1e-2
    srv.close()


def test_memory_budget_admission_and_errors(gcdf, weights):
    # budget fits one of these requests at a time: they must still all finish
    r0 = Req(40, 3000, 11)
    per_req = 40 * 36 + 3000 * 12 + 40 * 3000 * 40 + 40 * 16 + 40 * 36
    srv = gcdf.Context(weights.to_blob(), 256, "bf16x2", serve_mem_budget=int(per_req * 1.5), serve_slots=4)
    reqs = [r0] + [Req(40, 3000, 12 + i) for i in range(3)]
    wait_all(srv, [r.submit(srv) for r in reqs])
    one = gcdf.Context(weights.to_blob(), 256, "bf16x2")
    for r in reqs:
        for a, b in zip(r.arrays(), reference(one, r)):
            assert np.array_equal(a, b)
    # larger than the whole budget: rejected at submit
    big = Req(80, 3000, 30)
    with pytest.raises(gcdf.GcdfError) as e:
        big.submit(srv)
    assert e.value.status == gcdf.ENOMEM
    # unknown ticket, and a ticket already reported complete
    with pytest.raises(gcdf.GcdfError):
        srv.poll(987654321)
    t = Req(16, 512, 31).submit(srv)
    wait_all(srv, [t])
    with pytest.raises(gcdf.GcdfError):
        srv.poll(t)
    srv.close()


def test_outputs_subsets_and_drain_on_close(gcdf, weights):
    srv = gcdf.Context(weights.to_blob(), 256, "bf16x2", serve_mem_budget=4 * GiB, serve_slots=8)
    only_min = Req(25, 4000, 40, outputs=("min",))
    only_d = Req(10, 900, 41, outputs=("d",))
    for r in (only_min, only_d):
        r.submit(srv)
    srv.close()  # must wait for both
    one = gcdf.Context(weights.to_blob(), 256, "bf16x2")
    dmin, am = one.knot_min(only_min.k, only_min.p)
    assert np.array_equal(only_min.dmin.cpu().numpy(), dmin.cpu().numpy())
    assert np.array_equal(only_min.am.cpu().numpy(), am.cpu().numpy())
    assert np.array_equal(only_d.d.cpu().numpy(), one.eval(only_d.k, only_d.p).cpu().numpy())


def test_serving_disabled_rejects_submit(gcdf, weights):
    ctx = gcdf.Context(weights.to_blob(), 256, "bf16x2")
    with pytest.raises(gcdf.GcdfError):
        Req(16, 512, 50).submit(ctx)


@pytest.mark.parametrize("width,precision", [(512, "bf16x2"), (512, "bf16"), (512, "fp32"), (256, "fp32"),
                                             (256, "bf16x2_f16"), (512, "bf16x2_f16")])
def test_other_widths_and_precisions_match_one_shot(gcdf, width, precision):
    """Serving instantiations beyond the benchmark's (width 512 runs 8 waves in the
    BF16 modes, FP32 runs 4): bitwise equal to the one-shot query, including a
    request that arrives after the loop went idle and exited (relaunch)."""
    w = wl.weights(width, seed=22)
    srv = gcdf.Context(w.to_blob(), width, precision, serve_mem_budget=2 * GiB, serve_slots=4)
    one = gcdf.Context(w.to_blob(), width, precision)
    first = [Req(9, 700, 60), Req(5, 130, 61)]
    wait_all(srv, [r.submit(srv) for r in first])
    time.sleep(0.02)  # well past the 2 ms idle exit
    late = Req(12, 1000, 62)
    wait_all(srv, [late.submit(srv)])
    for r in first + [late]:
        for a, b in zip(r.arrays(), reference(one, r)):
            assert np.array_equal(a, b)
    srv.close()


@pytest.mark.parametrize("slots", [2, 3, 4])
def test_many_small_requests_through_few_slots(gcdf, weights, slots):
    """Far more requests in flight than slots, small and uneven (1-7 knots, 1-300
    points: a few tiles each), so slots are reused while workgroups whose cursors
    lag still walk past the completed requests; every result bitwise equal to the
    one-shot calls, within a host-side deadline."""
    print("case many small requests, slots=%d" % slots, flush=True)
    srv = gcdf.Context(weights.to_blob(), 256, "bf16x2_f16", serve_mem_budget=2 * GiB, serve_slots=slots)
    one = gcdf.Context(weights.to_blob(), 256, "bf16x2_f16")
    rng = np.random.default_rng(40 + slots)
    reqs = [Req(int(rng.integers(1, 8)), int(rng.integers(1, 301)), 300 + 7 * i) for i in range(96)]
    wait_all(srv, [r.submit(srv) for r in reqs], timeout=30.0)
    for r in reqs:
        for a, b in zip(r.arrays(), reference(one, r)):
            assert np.array_equal(a, b)
    srv.close()


def test_jmin_needs_the_minimum(gcdf, weights):
    srv = gcdf.Context(weights.to_blob(), 256, "bf16x2", serve_mem_budget=GiB, serve_slots=2)
    r = Req(4, 100, 70)
    with pytest.raises(gcdf.GcdfError) as e:
        srv.submit(r.k, r.p, r.d, r.J, None, None, r.Jm)
    assert e.value.status == gcdf.EINVAL
    with pytest.raises(ValueError):  # argmin of the wrong dtype never reaches the library
        srv.submit(r.k, r.p, r.d, r.J, r.dmin, r.dmin, r.Jm)
    srv.close()
