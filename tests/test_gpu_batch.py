"""Many interferograms through the job server (ww_server_*) and the batch
call (ww_unwrap_batch, one min-cost-flow solve over the union of the jobs'
graphs): every job's K, phi and cost must be byte-identical to the plain
one-job ww_unwrap on the same inputs, alone or in a mix, with host or device
arrays, and its cost must equal the CPU oracle's optimum."""
import time

import numpy as np
import pytest

import oracle
from paper_2609_36267_amd import binding as ww
from paper_2609_36267_amd import synth

pytestmark = pytest.mark.gpu

# (m, n, looks, seed): several tiles and ragged tails, three looks values
JOBS = [(96, 130, 9, 11), (200, 150, 5, 12), (64, 300, 15, 13), (257, 129, 9, 14),
        (33, 45, 5, 15), (150, 150, 15, 16), (2, 300, 9, 17), (300, 2, 5, 18)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    ww.load()
    return torch


@pytest.fixture(scope="module")
def scenes():
    out = []
    for m, n, L, seed in JOBS:
        sc = synth.make(m, n, looks=L, seed=seed, mask_frac=0.05, disks=1,
                        disk_radius=(8, 20), keep_truth=False, workers=1)
        out.append(sc)
    return out


@pytest.fixture(scope="module")
def plain(torch_cuda, scenes):
    """Plain path results: (K, phi, cost) as numpy."""
    res = []
    for sc in scenes:
        K, phi, tot = ww.unwrap(sc.psi, sc.coh, sc.valid, sc.looks)
        res.append((K.cpu().numpy(), phi.cpu().numpy(), tot))
    return res


def same_phi(a, b):
    return np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_plain_costs_equal_oracle(plain, scenes):
    for sc, (_, _, tot) in zip(scenes, plain):
        _, _, total = oracle.unwrap(sc.psi, sc.coh, sc.valid, sc.looks)
        assert tot == total, (sc.psi.shape, sc.looks)


@pytest.fixture(scope="module")
def certs(scenes):
    """The oracle's optimum of every job: (K, fixed-edge masks, reference)."""
    out = []
    for sc in scenes:
        m, n = sc.psi.shape
        o = oracle.unwrap(sc.psi, sc.coh, sc.valid, sc.looks, want=True)
        fx, fy = oracle.fixed_edges(o["costs"], o["dkx"], o["dky"], o["pot"])
        out.append((o["K"], fx, fy, oracle.ref_index(sc.valid, m, n), o["total"]))
    return out


def check_batch_job(sc, cert, K, phi, tot):
    """A batch result: the oracle's optimal cost, the oracle's K on every
    pixel the optimum fixes, phi within tolerance of psi + 2 pi K."""
    from tests.helpers import assert_same_on_certified_pixels, phase_tolerance_ok
    Ko, fx, fy, ref, total = cert
    assert tot == total
    K = K if isinstance(K, np.ndarray) else K.cpu().numpy()
    phi = phi if isinstance(phi, np.ndarray) else phi.cpu().numpy()
    assert_same_on_certified_pixels(K, Ko, fx, fy, ref)
    ok, err = phase_tolerance_ok(phi, sc.psi, K, sc.valid)
    assert ok, err


@pytest.mark.parametrize("group", [1, 3, 8, 0])
def test_batch_matches_plain(torch_cuda, scenes, plain, certs, group):
    """Groups of 1, 3 and all jobs per solve (the two jobs without loops
    take the plain path inside the call): the plain path's cost, the
    oracle's K wherever the optimum is unique, byte-identical to the plain
    path for one job per solve, and identical bytes on a repeated call."""
    torch = torch_cuda
    jobs = [(torch.from_numpy(sc.psi).cuda(), torch.from_numpy(sc.coh).cuda(),
             torch.from_numpy(sc.valid).cuda(), sc.looks) for sc in scenes]
    results, arr = ww.unwrap_batch(jobs, group=group)
    again, _ = ww.unwrap_batch(jobs, group=group)
    for sc, cert, (K, phi, tot), (Kp, phip, totp), j, (K2, phi2, tot2) in zip(
            scenes, certs, results, plain, arr, again):
        assert j.status == 0
        assert tot == totp == tot2
        check_batch_job(sc, cert, K, phi, tot)
        assert np.array_equal(K.cpu().numpy(), K2.cpu().numpy())
        assert same_phi(phi.cpu().numpy(), phi2.cpu().numpy())
        if group == 1:
            assert np.array_equal(K.cpu().numpy(), Kp)
            assert same_phi(phi.cpu().numpy(), phip)
        assert j.t_submit <= j.t_start <= j.t_end


@pytest.mark.parametrize("sched", [(64, 256, 0, 0, 1 << 30), (1, 1, 2, 1, 1), (64, 256, 8, 1, 0),
                                   (64, 256, 4, 0, 1024, 8), (64, 256, 4, 0, 1024, 8, 64),
                                   (1, 1, 2, 1, 1, 2, 16)])
def test_batch_schedules_and_checks(torch_cuda, scenes, certs, sched, monkeypatch):
    """One solve over all jobs under extreme schedules, the reversed frame
    included, with the solver's debug checks on (non-negative reduced costs
    in every job after every pass, tile lists in bounds and without
    repeats): every job reaches the oracle's optimum."""
    torch = torch_cuda
    monkeypatch.setenv("WW_MCF_CHECK", "1")
    jobs = [(torch.from_numpy(sc.psi).cuda(), torch.from_numpy(sc.coh).cuda(),
             torch.from_numpy(sc.valid).cuda(), sc.looks) for sc in scenes]
    results, arr = ww.unwrap_batch(jobs, sched=sched)
    for sc, cert, (K, phi, tot), j in zip(scenes, certs, results, arr):
        assert j.status == 0, j.error
        check_batch_job(sc, cert, K, phi, tot)


@pytest.mark.parametrize("sched", [None, (64, 256, 4, 0, 1024, 8)])
def test_batch_root_walk_modes_identical(torch_cuda, scenes, certs, sched, monkeypatch):
    """One solve over all jobs with the root walks taken by one thread each
    (WW_MCF_ROOTS=t), by a workgroup each (w) and split by length (the
    default): every job's K, phi and cost byte-identical across the three,
    and the oracle's optimum."""
    torch = torch_cuda
    jobs = [(torch.from_numpy(sc.psi).cuda(), torch.from_numpy(sc.coh).cuda(),
             torch.from_numpy(sc.valid).cuda(), sc.looks) for sc in scenes]
    out = {}
    for mode in ("a", "t", "w"):
        monkeypatch.setenv("WW_MCF_ROOTS", mode)
        results, arr = ww.unwrap_batch(jobs, sched=sched)
        assert all(j.status == 0 for j in arr), mode
        out[mode] = [(K.cpu().numpy(), phi.cpu().numpy(), tot) for K, phi, tot in results]
    monkeypatch.delenv("WW_MCF_ROOTS")
    for mode in ("t", "w"):
        for (Ka, pa, ta), (Kb, pb, tb) in zip(out["a"], out[mode]):
            assert ta == tb, mode
            assert np.array_equal(Ka, Kb), mode
            assert same_phi(pa, pb), mode
    for sc, cert, (K, phi, tot) in zip(scenes, certs, out["a"]):
        check_batch_job(sc, cert, K, phi, tot)


def test_batch_stack_of_many_jobs(torch_cuda):
    """24 jobs of the stack recipe at reduced size (rows 64-300, cols
    64-420, L in {5, 9, 15}) in one solve, host-side arrays for every third:
    each reaches the CPU oracle's optimum."""
    torch = torch_cuda
    rng = np.random.default_rng(77)
    scs, jobs = [], []
    for k in range(24):
        m, n = int(rng.integers(64, 301)), int(rng.integers(64, 421))
        sc = synth.make(m, n, looks=int(rng.choice([5, 9, 15])), seed=300 + k, mask_frac=0.03,
                        disks=1, disk_radius=(6, 16), keep_truth=False, workers=1)
        scs.append(sc)
        if k % 3 == 0:
            jobs.append((sc.psi, sc.coh, sc.valid, sc.looks))
        else:
            jobs.append((torch.from_numpy(sc.psi).cuda(), torch.from_numpy(sc.coh).cuda(),
                         torch.from_numpy(sc.valid).cuda(), sc.looks))
    results, arr = ww.unwrap_batch(jobs)
    for sc, (K, phi, tot), j in zip(scs, results, arr):
        assert j.status == 0, j.error
        m, n = sc.psi.shape
        o = oracle.unwrap(sc.psi, sc.coh, sc.valid, sc.looks, want=True)
        fx, fy = oracle.fixed_edges(o["costs"], o["dkx"], o["dky"], o["pot"])
        check_batch_job(sc, (o["K"], fx, fy, oracle.ref_index(sc.valid, m, n), o["total"]), K, phi, tot)


def test_batch_bad_job_fails_alone(torch_cuda, scenes, plain):
    torch = torch_cuda
    jobs = [(torch.from_numpy(sc.psi).cuda(), torch.from_numpy(sc.coh).cuda(),
             torch.from_numpy(sc.valid).cuda(), sc.looks) for sc in scenes[:4]]
    jobs[2] = jobs[2][:3] + (1,)  # L = 1 is outside [2, 64]
    arr = (ww.Job * 4)()
    keep = []
    for k, (psi, coh, valid, looks) in enumerate(jobs):
        j, kp = ww.make_job(psi, coh, valid, looks, tag=k)
        arr[k] = j
        keep.append(kp)
    rc = ww.load().ww_unwrap_batch(arr, 4, 0, None)
    assert rc == ww.E_INVALID_ARG
    assert arr[2].status == ww.E_INVALID_ARG and b"looks" in arr[2].error
    for k in (0, 1, 3):
        assert arr[k].status == 0 and arr[k].total_cost == plain[k][2]


def test_server_per_job_schedule(torch_cuda, scenes, plain):
    """Jobs carrying their own schedule (use_sched) keep the optimum, and
    the process-wide schedule is untouched."""
    torch = torch_cuda
    before = ww.get_mcf_params().as_tuple()
    with ww.Server(slots=3) as srv:
        for k, sc in enumerate(scenes[:6]):
            j = srv.submit(torch.from_numpy(sc.psi).cuda(), torch.from_numpy(sc.coh).cuda(),
                           torch.from_numpy(sc.valid).cuda(), sc.looks, tag=k,
                           sched=[(1, 1, 2, 1, 1, 2, 64), (64, 256, 0, 0, 1 << 30, 2, 16), None][k % 3])
        done = srv.drain()
    assert ww.get_mcf_params().as_tuple() == before
    for j, K, phi in done:
        assert j.status == 0, j.error
        assert j.total_cost == plain[j.tag][2]


def test_server_host_arrays_in_a_mix(torch_cuda, scenes, plain):
    """Jobs arrive while others run; host arrays are copied in and out."""
    with ww.Server(slots=3) as srv:
        jobs = []
        for k, sc in enumerate(scenes * 2):
            jobs.append(srv.submit(sc.psi, sc.coh, sc.valid, sc.looks, tag=k))
            if k % 3 == 2:
                time.sleep(0.002)
        done = srv.drain()
    assert len(done) == 2 * len(scenes)
    for j, K, phi in done:
        assert j.status == 0, j.error
        Kp, phip, totp = plain[j.tag % len(scenes)]
        assert j.total_cost == totp
        assert np.array_equal(K, Kp)
        assert same_phi(phi, phip)


def test_server_device_arrays_and_poll(torch_cuda, scenes, plain):
    torch = torch_cuda
    with ww.Server(slots=2) as srv:
        for k, sc in enumerate(scenes):
            srv.submit(torch.from_numpy(sc.psi).cuda(), torch.from_numpy(sc.coh).cuda(),
                       torch.from_numpy(sc.valid).cuda(), sc.looks, tag=k)
        got = []
        t0 = time.time()
        while len(got) < len(scenes) and time.time() - t0 < 60:
            got += srv.poll(wait_ms=100)
        assert srv.in_flight() == 0
    assert sorted(j.tag for j, _, _ in got) == list(range(len(scenes)))
    for j, K, phi in got:
        Kp, phip, totp = plain[j.tag]
        assert j.total_cost == totp
        assert np.array_equal(K.cpu().numpy(), Kp)
        assert same_phi(phi.cpu().numpy(), phip)


def test_job_out_of_memory_fails_alone(torch_cuda, scenes, plain, monkeypatch):
    """A job whose workspace cannot be allocated (device allocations above
    WW_SCRATCH_LIMIT refused as a failed allocation would be) ends with
    WW_E_OOM and its message; the other jobs of the same server finish with
    their costs alone, and the server takes the big job once the limit is
    gone."""
    torch = torch_cuda
    big = synth.make(600, 600, looks=9, seed=21, mask_frac=0.05, disks=1, disk_radius=(20, 40),
                     keep_truth=False, workers=1)
    big_cost = ww.unwrap(big.psi, big.coh, big.valid, big.looks)[2]
    small = list(range(4))  # at most 33 k pixels: every buffer well below 4 MB
    assert max(scenes[k].psi.size for k in small) < 40000
    dev = lambda sc: (torch.from_numpy(sc.psi).cuda(), torch.from_numpy(sc.coh).cuda(),  # noqa: E731
                      torch.from_numpy(sc.valid).cuda())
    monkeypatch.setenv("WW_SCRATCH_LIMIT", str(4 << 20))  # the big job's keys alone take 8.6 MB
    with ww.Server(slots=2) as srv:
        for k in small:
            srv.submit(*dev(scenes[k]), scenes[k].looks, tag=k)
        srv.submit(*dev(big), big.looks, tag=99)
        done = srv.drain()
        monkeypatch.delenv("WW_SCRATCH_LIMIT")
        assert len(done) == len(small) + 1
        for j, K, phi in done:
            if int(j.tag) == 99:
                assert j.status == ww.E_OOM, (j.status, j.error)
                assert b"WW_SCRATCH_LIMIT" in j.error
            else:
                assert j.status == 0, j.error
                assert int(j.total_cost) == plain[int(j.tag)][2]
        srv.submit(*dev(big), big.looks, tag=99)
        (j, K, phi), = srv.drain()
        assert j.status == 0, j.error
        assert int(j.total_cost) == big_cost


def test_tiny_budget_runs_jobs_one_at_a_time(torch_cuda, scenes, plain):
    """With a budget below any job's footprint each job runs alone."""
    with ww.Server(slots=4, hbm_budget_bytes=1) as srv:
        for k, sc in enumerate(scenes):
            srv.submit(sc.psi, sc.coh, sc.valid, sc.looks, tag=k)
        done = srv.drain()
    spans = sorted((j.t_start, j.t_end) for j, _, _ in done)
    for (s0, e0), (s1, e1) in zip(spans, spans[1:]):
        assert s1 >= e0
    for j, K, phi in done:
        assert j.total_cost == plain[j.tag][2]
        assert j.footprint_bytes > 1


def test_bad_job_fails_alone(torch_cuda, scenes, plain):
    sc = scenes[0]
    with ww.Server(slots=2) as srv:
        good = srv.submit(sc.psi, sc.coh, sc.valid, sc.looks, tag=0)
        bad = srv.submit(sc.psi, sc.coh, sc.valid, 1, tag=1)  # L = 1 is outside [2, 64]
        done = {j.tag: j for j, _, _ in srv.drain()}
    assert done[1].status == ww.E_INVALID_ARG and b"looks" in done[1].error
    assert done[0].status == 0 and done[0].total_cost == plain[0][2]
    assert good.tag == 0 and bad.tag == 1


def test_window_schedule_keeps_the_optimum(torch_cuda, scenes, plain):
    """Any window schedule reaches the same optimal cost, and K agrees with
    the oracle wherever the optimum is unique; the autotuner installs one of
    its candidates."""
    from paper_2609_36267_amd import autotune
    from tests.helpers import assert_same_on_certified_pixels, assert_same_on_fixed_edges
    torch = torch_cuda
    old = ww.get_mcf_params()
    try:
        for k in (0, 1, 3):
            sc = scenes[k]
            m, n = sc.psi.shape
            out = oracle.unwrap(sc.psi, sc.coh, sc.valid, sc.looks, want=True)
            # windows, and the pass schedules: the paper's (eight full passes,
            # then first-deficit passes), full passes only, first-deficit only
            for sched in ((1, 1, 0, 0), (16, 64, 0, 0), (1 << 28, 1 << 20, 0, 0), (64, 256, 8, 1),
                          (16, 64, 1000, 0), (64, 256, 0, 1), (64, 256, 2, 0, 1), (64, 256, 0, 0, 64),
                          (64, 256, 0, 0, 1 << 30)):
                ww.set_mcf_params(*sched)
                K, phi, tot = ww.unwrap(sc.psi, sc.coh, sc.valid, sc.looks)
                assert tot == out["total"] == plain[k][2]
                r = ww.mcf_solve(out["res"], out["costs"], m, n)
                fx, fy = assert_same_on_fixed_edges(out["costs"], out["dkx"], out["dky"], out["pot"],
                                                    r.dk_x.cpu().numpy(), r.dk_y.cpu().numpy())
                assert_same_on_certified_pixels(K.cpu().numpy(), out["K"], fx, fy,
                                                oracle.ref_index(sc.valid, m, n))
        jobs = [(torch.from_numpy(sc.psi).cuda(), torch.from_numpy(sc.coh).cuda(),
                 torch.from_numpy(sc.valid).cuda(), sc.looks) for sc in scenes[:3]]
        choice, table = autotune.tune_schedule(jobs, candidates=[(64, 256), (16, 64),
                                                                 autotune.PAPER_SCHEDULE])
        p = ww.get_mcf_params()
        assert choice in table
        assert p.as_tuple() == autotune.pad(choice)
    finally:
        ww.set_mcf_params(*old.as_tuple())
