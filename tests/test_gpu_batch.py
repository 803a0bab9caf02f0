"""GPU tests of the batched persistent step: FP32 instances of uneven shape
and dimension, against the FP64 oracle; bitwise independence from the rest of
the batch; graph replays equal direct launches; isolation of a blown-up
instance."""
import numpy as np
import pytest
import torch

import oracle
from paper_1605_03958_amd import inputs, sscn
from paper_1605_03958_amd.sscn import F32, IMAG, REAL, Problem

pytestmark = pytest.mark.gpu


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def errors(a, b, dim):
    """(relative L2, largest deviation / largest |b|, relative L2 over the
    grid faces -- the points at either end of a line along a used axis,
    where a wrong boundary or line-end treatment would show)."""
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    a = a.reshape(b.shape) if a.size == b.size else a
    d = a - b
    face = np.zeros(b.shape, dtype=bool)
    for ax in range(dim):
        sl = [slice(None)] * 3
        for end in (0, -1):
            sl[2 - ax] = end
            face[tuple(sl)] = True
    # faces far out in the trap hold values orders below the peak, whose
    # FP32 error is rounding relative to the peak: the faces' norm is floored
    # at 1e-2 of the peak per face point (a wrong boundary term would still
    # show: it errs by a fraction of the face values themselves)
    floor = 1e-2 * np.max(np.abs(b)) * np.sqrt(face.sum())
    return (float(np.linalg.norm(d) / np.linalg.norm(b)),
            float(np.max(np.abs(d)) / np.max(np.abs(b))),
            float(np.linalg.norm(d[face]) / max(np.linalg.norm(b[face]), floor)))


def assert_fp32_close(a, b, dim, what=""):
    """FP32 state against the FP64 oracle: relative L2 <= 5e-5, every point
    within 2e-5 of the largest value, faces to relative L2 <= 5e-5."""
    l2, mx, fc = errors(a, b, dim)
    print(f"{what} rel-L2 {l2:.2e} max {mx:.2e} faces {fc:.2e}", flush=True)
    assert l2 <= 5e-5 and mx <= 2e-5 and fc <= 5e-5, (what, l2, mx, fc)


def oprob(p: Problem) -> oracle.Problem:
    return oracle.Problem(p.dim, p.n, p.dx, p.omega, p.g, p.dt, p.mode, p.renorm_every)


def make(dim, n, mode, g=5.0, dx=None, seed=0, observe_every=10):
    dx = dx or tuple([0.1 if dim == 1 else 0.2] * dim)
    om = (1.0, 1.5, 2.0)[:dim]
    h = min(dx)
    dt = 0.1 * h * h if mode == IMAG else 0.02 * h * h
    p = Problem(dim, n, dx, om, g, dt, mode, F32, 1 if mode == IMAG else 0, observe_every)
    if mode == IMAG:
        psi0 = inputs.ho_gaussian(dim, p.n, p.dx, p.omega, noise=1e-3, seed=seed)
    else:
        psi0 = inputs.thomas_fermi(dim, p.n, p.dx, p.omega, 1.25 * g + 1, phase_sigma=0.05, seed=seed)
    return p, psi0


# shapes that exercise every tile variant of the persistent kernel
MIX = [
    (1, (64, 1, 1), IMAG), (1, (300, 1, 1), IMAG), (1, (1000, 1, 1), IMAG), (1, (3000, 1, 1), IMAG),
    (1, (12000, 1, 1), IMAG), (1, (500, 1, 1), REAL), (1, (6000, 1, 1), REAL), (1, (9000, 1, 1), REAL),
    (2, (40, 50, 1), IMAG), (2, (64, 130, 1), REAL), (2, (70, 700, 1), IMAG), (2, (33, 600, 1), REAL),
    (3, (20, 24, 30), IMAG), (3, (16, 20, 12), REAL), (3, (48, 49, 50), IMAG),
]


def run_batch(cases, steps, stream=None, slots=None):
    b = sscn.Batch(len(cases) if slots is None else max(slots) + 1, stream=stream)
    slots = slots or list(range(len(cases)))
    for s, (p, psi0) in zip(slots, cases):
        b.admit(s, p, psi0, mu_tol=0.0, max_steps=steps)
    b.step(steps)
    st = b.poll(wait=True)
    assert not b.error()
    out = [b.evict(s).cpu().numpy() for s in slots]
    b.close()
    return out, [st[s] for s in slots]


def test_batch_matches_oracle_across_tile_variants():
    cases = [make(d, n, m, seed=i) for i, (d, n, m) in enumerate(MIX)]
    steps = 30
    got, st = run_batch(cases, steps)
    for (p, psi0), g, s in zip(cases, got, st):
        print(f"dim={p.dim} n={p.n} mode={p.mode}", flush=True)
        assert s.state == sscn.SLOT_DONE and s.steps == steps
        ref = oracle.run(oprob(p), psi0, steps).psi
        assert_fp32_close(g, ref, p.dim, f"n={p.n} mode={p.mode}")
        orf = oracle.observe(oprob(p), ref)
        assert abs(s.obs.mu - orf.mu) <= 1e-5 * max(1.0, abs(orf.mu))


def test_every_tile_variant_matches_the_oracle():
    """Tile hints force each points-per-thread variant of the persistent
    kernel on small instances of distinct shapes, in imaginary and real
    time, 20 steps against the oracle: the x lines of 3D instances in one
    wave (1..4 points per thread), longer x lines of 2D and 3D instances
    over several waves (4 and 8 points per thread), the y and z lines
    (2..16), and 1D lines in one wave with 6..16 points per thread (the solo
    cycle of the persistent kernel: no stream here)."""
    row = {IMAG: [1, 2, 3, 4], REAL: [1, 2, 3, 4]}
    col = {IMAG: [2, 3, 4, 5, 6, 8, 10, 12, 16], REAL: [2, 3, 4, 5, 6, 8]}
    cases = []
    i = 0
    try:
        for mode in (IMAG, REAL):
            m = max(len(row[mode]), len(col[mode]))
            for k in range(m):
                r = row[mode][k % len(row[mode])]
                cy = col[mode][k % len(col[mode])]
                cz = col[mode][(k + 3) % len(col[mode])]
                n = (25 + 3 * i, 20 + i, 18 + 2 * i)
                p, psi0 = make(3, n, mode, seed=60 + i)
                sscn.batch_set_tile_hint(p, (r, cy, cz))
                g = sscn.batch_plan_info(p)
                assert [g[0]["chunk"], g[1]["chunk"], g[2]["chunk"]] == [r, cy, cz]
                cases.append((p, psi0))
                i += 1
        # multi-wave x lines of 2D and 3D instances (no hint needed)
        for dim, n, mode, want in ((2, (700, 40, 1), IMAG, 4), (2, (700, 40, 1), REAL, 4),
                                   (2, (4500, 8, 1), IMAG, 8), (3, (300, 12, 10), REAL, 4)):
            p, psi0 = make(dim, n, mode, seed=60 + i)
            g = sscn.batch_plan_info(p)[0]
            assert g["chunk"] == want and g["waves"] > 1, g
            cases.append((p, psi0))
            i += 1
        # single-wave 1D lines of 6..16 points per thread
        for mode, cs in ((IMAG, (6, 8, 12, 16)), (REAL, (6, 8))):
            for c in cs:
                p, psi0 = make(1, (64 * c - 5 - i, 1, 1), mode, seed=60 + i)
                sscn.batch_set_tile_hint(p, (c, 0, 0))
                g = sscn.batch_plan_info(p)[0]
                assert g["chunk"] == c and g["waves"] == 1, g
                cases.append((p, psi0))
                i += 1
        got, st = run_batch(cases, 20)
    finally:
        sscn.batch_clear_tile_hints()
    for (p, psi0), gv, s in zip(cases, got, st):
        assert s.state == sscn.SLOT_DONE and s.steps == 20
        ref = oracle.run(oprob(p), psi0, 20).psi
        assert_fp32_close(gv, ref, p.dim, f"n={p.n} mode={p.mode}")


def test_alone_equals_in_the_mix_bitwise():
    a = make(3, (20, 24, 30), IMAG, seed=3)
    r = make(2, (64, 130, 1), REAL, seed=4)
    others = [make(d, n, m, seed=10 + i) for i, (d, n, m) in enumerate(MIX[:6])]
    alone, _ = run_batch([a, r], 25, slots=[5, 9])
    mix, _ = run_batch(others[:3] + [a] + others[3:] + [r], 25)
    assert np.array_equal(alone[0], mix[3])
    assert np.array_equal(alone[1], mix[7])


def test_graph_replays_equal_direct_launches():
    import torch
    cases = [make(d, n, m, seed=20 + i) for i, (d, n, m) in enumerate(MIX[8:14])]
    s = torch.cuda.Stream()
    b = sscn.Batch(len(cases), stream=s)
    for i, (p, psi0) in enumerate(cases):
        b.admit(i, p, psi0, mu_tol=0.0, max_steps=40)
    for _ in range(4):          # four replays of the same 10-step graph
        b.step(10)
        b.poll(wait=True)
        torch.zeros(1000, device="cuda").sum().item()   # unrelated eager work in between
    assert not b.error()
    graph = [b.evict(i).cpu().numpy() for i in range(len(cases))]
    b.close()
    direct, _ = run_batch(cases, 40, stream=torch.cuda.default_stream())
    for g, d in zip(graph, direct):
        assert np.array_equal(g, d)


def test_blown_up_instance_is_isolated():
    good = [make(d, n, m, seed=30 + i) for i, (d, n, m) in enumerate(MIX[8:12])]
    p, psi0 = make(2, (40, 50, 1), IMAG, seed=40)
    bad = psi0.copy()
    bad[0, 20, 20] = np.nan
    ref, _ = run_batch(good, 20)
    got, st = run_batch(good[:2] + [(p, bad)] + good[2:], 20)
    assert st[2].state == sscn.SLOT_NONFINITE and st[2].steps == 1
    for i, j in ((0, 0), (1, 1), (2, 3), (3, 4)):
        assert np.array_equal(ref[i], got[j])


def test_ground_state_stops_like_the_oracle():
    p, psi0 = make(2, (48, 40, 1), IMAG, g=10.0, dx=(0.3, 0.3), seed=7)
    b = sscn.Batch(1)
    b.admit(0, p, psi0, mu_tol=1e-5, max_steps=200000)
    for _ in range(200):
        b.step(100)
        st = b.poll(wait=True)[0]
        if st.state != sscn.SLOT_RUNNING:
            break
    assert st.state == sscn.SLOT_CONVERGED
    psi = b.evict(0).cpu().numpy()
    r = oracle.run(oprob(p), psi0, 200000, observe_every=10, mu_tol=1e-5)
    assert r.converged
    print(f"batch stop {st.steps} oracle stop {r.steps} mu {st.obs.mu} oracle {r.trace[-1, 2]}", flush=True)
    assert abs(st.steps - r.steps) <= 0.1 * r.steps
    assert abs(st.obs.mu - r.trace[-1, 2]) <= 1e-4
    n = np.prod(p.dx[:2]) * np.sum(np.abs(psi.astype(np.float64)) ** 2)
    assert abs(n - 1) <= 1e-5          # evict applied the pending renormalisation


def test_batch_equals_single_problem_fp32():
    """Same arithmetic as the single-problem kernels (only the order of the
    norm partial sums differs)."""
    p, psi0 = make(3, (32, 30, 28), IMAG, seed=8)
    got, _ = run_batch([(p, psi0)], 25)
    s = sscn.Solver(p, psi0)
    s.step(25)
    single = s.state()
    s.close()
    assert rel_l2(got[0], single) <= 1e-6


def test_work_list_capacity_is_enforced():
    p, psi0 = make(3, (20, 24, 30), IMAG)
    need = sum(g["items"] for g in sscn.batch_plan_info(p)) + -(-p.points // 16384) + 1
    b = sscn.Batch(2, max_items=need - 1)
    with pytest.raises(sscn.SSCNError) as e:
        b.admit(0, p, psi0)
    assert e.value.code == sscn.E_NOSPACE
    b.close()
    b = sscn.Batch(2, max_items=need)
    b.admit(0, p, psi0)
    b.close()


@pytest.mark.parametrize("n,mode", [(5000, IMAG), (2048, REAL), (9912, IMAG), (12000, REAL)])
def test_solo_instance_steps_and_mix_independence(n, mode):
    """A 1D instance runs whole steps inside one block: alone (the solo
    kernel, line held in registers) it advances 64 steps per launch; next to
    a 3D instance (the persistent kernel's solo cycle) it advances at least
    one per launch, and its state is bitwise the same either way."""
    one = make(1, (n, 1, 1), mode, seed=50)
    big = make(3, (48, 49, 50), IMAG, seed=51)
    b = sscn.Batch(2)
    b.admit(0, one[0], one[1], mu_tol=0.0, max_steps=300)
    b.step(2)
    st = b.poll(wait=True)[0]
    assert st.state == sscn.SLOT_RUNNING and st.steps == 128
    b.step(3)
    st = b.poll(wait=True)[0]
    assert st.state == sscn.SLOT_DONE and st.steps == 300
    alone_obs = st.obs
    alone = b.evict(0).cpu().numpy()
    b.close()

    # on the default stream the persistent kernel runs the solo instance's
    # steps itself; on a stream of its own the solo kernel runs them beside it
    for stream in (None, torch.cuda.Stream()):
        b = sscn.Batch(2, stream=stream)
        b.admit(1, big[0], big[1], mu_tol=0.0, max_steps=1 << 30)
        b.admit(0, one[0], one[1], mu_tol=0.0, max_steps=300)
        launches = 0
        while True:
            b.step(1)
            launches += 1
            st = b.poll(wait=True)
            assert st[1].steps == launches and st[0].steps >= min(launches, 300)
            if st[0].state != sscn.SLOT_RUNNING:
                break
            assert launches < 300
        assert not b.error()
        assert st[0].state == sscn.SLOT_DONE and st[0].steps == 300
        print(f"solo finished 300 steps in {launches} launches beside a 48x49x50 instance "
              f"({'default' if stream is None else 'own'} stream)", flush=True)
        mix_obs = st[0].obs
        mix = b.evict(0).cpu().numpy()
        b.close()
        assert np.array_equal(alone, mix)
        assert alone_obs == mix_obs
    ref = oracle.run(oprob(one[0]), one[1], 300).psi
    assert_fp32_close(mix, ref, 1, f"solo n={n} mode={mode}")


def test_item_split_setting():
    """The work-item split is a batch setting: refused once instances are
    admitted; at any split results match the oracle, and within one split an
    instance is bitwise the same alone and in a mix."""
    big = make(3, (60, 64, 56), IMAG, seed=70)
    other = [make(d, n, m, seed=71 + i) for i, (d, n, m) in enumerate(MIX[8:13])]
    b = sscn.Batch(2, split=8)
    b.admit(0, big[0], big[1], mu_tol=0.0, max_steps=20)
    with pytest.raises(sscn.SSCNError) as e:
        lib_rc = sscn.lib().sscn_batch_set_split(b._h, 64)
        sscn._check(lib_rc, "sscn_batch_set_split")
    assert e.value.code == sscn.E_INVALID
    b.close()
    ref = oracle.run(oprob(big[0]), big[1], 20).psi
    for split in (1, 8, 64, 4096):
        def run(cases, slots):
            bb = sscn.Batch(max(slots) + 1, split=split)
            for s_, (p, psi0) in zip(slots, cases):
                bb.admit(s_, p, psi0, mu_tol=0.0, max_steps=20)
            bb.step(20)
            bb.poll(wait=True)
            assert not bb.error()
            out = [bb.evict(s_).cpu().numpy() for s_ in slots]
            bb.close()
            return out
        alone = run([big], [3])[0]
        mix = run(other[:2] + [big] + other[2:], list(range(6)))[2]
        assert np.array_equal(alone, mix), split
        err = rel_l2(alone, ref)
        print(f"split {split}: rel L2 vs oracle {err:.2e}", flush=True)
        assert err <= 5e-5


def _run_alone(case, mu_tol, max_steps, stream=None):
    b = sscn.Batch(1, stream=stream)
    b.admit(0, case[0], case[1], mu_tol=mu_tol, max_steps=max_steps)
    while True:
        b.step(20)
        st = b.poll(wait=True)[0]
        if st.state != sscn.SLOT_RUNNING:
            break
    assert not b.error()
    out = (st.state, st.steps, st.obs, b.evict(0).cpu().numpy())
    b.close()
    return out


def test_concurrent_solo_launches_converge_like_alone():
    """On a stream of its own, a batch of solo lines (a fast real one, a fast
    complex one, a complex line of 16 points per thread that the persistent
    kernel keeps) and two larger instances runs the solo kernel beside the
    persistent launches.  Every instance stops at the same step with the same
    state and observables as alone, and the ground-state line converges."""
    cases = [make(1, (3000, 1, 1), IMAG, seed=80), make(1, (2048, 1, 1), REAL, seed=81),
             make(1, (12000, 1, 1), REAL, seed=82), make(3, (40, 44, 36), IMAG, seed=83),
             make(2, (120, 96, 1), IMAG, seed=84)]
    tol = [1e-6, 0.0, 0.0, 1e-6, 1e-6]
    cap = [60000, 700, 700, 3000, 3000]
    alone = [_run_alone(c, t, m) for c, t, m in zip(cases, tol, cap)]
    b = sscn.Batch(len(cases), stream=torch.cuda.Stream())
    for i, (c, t, m) in enumerate(zip(cases, tol, cap)):
        b.admit(i, c[0], c[1], mu_tol=t, max_steps=m)
    done = {}
    while len(done) < len(cases):
        b.step(20)
        st = b.poll(wait=True)
        for i, x in enumerate(st):
            if i not in done and x.state != sscn.SLOT_RUNNING:
                done[i] = (x.state, x.steps, x.obs, b.evict(i).cpu().numpy())
    assert not b.error()
    b.close()
    for i in range(len(cases)):
        a, m = alone[i], done[i]
        print(f"case {i} n={cases[i][0].n} mode={cases[i][0].mode}: state {m[0]} steps {m[1]}", flush=True)
        assert a[0] == m[0] and a[1] == m[1]
        assert a[2] == m[2]
        assert np.array_equal(a[3], m[3])
    assert done[0][0] == sscn.SLOT_CONVERGED


def test_many_solo_lines_beside_a_larger_instance():
    """More solo lines than the solo kernel may take CUs for (over half the
    persistent grid) keep running inside the persistent kernel; the results
    are those of each line alone."""
    lines = [make(1, (64 + 8 * (i % 5), 1, 1), IMAG, seed=90 + i) for i in range(200)]
    big = make(3, (24, 20, 28), IMAG, seed=89)
    b = sscn.Batch(len(lines) + 1, stream=torch.cuda.Stream())
    b.admit(len(lines), big[0], big[1], mu_tol=0.0, max_steps=40)
    for i, c in enumerate(lines):
        b.admit(i, c[0], c[1], mu_tol=0.0, max_steps=40)
    b.step(40)
    st = b.poll(wait=True)
    assert not b.error()
    assert all(x.state == sscn.SLOT_DONE and x.steps == 40 for x in st)
    got = [b.evict(i).cpu().numpy() for i in (0, 7, 199)]
    b.close()
    for i, g in zip((0, 7, 199), got):
        a = _run_alone(lines[i], 0.0, 40)
        assert np.array_equal(a[3], g)
        assert_fp32_close(g, oracle.run(oprob(lines[i][0]), lines[i][1], 40).psi, 1, f"line {i}")


@pytest.mark.parametrize("n,mode,sigma", [(3000, IMAG, 0.1), (9912, IMAG, 2.0), (3000, REAL, 0.5), (96, IMAG, 0.025),
                                          (300, IMAG, 0.025)])
def test_solo_lines_with_deeper_scans(n, mode, sigma):
    """Solo lines whose row scans need several Kogge-Stone steps (larger
    sigma, or few points per thread) are bitwise the same in the solo kernel
    (alone) as in the persistent kernel (beside a 3D instance)."""
    h = 0.1
    p = Problem(1, (n, 1, 1), (h,), (1.0,), 5.0, sigma * 4 * h * h, mode, F32, 1 if mode == IMAG else 0, 10)
    psi0 = inputs.ho_gaussian(1, p.n, p.dx, p.omega, noise=1e-3, seed=7)
    if mode == REAL:
        psi0 = psi0.astype(np.complex128)
    alone = _run_alone((p, psi0), 0.0, 30)
    big = make(3, (24, 20, 28), IMAG, seed=8)
    b = sscn.Batch(2)
    b.admit(1, big[0], big[1], mu_tol=0.0, max_steps=1 << 30)
    b.admit(0, p, psi0, mu_tol=0.0, max_steps=30)
    while True:
        b.step(1)
        st = b.poll(wait=True)[0]
        if st.state != sscn.SLOT_RUNNING:
            break
    assert not b.error()
    mix = b.evict(0).cpu().numpy()
    b.close()
    assert alone[1] == st.steps == 30 and alone[2] == st.obs
    assert np.array_equal(alone[3], mix)
    assert_fp32_close(mix, oracle.run(oprob(p), psi0, 30).psi, 1, f"deep-scan n={p.n}")


def test_admit_waits_for_an_input_made_on_the_current_stream():
    """A device input produced on the caller's stream behind a long kernel is
    copied into the slot only once it is there (the batch runs on a stream
    of its own)."""
    p, psi0 = make(2, (48, 40, 1), IMAG, seed=3)
    want = np.asarray(psi0).reshape(p.shape).astype(np.float32)
    b = sscn.Batch(1, stream=torch.cuda.Stream())
    src = torch.from_numpy(want).cuda()
    big = torch.randn(4096, 4096, device="cuda")
    busy = big @ big
    dev = src + 0.0 * busy[:1, :1]  # ready only after the product
    b.admit(0, p, dev)
    got = b.psi[0].cpu().numpy()
    assert np.array_equal(got, want)
    b.step(5)
    b.stream.synchronize()
    ref = sscn.Batch(1)
    ref.admit(0, p, psi0)
    ref.step(5)
    torch.cuda.synchronize()
    assert np.array_equal(b.psi[0].cpu().numpy(), ref.psi[0].cpu().numpy())


def test_largest_mix_draws_match_the_oracle():
    """The largest instances of the 64-instance mix (seeded draws 0, 36 and
    61: a 1D line of 13042 points, 1015^2 and 159^3), admitted together with
    the same parameters as in the mix (imaginary time, dt = 0.1 dx^2, FP32),
    30 steps against the FP64 oracle."""
    cases = []
    for i in (0, 36, 61):
        d = inputs.batch_draw(i)
        h = d.dx[0]
        p = Problem(d.dim, d.n, d.dx[:d.dim], d.omega[:d.dim], d.g, 0.1 * h * h, IMAG, F32, 1, 10)
        cases.append((p, inputs.ho_gaussian(d.dim, d.n, d.dx, d.omega, noise=1e-3, seed=d.seed)))
    got, st = run_batch(cases, 30, stream=torch.cuda.Stream())
    for (p, psi0), g, s in zip(cases, got, st):
        assert s.state == sscn.SLOT_DONE and s.steps == 30
        ref = oracle.run(oprob(p), psi0, 30).psi
        assert_fp32_close(g, ref, p.dim, f"mix draw n={p.n}")
        orf = oracle.observe(oprob(p), ref)
        assert abs(s.obs.mu - orf.mu) <= 1e-5 * max(1.0, abs(orf.mu))
