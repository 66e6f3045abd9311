"""GPU parity: libkxg (HIP, through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.

Tolerances (max-norm relative error of the result, ||x - x_ref||_inf /
||x_ref||_inf): 1e-10 for FP64 steps, 1e-5 for the FP32 contraction, 1e-3
for the 16-bit split contractions; kinematic decisions (which (i,n,m) survive
the cuts) must agree exactly.
"""
import numpy as np
import pytest

import oracle
from paper_2607_00755_amd import inputs, kxg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {kxg.F64: 1e-10, kxg.F32: 1e-5, kxg.BF16X3: 1e-3, kxg.F16X3: 1e-3, kxg.F16X2: 1e-3}
ALL = (kxg.F64, kxg.F32, kxg.BF16X3, kxg.F16X3, kxg.F16X2)
SIXTEEN = (kxg.BF16X3, kxg.F16X3, kxg.F16X2)


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def pointwise(a, b, floor=1e-6):
    """Largest pointwise relative error |a_i - b_i| / |b_i| over the bins
    with |b_i| >= floor * max |b| (the tail-sensitive second metric)."""
    a, b = np.asarray(a), np.asarray(b)
    sel = np.abs(b) >= floor * np.max(np.abs(b))
    return float(np.max(np.abs(a[sel] - b[sel]) / np.abs(b[sel])))


def golden_rk4():
    """The oracle's states after 2000 RK4 steps for 16 seeded solves of each
    N=256 batch workload (written by tests/golden/make_rk4_n256.py)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rk4_n256_2000.npz")
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def batch(p, B, seed=7):
    solves = inputs.draw_solves(B, seed=seed)
    return np.stack([s.f0(p) for s in solves])


def oracle_C(op, f0, project):
    out = []
    for b in range(f0.shape[0]):
        C, _, _ = op.collision(f0[b])
        out.append(op.project(f0[b], C)[0] if project else C)
    return np.stack(out)


def closed_form_condition(p, op, mass=1.0):
    """kappa = (p_i + p~ + p_n + p_m) / |S| per (i, n, m): how much the
    cancellation in the closed-form angular sum S (App. B, the isotropic
    double integral in closed form) amplifies rounding; 1 where A is zero."""
    K = op.grid.K
    Kt = np.maximum((K[None, :, None] + K[None, None, :]) - K[:, None, None], 0.0)
    p1, p2 = p[:, None, None], np.sqrt(Kt * (Kt + 2 * mass))
    p3, p4 = p[None, :, None], p[None, None, :]
    S = (abs(p1 - p2 - p3 - p4) + abs(p1 - p2 + p3 + p4) + abs(p1 + p2 - p3 + p4)
         + abs(p1 + p2 + p3 - p4) - abs(p1 - p2 - p3 + p4) - abs(p1 - p2 + p3 - p4)
         - abs(p1 + p2 - p3 - p4) - (p1 + p2 + p3 + p4))
    return np.where(op.A != 0.0, (p1 + p2 + p3 + p4) / np.where(S != 0, np.abs(S), 1.0), 1.0)


# ---------------------------------------------------------------- kernel build
@pytest.mark.parametrize("n,quad,pmin,pmax", [(20, kxg.QUAD_GL, 1e-2, 5.0),
                                              (37, kxg.QUAD_GL, 1e-3, 20.0),
                                              (48, kxg.QUAD_EXACT, 1e-3, 20.0),
                                              (4, kxg.QUAD_GL, 0.1, 3.0)])
def test_kernel_tensors_match_oracle(dev, n, quad, pmin, pmax):
    p = inputs.log_grid(n, pmin, pmax)
    k = kxg.Kernel(p, precs=(kxg.F64,), quad=quad)
    A, R = k.export()
    op = oracle.Operator(p, quad=quad)
    assert np.array_equal(A != 0.0, op.A != 0.0)          # identical cut decisions
    # element by element to 1e-12 relative (a floor of 1e-15 of the largest
    # weight for elements that are themselves that small); the closed form
    # adds the rounding of its signed sum S of eight |p1 +- p2 +- p3 +- p4|
    # terms, at most ~48 eps sum(p) absolute, i.e. 48 eps kappa relative with
    # kappa = sum(p) / |S| (up to 1e4 next to the kinematic boundary)
    tolA = 1e-12 * np.abs(op.A) + 1e-15 * np.max(op.A)
    if quad == kxg.QUAD_EXACT:
        tolA = tolA + 64 * np.finfo(float).eps * closed_form_condition(p, op) * np.abs(op.A)
    nz = op.A != 0.0
    worst = float(np.max(np.abs(A - op.A)[nz] / np.abs(op.A[nz])))
    print("n=%d quad=%d: worst relative element error %.3e, worst error / bound %.3f"
          % (n, quad, worst, float(np.max(np.abs(A - op.A) / tolA))), flush=True)
    assert np.all(np.abs(A - op.A) <= tolA), worst
    assert np.array_equal(R != 0.0, op.R != 0.0)
    assert rel(R, op.R) <= 1e-12
    g = k.grid()
    assert np.array_equal(g["E"], op.grid.E) and np.array_equal(g["K"], op.grid.K)
    assert np.allclose(g["h"], op.grid.h, rtol=1e-15, atol=0)


def test_kernel_tensors_width_override(dev):
    p = inputs.log_grid(24, 1e-2, 10.0)
    dp = p * np.log(p[1] / p[0])
    k = kxg.Kernel(p, precs=(kxg.F64,), dp=dp)
    A, R = k.export()
    op = oracle.Operator(p, dp=dp)
    assert rel(A, op.A) <= 1e-12 and rel(R, op.R) <= 1e-12


# ---------------------------------------------------------------- evaluation
@pytest.mark.parametrize("n", [32, 37, 100])
@pytest.mark.parametrize("B", [1, 3, 7])
def test_eval_f64(dev, n, B):
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = batch(p, B)
    k = kxg.Kernel(p, precs=(kxg.F64,), b_cap=8)
    op = oracle.Operator(p)
    f = torch.tensor(f0, device=dev)
    for project in (False, True):
        C, d = k.eval(f, prec=kxg.F64, project=project)
        torch.cuda.synchronize()
        ref = oracle_C(op, f0, project)
        assert rel(C.cpu().numpy(), ref) <= TOL[kxg.F64]
    d = d.cpu().numpy()
    for b in range(B):
        Craw, _, _ = op.collision(f0[b])
        _, od = op.project(f0[b], Craw)
        assert np.allclose(d[b, [0, 1]], od[[0, 1]], rtol=1e-7, atol=1e-12 * abs(od[0]))
        assert np.allclose(d[b, [2, 3, 6, 7]], od[[2, 3, 6, 7]], rtol=1e-8, atol=1e-14)
        assert abs(d[b, 4]) < 1e-12 and abs(d[b, 5]) < 1e-12
        assert d[b, 10] == 0.0
        assert abs(d[b, 8] - op.gamma0(f0[b])) <= 1e-12 * d[b, 8]


@pytest.mark.parametrize("B,cap", [(1, 4), (3, 4), (4, 4), (1, 130), (5, 130), (33, 130),
                                   (70, 130), (130, 130)])
def test_eval_f32(dev, B, cap):
    """cap <= 4: single-distribution stream kernel; otherwise the MFMA GEMM."""
    n = 64
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = batch(p, B, seed=3)
    k = kxg.Kernel(p, precs=(kxg.F32,), b_cap=cap)
    op = oracle.Operator(p)
    C, _ = k.eval(torch.tensor(f0, device=dev), prec=kxg.F32, project=True)
    torch.cuda.synchronize()
    assert rel(C.cpu().numpy(), oracle_C(op, f0, True)) <= TOL[kxg.F32]


@pytest.mark.parametrize("n", [37, 100])
@pytest.mark.parametrize("B", [1, 3])
def test_eval_f32_single_ragged(dev, n, B):
    """FP32 single-distribution handles stream the packed kept blocks in
    FP32; grids whose last i-block and last 16-blocks are partial."""
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = batch(p, B, seed=13)
    k = kxg.Kernel(p, precs=(kxg.F32,), b_cap=4)
    op = oracle.Operator(p)
    for project in (False, True):
        C, _ = k.eval(torch.tensor(f0, device=dev), prec=kxg.F32, project=project)
        torch.cuda.synchronize()
        assert rel(C.cpu().numpy(), oracle_C(op, f0, project)) <= TOL[kxg.F32]


@pytest.mark.parametrize("prec", SIXTEEN)
@pytest.mark.parametrize("B,n", [(3, 40), (40, 64), (130, 100)])
def test_eval_16bit(dev, prec, B, n):
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = batch(p, B, seed=5)
    k = kxg.Kernel(p, precs=(prec,), b_cap=130)
    op = oracle.Operator(p)
    C, _ = k.eval(torch.tensor(f0, device=dev), prec=prec, project=True)
    torch.cuda.synchronize()
    assert rel(C.cpu().numpy(), oracle_C(op, f0, True)) <= TOL[prec]


def test_eval_full_size_batched_f32_sampled(dev):
    """N=256, B=512 FP32 GEMM (the batched workload) on sampled rows; the
    plain FP64 stream over the packed blocks (the single-distribution path)
    on the same rows, one by one and as a group of four."""
    w = inputs.batched_fp32_n256()
    p = w.grid()
    f0 = w.f0()
    k = kxg.Kernel(p, precs=(kxg.F32, kxg.BF16X3), b_cap=512)
    f = torch.tensor(f0, device=dev)
    C, _ = k.eval(f, prec=kxg.F32, project=True)
    C16, _ = k.eval(f, prec=kxg.BF16X3, project=True)
    rows = (0, 1, 127, 128, 300, 511)
    C64 = [k.eval(f[b:b + 1].contiguous(), prec=kxg.F64, project=True)[0] for b in rows]
    C64g, _ = k.eval(f[list(rows[:4])].contiguous(), prec=kxg.F64, project=True)
    torch.cuda.synchronize()
    C, C16 = C.cpu().numpy(), C16.cpu().numpy()
    C64 = [c.cpu().numpy()[0] for c in C64]
    C64g = C64g.cpu().numpy()
    op = oracle.Operator(p)
    for j, b in enumerate(rows):
        ref = oracle_C(op, f0[b:b + 1], True)[0]
        assert rel(C[b], ref) <= TOL[kxg.F32], b
        assert rel(C16[b], ref) <= TOL[kxg.BF16X3], b
        assert rel(C64[j], ref) <= TOL[kxg.F64], b
        if j < 4:
            assert np.array_equal(C64g[j], C64[j]), b


def test_batch_invariance_bitwise(dev):
    n = 64
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = batch(p, 200, seed=9)
    k = kxg.Kernel(p, precs=(kxg.F32, kxg.BF16X3), b_cap=200)
    for prec in (kxg.F32, kxg.BF16X3):
        full, _ = k.eval(torch.tensor(f0, device=dev), prec=prec)
        full = full.cpu().numpy()
        for sel in ([5, 17, 190, 3, 0, 44], list(range(40, 110)), [150] * 9):
            part, _ = k.eval(torch.tensor(f0[sel], device=dev), prec=prec)
            assert np.array_equal(part.cpu().numpy(), full[sel]), (prec, len(sel))


def test_gemm_width_invariance_bitwise(dev):
    """The FP32 GEMM runs a call of B rows with one, two or four 32-row batch
    blocks per wave, whichever keeps the busiest CU shortest for that B.  At
    N=256 on a b_cap=512 handle the calls below take all three widths; every
    row must come out bitwise the same as in the full batch."""
    w = inputs.batched_fp32_n256(512)
    p = w.grid()
    f0 = torch.tensor(w.f0(), device=dev)
    k = kxg.Kernel(p, precs=(kxg.F32,), b_cap=512)
    units = k.stats()["gemm_units"]

    def width(B):                      # the launch rule, restated
        best, tb = 4, None
        for wd in (4, 2, 1):
            wgs = units * -(-B // (32 * wd))
            t = wd * -(-wgs // 256)
            if tb is None or t < tb or (t == tb and wgs <= 512):
                best, tb = wd, t
        return best

    sels = [list(range(512)), list(range(0, 512, 2)), list(range(100, 196)), [511, 3, 250],
            list(range(17, 317))]
    assert {width(len(s)) for s in sels} == {1, 2, 4}, [(len(s), width(len(s))) for s in sels]
    full, _ = k.eval(f0, prec=kxg.F32)
    full = full.cpu().numpy()
    for sel in sels:
        part, _ = k.eval(f0[sel].contiguous(), prec=kxg.F32)
        assert np.array_equal(part.cpu().numpy(), full[sel]), (len(sel), width(len(sel)))


@pytest.mark.parametrize("n", [40, 200])
def test_single_distribution_stream_bitwise(dev, n):
    """The FP64 stream path evaluates one distribution (one per pass) and
    three (grouped passes); the result and the diagnostics of a row must
    not depend on that, over many calls in a row."""
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = batch(p, 3, seed=31)
    k = kxg.Kernel(p, precs=(kxg.F64,), b_cap=8)
    f3 = torch.tensor(f0, device=dev)
    for rnd in range(25):
        scale = 1.0 + 0.1 * rnd
        C3, d3 = k.eval(f3 * scale, prec=kxg.F64)
        b = rnd % 3
        C1, d1 = k.eval((f3[b:b + 1] * scale).contiguous(), prec=kxg.F64)
        torch.cuda.synchronize()
        assert torch.equal(C1[0], C3[b]), (rnd, b)
        assert torch.equal(d1[0], d3[b]), (rnd, b)
    C, _ = k.eval(f3[:1].contiguous(), prec=kxg.F64)
    assert rel(C.cpu().numpy(), oracle_C(oracle.Operator(p), f0[:1], True)) <= TOL[kxg.F64]


def test_single_slot_fp64_stepper_matches_batched_slot(dev):
    """A one-slot FP64 stepper follows the same trajectory, bit for bit, as
    the same solve in a three-slot stepper."""
    n = 48
    p = inputs.log_grid(n, 1e-2, 10.0)
    f0 = batch(p, 3, seed=5)
    k = kxg.Kernel(p, precs=(kxg.F64,), b_cap=4)
    one = kxg.Stepper(k, kind=kxg.RK4, prec=kxg.F64, b_cap=1)
    three = kxg.Stepper(k, kind=kxg.RK4, prec=kxg.F64, b_cap=3)
    one.set(0, torch.tensor(f0[1], device=dev), lam=1.0, t_end=1e9, h_i=1.0)
    for b in range(3):
        three.set(b, torch.tensor(f0[b], device=dev), lam=1.0, t_end=1e9, h_i=1.0)
    side = torch.cuda.Stream()
    one.advance(12, stream=side)
    three.advance(12, stream=side)
    side.synchronize()
    a = one.get(0, stream=side)
    c = three.get(1, stream=side)
    side.synchronize()
    assert torch.equal(a, c)


def test_edge_cases(dev):
    p = inputs.log_grid(16, 1e-2, 5.0)
    k = kxg.Kernel(p, precs=(kxg.F64, kxg.F32), b_cap=9)
    z = torch.zeros((9, 16), dtype=torch.float64, device=dev)
    for prec in (kxg.F64, kxg.F32):
        C, d = k.eval(z, prec=prec)
        torch.cuda.synchronize()
        assert torch.all(C == 0) and torch.all(d[:, 10] == 0)
    with pytest.raises(kxg.KxgError) as ei:
        k.eval(z, prec=kxg.BF16X3)
    assert ei.value.status == kxg.EUNSUPPORTED
    with pytest.raises(kxg.KxgError) as ei:
        k.eval(torch.zeros((10, 16), dtype=torch.float64, device=dev))
    assert ei.value.status == kxg.EINVAL
    with pytest.raises(kxg.KxgError) as ei:         # an empty batch
        k.eval(torch.zeros((0, 16), dtype=torch.float64, device=dev))
    assert ei.value.status == kxg.EINVAL
    bad = torch.tensor(batch(p, 9), device=dev)
    bad[4, 3] = float("nan")
    bad[6, 2] = -1.0
    C, d = k.eval(bad, prec=kxg.F32)
    torch.cuda.synchronize()
    st = d[:, 10].cpu().numpy()
    assert st[4] == 1 + 4 and st[6] == 2 and np.all(st[[0, 1, 2, 3, 5, 7, 8]] == 0)
    assert torch.isfinite(C[[0, 1, 2, 3, 5, 7, 8]]).all()


def test_largest_grid(dev):
    """n = 1024, the largest grid (32 i-blocks: every word of the packed
    slot counts in use): the FP32 and BF16x3 GEMMs agree with the FP64
    stream to their tolerances, the projection conserves number and energy,
    and n = 1025 is refused."""
    n, B = 1024, 6
    p = inputs.log_grid(n, 1e-3, 20.0)
    f = torch.tensor(batch(p, B, seed=23), device=dev)
    k = kxg.Kernel(p, precs=(kxg.F64, kxg.F32, kxg.BF16X3), b_cap=8)
    C64, _ = k.eval(f, prec=kxg.F64)
    C32, _ = k.eval(f, prec=kxg.F32)
    C16, _ = k.eval(f, prec=kxg.BF16X3)
    torch.cuda.synchronize()
    ref = C64.cpu().numpy()
    for C, prec in ((C32, kxg.F32), (C16, kxg.BF16X3)):
        got = C.cpu().numpy()
        for b in range(B):
            assert rel(got[b], ref[b]) <= TOL[prec], (prec, b)
    g = k.grid()
    h, E = g["h"], g["E"]
    for b in range(B):
        assert abs(np.sum(h * ref[b])) <= 1e-12 * np.sum(h * np.abs(ref[b]))
        assert abs(np.sum(h * E * ref[b])) <= 1e-12 * np.sum(h * E * np.abs(ref[b]))
    with pytest.raises(kxg.KxgError) as ei:
        kxg.Kernel(inputs.log_grid(n + 1, 1e-3, 20.0), precs=(kxg.F64,), b_cap=1)
    assert ei.value.status == kxg.EINVAL


def test_moments(dev):
    p = inputs.log_grid(50, 1e-3, 20.0)
    f0 = batch(p, 5)
    k = kxg.Kernel(p, precs=(kxg.F64,), b_cap=5)
    op = oracle.Operator(p)
    m = k.moments(torch.tensor(f0, device=dev)).cpu().numpy()
    ref = np.stack([op.moments(x) for x in f0])
    assert rel(m, ref) <= 1e-13


# ---------------------------------------------------------------- steppers
def test_rk4_single_fp64_n32(dev):
    w = inputs.single_fp64_n32()
    p = w.grid()
    f0 = w.f0()[0]
    op = oracle.Operator(p)
    dt = 0.1 / op.gamma0(f0)
    ref, traj = op.rk4(f0, 1.0, dt, 100, traj=True)
    k = kxg.Kernel(p, precs=(kxg.F64,), b_cap=1)
    st = kxg.Stepper(k, kind=kxg.RK4, prec=kxg.F64, b_cap=1)
    ft = torch.tensor(f0, device=dev)
    st.set(0, ft, lam=1.0, t_end=1e9, dt=dt, h_i=1.0, max_steps=100)
    mom = [k.moments(ft).cpu().numpy()[0]]
    for s in range(100):
        st.advance(1)
        mom.append(k.moments(st.get(0)).cpu().numpy()[0])
    got = st.get(0).cpu().numpy()
    assert rel(got, ref) <= 1e-10
    q = st.query()[0]
    assert q["steps"] == 100 and q["status"] == 2       # stopped by the step cap, t_end not reached
    mom = np.array(mom)
    assert np.max(np.abs(np.diff(mom[:, 0])) / mom[:-1, 0]) <= 1e-12
    assert np.max(np.abs(np.diff(mom[:, 1])) / mom[:-1, 1]) <= 1e-12
    assert np.all(np.diff(mom[:, 2]) >= -1e-12 * np.abs(mom[:-1, 2]))


@pytest.mark.parametrize("prec,n", [(kxg.F64, 64), (kxg.F32, 64), (kxg.F32, 128)])
def test_heun_expansion_replay(dev, prec, n):
    """Replay the oracle's accepted step sequence (FP64 adaptive Heun in
    u = ln a with drift) on the GPU and compare the state at the end."""
    p = inputs.log_grid(n, 1e-3, 20.0)
    s = inputs.draw_solves(1, lam_range=(1e-2, 1e2), seed=21)[0]
    f0 = s.f0(p)
    op = oracle.Operator(p)
    Hi = op.gamma0(f0)
    r = op.heun(f0 * p ** 3, s.lam, Hi, 0.3, 1e-3, expansion=True, max_steps=120)
    nsteps = len(r["dt"])
    assert nsteps >= 20
    k = kxg.Kernel(p, precs=(prec,), b_cap=1)
    st = kxg.Stepper(k, kind=kxg.HEUN, prec=prec, b_cap=1, expansion=kxg.EXP_RADIATION,
                     adapt=False)
    st.set(0, torch.tensor(f0, device=dev), lam=s.lam, t_end=10.0, dt=r["dt"][0], h_i=Hi)
    for j in range(nsteps):
        st.set_dt([r["dt"][j]])
        st.advance(1)
    got = st.get(0).cpu().numpy()
    u = r["u"][-1] + r["dt"][-1]
    ref = r["x"] / (np.exp(3 * u) * p ** 3)
    assert rel(got, ref) <= TOL[prec]
    q = st.query()[0]
    assert q["steps"] == nsteps and abs(q["t"] - u) <= 1e-14
    assert abs(q["outflow"] - r["outflow"]) <= TOL[prec] * abs(r["outflow"]) + 1e-300


def test_heun_drift_fp32_n128_full_replay(dev):
    """The N=128 FP32 evolution with radiation-era drift at full length: the
    oracle's FP64 adaptive Heun takes 1e4 accepted steps in u = ln a, the
    device replays them in FP32 (one step per call, dt from the oracle);
    state, time and outflow at the end within 1e-5."""
    w = inputs.single_fp32_n128()
    p = w.grid()
    s = w.solves[0]
    f0 = w.f0()[0]
    op = oracle.Operator(p)
    Hi = op.gamma0(f0)
    r = op.heun(f0 * p ** 3, s.lam, Hi, 0.5 * np.log(2e4), 1e-3, expansion=True, max_steps=10000)
    nsteps = len(r["dt"])
    assert nsteps == 10000
    k = kxg.Kernel(p, precs=(kxg.F32,), b_cap=1)
    st = kxg.Stepper(k, kind=kxg.HEUN, prec=kxg.F32, b_cap=1, expansion=kxg.EXP_RADIATION,
                     adapt=False)
    st.set(0, torch.tensor(f0, device=dev), lam=s.lam, t_end=10.0, dt=r["dt"][0], h_i=Hi)
    for j in range(nsteps):
        st.set_dt([r["dt"][j]])
        st.advance(1)
    got = st.get(0).cpu().numpy()
    u = r["u"][-1] + r["dt"][-1]
    ref = r["x"] / (np.exp(3 * u) * p ** 3)
    assert rel(got, ref) <= TOL[kxg.F32], rel(got, ref)
    q = st.query()[0]
    assert q["steps"] == nsteps and abs(q["t"] - u) <= 1e-12 * u
    assert abs(q["outflow"] - r["outflow"]) <= TOL[kxg.F32] * abs(r["outflow"]) + 1e-300


def test_heun_adaptive_fp64_free_run(dev):
    n = 48
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = inputs.bump_pair(p, 0.2, 2.0, 1.0, 1.0, 0.3, 0.3)
    op = oracle.Operator(p)
    Hi = op.gamma0(f0)
    r = op.heun(f0 * p ** 3, 3.0, Hi, 0.1, 1e-3, expansion=True, max_steps=5000)
    k = kxg.Kernel(p, precs=(kxg.F64,), b_cap=1)
    st = kxg.Stepper(k, kind=kxg.HEUN, prec=kxg.F64, b_cap=1, expansion=kxg.EXP_RADIATION,
                     rtol=1e-6, atol_rel=1e-12)
    st.set(0, torch.tensor(f0, device=dev), lam=3.0, t_end=0.1, dt=1e-3, h_i=Hi)
    for _ in range(200):
        st.advance(50)
        if st.query()[0]["status"] != 0:
            break
    q = st.query()[0]
    assert q["status"] == 1 and abs(q["t"] - 0.1) < 1e-14
    assert abs(q["steps"] - len(r["dt"])) <= 2
    ref = r["x"] / (np.exp(3 * 0.1) * p ** 3)
    assert rel(st.get(0).cpu().numpy(), ref) <= 1e-6


def test_checkpoint_resume_bitwise(dev):
    p = inputs.log_grid(40, 1e-3, 20.0)
    f0 = batch(p, 2, seed=4)
    k = kxg.Kernel(p, precs=(kxg.F32,), b_cap=2)
    mk = lambda: kxg.Stepper(k, kind=kxg.HEUN, prec=kxg.F32, b_cap=2,
                             expansion=kxg.EXP_RADIATION)
    a = mk()
    for b in range(2):
        a.set(b, torch.tensor(f0[b], device=dev), lam=5.0, t_end=0.5, dt=1e-3, h_i=0.0)
    a.advance(30)
    blob = a.save(1)
    a.advance(40)
    straight = a.get(1).cpu().numpy()
    bst = mk()
    bst.load(1, blob)
    bst.advance(40)
    assert np.array_equal(bst.get(1).cpu().numpy(), straight)
    assert bst.query()[1]["steps"] == a.query()[1]["steps"]


def test_failed_slot_does_not_poison_batch(dev):
    p = inputs.log_grid(32, 1e-2, 10.0)
    f0 = batch(p, 3, seed=8)
    k = kxg.Kernel(p, precs=(kxg.F64,), b_cap=3)
    op = oracle.Operator(p)
    st = kxg.Stepper(k, kind=kxg.RK4, prec=kxg.F64, b_cap=3)
    bad = f0[1].copy()
    bad[5] = np.nan
    dts = [0.1 / op.gamma0(f0[b]) for b in range(3)]
    for b, x in enumerate((f0[0], bad, f0[2])):
        st.set(b, torch.tensor(x, device=dev), lam=1.0, t_end=1e9, dt=dts[b], h_i=1.0)
    st.advance(5)
    q = st.query()
    assert q[1]["status"] == -1 and q[0]["status"] == 0 and q[2]["status"] == 0
    for b in (0, 2):
        ref = op.rk4(f0[b], 1.0, dts[b], 5)
        assert rel(st.get(b).cpu().numpy(), ref) <= 1e-10
    st.release(1)
    assert st.query()[1]["status"] == -3


@pytest.mark.parametrize("kind,prec,B", [(kxg.RK4, kxg.F32, 40), (kxg.HEUN, kxg.F64, 3),
                                          (kxg.HEUN, kxg.BF16X3, 20)])
def test_graph_replay_matches_eager(dev, kind, prec, B):
    """Advancing on a side stream replays a captured HIP graph; every replay
    must match the same iteration launched eagerly on the default stream."""
    p = inputs.log_grid(48, 1e-3, 20.0)
    f0 = batch(p, B, seed=12)
    k = kxg.Kernel(p, precs=(prec,), b_cap=64)
    exp = kxg.EXP_RADIATION if kind == kxg.HEUN else kxg.EXP_NONE
    steppers = [kxg.Stepper(k, kind=kind, prec=prec, b_cap=64, expansion=exp) for _ in range(2)]
    side = torch.cuda.Stream()
    for st in steppers:
        for b in range(B):
            st.set(b, torch.tensor(f0[b], device=dev), lam=2.0, t_end=1e3, h_i=0.0)
    torch.cuda.synchronize()
    out = [torch.empty(48, dtype=torch.float64, device=dev) for _ in range(2)]
    for rnd in range(6):
        steppers[0].advance(1, stream=side)          # graph replay
        side.synchronize()
        steppers[1].advance(1)                       # eager launches
        torch.cuda.synchronize()
        _ = (torch.ones(1000, device=dev) * rnd).sum().item()   # unrelated eager work
        for b in (0, B - 1):
            steppers[0].get(b, out=out[0], stream=side)
            side.synchronize()
            steppers[1].get(b, out=out[1])
            torch.cuda.synchronize()
            assert torch.equal(out[0], out[1]), (rnd, b)
        q0, q1 = steppers[0].query(stream=side), steppers[1].query()
        assert [x["steps"] for x in q0[:B]] == [x["steps"] for x in q1[:B]]


@pytest.mark.parametrize("kind,prec", [(kxg.RK4, kxg.F32), (kxg.HEUN, kxg.F64)])
def test_multi_iteration_graph_matches_eager(dev, kind, prec):
    """Long advances on a side stream replay a graph of eight captured
    iterations (then single ones for the rest); the state after 8 + 11
    iterations must equal that of the same iterations launched eagerly."""
    B = 24
    p = inputs.log_grid(40, 1e-3, 20.0)
    f0 = batch(p, B, seed=21)
    k = kxg.Kernel(p, precs=(prec,), b_cap=32)
    exp = kxg.EXP_RADIATION if kind == kxg.HEUN else kxg.EXP_NONE
    steppers = [kxg.Stepper(k, kind=kind, prec=prec, b_cap=32, expansion=exp) for _ in range(2)]
    side = torch.cuda.Stream()
    for st in steppers:
        for b in range(B):
            st.set(b, torch.tensor(f0[b], device=dev), lam=1.5, t_end=1e3, h_i=0.0)
    torch.cuda.synchronize()
    out = [torch.empty(40, dtype=torch.float64, device=dev) for _ in range(2)]
    for n_iter in (8, 11):
        steppers[0].advance(n_iter, stream=side)
        side.synchronize()
        steppers[1].advance(n_iter)
        torch.cuda.synchronize()
        for b in range(B):
            steppers[0].get(b, out=out[0], stream=side)
            side.synchronize()
            steppers[1].get(b, out=out[1])
            torch.cuda.synchronize()
            assert torch.equal(out[0], out[1]), (n_iter, b)
        q0, q1 = steppers[0].query(stream=side), steppers[1].query()
        assert [x["steps"] for x in q0[:B]] == [x["steps"] for x in q1[:B]]
        assert [x["t"] for x in q0[:B]] == [x["t"] for x in q1[:B]]


def test_graphs_kept_per_batch_bucket_match_eager(dev):
    """The stepper keeps the graphs of every batch bucket (16 slots) it has
    replayed: as slots are filled, retired and refilled, the batch moves
    between buckets and back (16 -> 48 -> 32 -> 48 -> 16), replaying graphs
    captured earlier. Every phase must match the same slot history launched
    eagerly on the default stream, bit for bit."""
    n, cap = 40, 64
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = batch(p, cap, seed=33)
    k = kxg.Kernel(p, precs=(kxg.F32,), b_cap=cap)
    steppers = [kxg.Stepper(k, kind=kxg.HEUN, prec=kxg.F32, b_cap=cap,
                            expansion=kxg.EXP_RADIATION) for _ in range(2)]
    side = torch.cuda.Stream()
    streams = (side, None)

    def each(fn):
        for st, s in zip(steppers, streams):
            fn(st, s)
            if s is not None:
                s.synchronize()
        torch.cuda.synchronize()

    def fill(lo, hi, lam):
        each(lambda st, s: [st.set(b, torch.tensor(f0[b], device=dev), lam=lam, t_end=1e3,
                                   h_i=0.0, stream=s) for b in range(lo, hi)])

    def drop(lo, hi):
        each(lambda st, s: [st.release(b, stream=s) for b in range(lo, hi)])

    out = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(2)]
    used = set()
    phases = [("fill", 0, 10, 2.0), ("fill", 10, 40, 3.0), ("drop", 20, 40, 0.0),
              ("fill", 30, 45, 1.5), ("drop", 10, 45, 0.0)]
    for ph, (what, lo, hi, lam) in enumerate(phases):
        if what == "fill":
            fill(lo, hi, lam)
            used |= set(range(lo, hi))
        else:
            drop(lo, hi)
            used -= set(range(lo, hi))
        each(lambda st, s: st.advance(9, stream=s))
        for b in sorted(used):
            steppers[0].get(b, out=out[0], stream=side)
            side.synchronize()
            steppers[1].get(b, out=out[1])
            torch.cuda.synchronize()
            assert torch.equal(out[0], out[1]), (ph, b)
        q0, q1 = steppers[0].query(stream=side), steppers[1].query()
        assert [q0[b]["steps"] for b in sorted(used)] == [q1[b]["steps"] for b in sorted(used)]
        assert sum(q0[b]["steps"] for b in sorted(used)) > 0


@pytest.mark.parametrize("prec", ALL)
def test_eval_without_diagnostics_same_C(dev, prec):
    """With no diagnostics buffer the operator output is bitwise the same."""
    p = inputs.log_grid(64, 1e-3, 20.0)
    f = torch.tensor(batch(p, 5, seed=4), device=dev)
    k = kxg.Kernel(p, precs=(prec,), b_cap=8)
    C1, d1 = k.eval(f, prec=prec)
    C2, d2 = k.eval(f, prec=prec, diagnostics=False)
    torch.cuda.synchronize()
    assert d2 is None and d1 is not None
    assert torch.equal(C1, C2)


@pytest.mark.parametrize("prec", [kxg.BF16X3, kxg.F16X3])
def test_split_ablations_lose_accuracy(dev, prec):
    """The hi+lo split is what brings the 16-bit contraction to 1e-3: with
    the A split dropped (F2 split only) or no split at all, the error
    against the oracle is orders of magnitude larger; the ablations are
    refused at FP64/FP32 and together."""
    n, B = 64, 40
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = batch(p, B, seed=17)
    k = kxg.Kernel(p, precs=(kxg.F32, prec), b_cap=64)
    ref = oracle_C(oracle.Operator(p), f0, True)
    f = torch.tensor(f0, device=dev)
    err = {}
    for split in (3, 2, 1):
        C, _ = k.eval(f, prec=prec, split=split)
        torch.cuda.synchronize()
        err[split] = rel(C.cpu().numpy(), ref)
    assert err[3] <= TOL[prec], err
    assert err[2] > 20 * err[3] and err[1] > 20 * err[3], err
    with pytest.raises(kxg.KxgError):
        k.eval(f, prec=kxg.F32, split=2)
    out = torch.empty_like(f)
    st = kxg.lib().kxg_eval(k._h, int(prec), f.data_ptr(), B, out.data_ptr(),
                            kxg.SPLIT_F_ONLY | kxg.SPLIT_NONE, None, None)
    assert st == kxg.EINVAL


@pytest.mark.parametrize("prec", SIXTEEN)
def test_eval_16bit_large_batch_lds_path(dev, prec):
    """The LDS-shared GEMM at a large ragged batch (600 -> 1024 rows) and a
    ragged i-tile (n = 80: 3 blocks of 32 in a group of 4)."""
    n = 80
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = batch(p, 600, seed=14)
    k = kxg.Kernel(p, precs=(prec,), b_cap=600)
    f = torch.tensor(f0, device=dev)
    C, _ = k.eval(f, prec=prec, project=True)
    sub, _ = k.eval(f[:520].contiguous(), prec=prec, project=True)
    torch.cuda.synchronize()
    C, sub = C.cpu().numpy(), sub.cpu().numpy()
    op = oracle.Operator(p)
    for b in (0, 31, 32, 255, 511, 512, 599):
        assert rel(C[b], oracle_C(op, f0[b:b + 1], True)[0]) <= TOL[prec], b
    assert np.array_equal(sub, C[:520])


@pytest.mark.parametrize("prec", (kxg.F16X2, kxg.F16X3))
@pytest.mark.parametrize("n", [48, 112, 176])
def test_eval_16bit_lds_path_grid_sizes(dev, prec, n):
    """The LDS-shared GEMM over grid sizes whose work units differ in length
    (every remainder of the prefetch rotation and of the (kb, mb) pairs
    occurs among them): sampled rows of a ragged 520-row batch against the
    oracle."""
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = batch(p, 520, seed=21 + n)
    k = kxg.Kernel(p, precs=(prec,), b_cap=520)
    C, _ = k.eval(torch.tensor(f0, device=dev), prec=prec, project=True)
    torch.cuda.synchronize()
    C = C.cpu().numpy()
    op = oracle.Operator(p)
    rows = (0, 63, 64, 300, 511, 519)
    ref = oracle_C(op, f0[list(rows)], True)
    for j, b in enumerate(rows):
        assert rel(C[b], ref[j]) <= TOL[prec], (n, b)


# ---------------------------------------------------------------- exact forms
@pytest.mark.parametrize("n,B", [(37, 1), (48, 3)])
@pytest.mark.parametrize("log_interp,eta", [(True, 0), (False, 1), (False, -1), (True, 1),
                                            (True, -1)])
def test_exact_forms_match_oracle_direct(dev, n, B, log_interp, eta):
    """Paper's log interpolation (eq. app_log_interp) and Bose-Einstein /
    Fermi-Dirac factors (eq. Lambda_quantum) against the oracle's direct
    per-(i,n,m) evaluation with the product form of Lambda."""
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = batch(p, B, seed=23) * 0.3          # occupations below one
    k = kxg.Kernel(p, precs=(kxg.F64, kxg.F32), b_cap=4, brackets=True)
    f = torch.tensor(f0, device=dev)
    interp = oracle.LOG if log_interp else oracle.LIN
    ref = np.stack([oracle.direct(p, f0[b], interp=interp, eta=eta)[0] for b in range(B)])
    for prec in (kxg.F64, kxg.F32):
        C, d = k.eval(f, prec=prec, project=False, log_interp=log_interp, eta=eta)
        torch.cuda.synchronize()
        assert rel(C.cpu().numpy(), ref) <= TOL[prec], (prec, rel(C.cpu().numpy(), ref))
    op = oracle.Operator(p)
    Cp, _ = k.eval(f, prec=kxg.F64, project=True, log_interp=log_interp, eta=eta)
    torch.cuda.synchronize()
    refp = np.stack([op.project(f0[b], ref[b])[0] for b in range(B)])
    assert rel(Cp.cpu().numpy(), refp) <= TOL[kxg.F64]


@pytest.mark.parametrize("n,B", [(96, 1), (96, 3), (128, 3)])
@pytest.mark.parametrize("log_interp,eta", [(True, 0), (False, 1), (True, 1), (True, -1),
                                            (False, -1)])
def test_exact_forms_multi_split_match_oracle_direct(dev, n, B, log_interp, eta):
    """The exact forms at grid sizes where the stream runs several K splits
    per row (4 at n = 96, 8 at n = 128), with chunks that start inside a row,
    and the epilogue adds them: FP64 and FP32, raw and projected, against the
    oracle's direct per-(i,n,m) sum (App. B eq. app_log_interp, eq.
    Lambda_quantum)."""
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = batch(p, B, seed=29) * 0.3
    k = kxg.Kernel(p, precs=(kxg.F64, kxg.F32), b_cap=4, brackets=True)
    f = torch.tensor(f0, device=dev)
    interp = oracle.LOG if log_interp else oracle.LIN
    ref = np.stack([oracle.direct(p, f0[b], interp=interp, eta=eta)[0] for b in range(B)])
    op = oracle.Operator(p)
    refp = np.stack([op.project(f0[b], ref[b])[0] for b in range(B)])
    for prec in (kxg.F64, kxg.F32):
        for project, r in ((False, ref), (True, refp)):
            C, _ = k.eval(f, prec=prec, project=project, log_interp=log_interp, eta=eta)
            torch.cuda.synchronize()
            e = rel(C.cpu().numpy(), r)
            assert e <= TOL[prec], (prec, project, e)


def test_exact_form_log_interp_keeps_maxwell_boltzmann(dev):
    p = inputs.log_grid(40, 1e-2, 10.0)
    f0 = inputs.maxwell_boltzmann(p, 1.0, 0.4, 2.0)[None, :]
    k = kxg.Kernel(p, precs=(kxg.F64,), brackets=True)
    C, d = k.eval(torch.tensor(f0, device=dev), project=False, log_interp=True)
    torch.cuda.synchronize()
    gain_max = d[0, 9].item()
    assert torch.max(torch.abs(C)).item() <= 1e-13 * gain_max


def test_exact_form_needs_brackets(dev):
    p = inputs.log_grid(16, 1e-2, 5.0)
    k = kxg.Kernel(p, precs=(kxg.F64, kxg.BF16X3), b_cap=2)
    f = torch.ones((1, 16), dtype=torch.float64, device=dev)
    with pytest.raises(kxg.KxgError) as ei:
        k.eval(f, log_interp=True)
    assert ei.value.status == kxg.EUNSUPPORTED
    kb = kxg.Kernel(p, precs=(kxg.F64, kxg.BF16X3), b_cap=2, brackets=True)
    with pytest.raises(kxg.KxgError) as ei:
        kb.eval(f, prec=kxg.BF16X3, eta=1)
    assert ei.value.status == kxg.EUNSUPPORTED


# ---------------------------------------------------------------- workloads
def test_batched_fp32_rk4_subsample(dev):
    """N=256, B=512 FP32 RK4 on the device; 16 seeded solves of the batch
    against the FP64 oracle after 20 steps (dt = 0.1 / (lambda Gamma0))."""
    w = inputs.batched_fp32_n256(512)
    p = w.grid()
    f0 = w.f0()
    k = kxg.Kernel(p, precs=(kxg.F32,), b_cap=512)
    st = kxg.Stepper(k, kind=kxg.RK4, prec=kxg.F32, b_cap=512)
    ft = torch.tensor(f0, device=dev)
    for b, s in enumerate(w.solves):
        st.set(b, ft[b], lam=s.lam, t_end=1e30, h_i=1.0)
    st.advance(20)
    torch.cuda.synchronize()
    op = oracle.Operator(p)
    for b in np.linspace(0, 511, 16).astype(int):
        s = w.solves[b]
        dt = 0.1 / (s.lam * op.gamma0(f0[b]))
        ref = op.rk4(f0[b], s.lam, dt, 20)
        assert rel(st.get(b).cpu().numpy(), ref) <= TOL[kxg.F32], b


def test_batched_fp32_rk4_2000_steps_subsample(dev):
    """The full batched FP32 run (N=256, B=512, 2000 RK4 steps as graph
    replays on a side stream): 16 seeded solves within 1e-5 of the FP64
    oracle at the end, f and the number/energy moments."""
    w = inputs.batched_fp32_n256(512)
    p = w.grid()
    f0 = w.f0()
    gold = golden_rk4()
    assert int(gold["steps"]) == 2000
    k = kxg.Kernel(p, precs=(kxg.F32,), b_cap=512)
    st = kxg.Stepper(k, kind=kxg.RK4, prec=kxg.F32, b_cap=512)
    ft = torch.tensor(f0, device=dev)
    for b, s in enumerate(w.solves):
        st.set(b, ft[b], lam=s.lam, t_end=1e30, h_i=1.0)
    torch.cuda.synchronize()               # the sets ran on the default stream
    side = torch.cuda.Stream()
    st.advance(2000, stream=side)
    side.synchronize()
    q = st.query(stream=side)
    picks = gold["batched_rows"]
    got = torch.stack([st.get(int(b), stream=side) for b in picks])
    side.synchronize()
    mg = k.moments(got).cpu().numpy()
    m0 = k.moments(ft[torch.as_tensor(picks, device=dev)].contiguous()).cpu().numpy()
    got = got.cpu().numpy()
    worst_pw = 0.0
    for j, b in enumerate(picks):
        assert q[b]["steps"] == 2000, (int(b), q[b]["steps"])
        ref = gold["batched_f"][j]
        assert rel(got[j], ref) <= TOL[kxg.F32], (int(b), rel(got[j], ref))
        worst_pw = max(worst_pw, pointwise(got[j], ref))
        mr = gold["batched_moments"][j]
        assert np.all(np.abs(mg[j, :2] - mr[:2]) <= TOL[kxg.F32] * np.abs(mr[:2])), int(b)
        # FP64 projection and state: number and energy keep their initial
        # values to 1e-12 per step over the whole run
        drift = np.abs(mg[j, :2] - m0[j, :2]) / np.abs(m0[j, :2])
        assert np.all(drift <= 2000 * 1e-12), (int(b), drift)
    print("fp32 2000 steps: pointwise rel. error (bins >= 1e-6 max f) %.3e" % worst_pw, flush=True)


@pytest.mark.parametrize("prec", SIXTEEN)
def test_mixed_precision_2000_steps_subsample(dev, prec):
    """N=256, B=4096 16-bit split contraction with FP64 projection and state:
    after 2000 RK4 steps, f and the number/energy moments of 16 seeded
    solves within 1e-3 of the FP64 oracle; moments drift <= 1e-12 per step
    relative on the device."""
    w = inputs.mixed_n256(4096)
    p = w.grid()
    f0 = w.f0()
    gold = golden_rk4()
    assert int(gold["steps"]) == 2000
    k = kxg.Kernel(p, precs=(prec,), b_cap=4096)
    st = kxg.Stepper(k, kind=kxg.RK4, prec=prec, b_cap=4096)
    ft = torch.tensor(f0, device=dev)
    st.set_many(0, ft, lam=[s.lam for s in w.solves], t_end=1e30, h_i=1.0)
    torch.cuda.synchronize()               # the sets ran on the default stream
    picks = gold["mixed_rows"]
    out = torch.empty(256, dtype=torch.float64, device=dev)
    side = torch.cuda.Stream()             # graph replays, as the benchmark runs them
    m_prev = None
    for block in range(4):
        st.advance(1, stream=side)
        side.synchronize()
        fs = torch.stack([st.get(int(b), out=out).clone() for b in picks])
        m = k.moments(fs).cpu().numpy()
        if m_prev is not None:
            assert np.max(np.abs(m[:, :2] - m_prev[:, :2]) / np.abs(m_prev[:, :2])) <= 1e-12
        m_prev = m
    st.advance(2000 - 4, stream=side)
    side.synchronize()
    q = st.query()
    assert all(q[b]["steps"] == 2000 for b in picks), [(int(b), q[b]["steps"], q[b]["status"]) for b in picks]
    got = torch.stack([st.get(int(b), out=out).clone() for b in picks])
    mg = k.moments(got).cpu().numpy()
    m0 = k.moments(ft[torch.as_tensor(picks, device=dev)].contiguous()).cpu().numpy()
    got = got.cpu().numpy()
    worst_pw = worst = 0.0
    for j, b in enumerate(picks):
        ref = gold["mixed_f"][j]
        worst = max(worst, rel(got[j], ref))
        assert rel(got[j], ref) <= TOL[prec], (int(b), rel(got[j], ref))
        worst_pw = max(worst_pw, pointwise(got[j], ref))
        mr = gold["mixed_moments"][j]
        assert np.all(np.abs(mg[j, :2] - mr[:2]) <= TOL[prec] * np.abs(mr[:2])), int(b)
        drift = np.abs(mg[j, :2] - m0[j, :2]) / np.abs(m0[j, :2])
        assert np.all(drift <= 2000 * 1e-12), (int(b), drift)
    print("%s 2000 steps: max-norm rel. error %.3e, pointwise (bins >= 1e-6 max f) %.3e"
          % (kxg.PREC_NAMES[prec], worst, worst_pw), flush=True)


def test_expansion_conserves_comoving_number_on_device(dev):
    """Heun in ln a with drift (FP64): sum_i V_i g_i changes per accepted
    step only by the recorded outflow through p_min."""
    n = 64
    p = inputs.log_grid(n, 1e-3, 20.0)
    f0 = inputs.bump_pair(p, 0.2, 2.0, 1.0, 1.0, 0.3, 0.3)
    k = kxg.Kernel(p, precs=(kxg.F64,), b_cap=1)
    V = k.grid()["dp"] / p
    st = kxg.Stepper(k, kind=kxg.HEUN, prec=kxg.F64, b_cap=1, expansion=kxg.EXP_RADIATION)
    st.set(0, torch.tensor(f0, device=dev), lam=3.0, t_end=0.15, dt=1e-3, h_i=0.0)
    tot0 = float(np.sum(V * f0 * p ** 3))
    for _ in range(400):
        st.advance(25)
        q = st.query()[0]
        u = q["t"]
        g = st.get(0).cpu().numpy() * np.exp(3 * u) * p ** 3
        assert abs(np.sum(V * g) + q["outflow"] - tot0) <= 1e-12 * tot0 * max(q["steps"], 1)
        if q["status"] != 0:
            break
    assert q["status"] == 1


def test_peak_probe_is_plausible(dev):
    """The self-calibration reports rates below the datasheet peaks (FP32 and
    BF16 MFMA 157.3 and 2500 TFLOP/s, HBM 8000 GB/s) and not far under them."""
    pk = kxg.peak_probe()
    for key, peak in (("mfma_f32_tflops", 157.3), ("mfma_bf16_tflops", 2500.0), ("read_GBps", 8000.0),
                      ("copy_GBps", 8000.0)):
        assert 0.3 * peak < pk[key] < 1.1 * peak, (key, pk[key])


def test_zero_block_skipping_matches_oracle_tensor(dev):
    """The FP32 operand keeps exactly the (i-block, pair) blocks of the
    packed tensor that hold a non-zero weight (blocks of 32 rows i x 16 x 16
    (k, m), both orderings), counted here from the oracle's tensor."""
    for n in (40, 96):
        p = inputs.log_grid(n, 1e-3, 20.0)
        k = kxg.Kernel(p, precs=(kxg.F32,), b_cap=64)
        st = k.stats()
        A = oracle.Operator(p).A != 0.0
        nb, nib = (n + 15) // 16, (n + 31) // 32
        sym = A | A.transpose(0, 2, 1)
        kept = 0
        for ib in range(nib):
            for kb in range(nb):
                for mb in range(kb, nb):
                    kept += bool(sym[ib * 32:(ib + 1) * 32, kb * 16:(kb + 1) * 16,
                                     mb * 16:(mb + 1) * 16].any())
        assert st["packed_blocks"] == nib * nb * (nb + 1) // 2
        assert st["nonzero_blocks"] == kept < st["packed_blocks"]
