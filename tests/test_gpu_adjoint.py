"""GPU exact adjoint and adjoint-state gradient against the FP64 oracle and finite differences."""
import numpy as np
import pytest

import oracle
from paper_1603_03971_amd import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _grid(shape, h=10.0, vmax=3000.0, sponge=6):
    from paper_1603_03971_amd.grid import Grid

    nz, ny, nx = shape
    return Grid(nx, ny, nz, h, Grid.stable_dt(4, h, vmax), sponge_width=sponge)


def test_adjoint_step_matches_oracle():
    import torch

    from paper_1603_03971_amd import _abi

    shape = (29, 34, 41)
    g = _grid(shape)
    v = synth.random_smooth_velocity(shape, seed=71, vmin=1500, vmax=3000)
    ma, mb = synth.random_field(shape, 72), synth.random_field(shape, 73)
    kap = g.kappa_from_velocity(v)
    out, work = g.field(), g.field()
    _abi.rtm_adjoint_step(g.c, out, g.upload(ma), g.upload(mb), kap, work, torch.cuda.current_stream())
    torch.cuda.synchronize()
    sp = tuple(oracle.sponge_profile(n, 6) for n in (shape[2], shape[1], shape[0]))
    k64 = oracle.kappa_field(v.astype(np.float32), g.dt, g.h)
    ref = oracle.adjoint_step(ma.astype(np.float32), mb.astype(np.float32), k64, sp)
    e = oracle.rel_l2(g.download(out), ref)
    _say(f"adjoint step rel-L2 {e:.2e}")
    assert e <= 1e-6


@pytest.mark.parametrize("radius", [4, 2])
def test_adjoint_tiled_equals_per_cell_path_bitwise(radius):
    """The tiled adjoint kernel forms kappa g mu_a from two loads per ring element; the per-cell path
    (unaligned layouts) reads it from `work`, written by a separate pass.  Every tile option and z
    chunking, in place (mu_out = mu_b) or not, gives the per-cell path's bits, with NaN in the ghost
    cells of mu_a, mu_b and kappa (the tiled kernel must zero what lies outside the owned block), and
    no ghost cell of the output is written."""
    import torch

    from paper_1603_03971_amd import _abi
    from paper_1603_03971_amd.grid import Grid

    shape = (37, 45, 70)      # nz, ny, nx: ragged tiles in x and y, several z chunks
    nz, ny, nx = shape
    g = Grid(nx, ny, nz, 10.0, Grid.stable_dt(radius, 10.0, 3000.0), radius=radius, sponge_width=6)
    v = synth.random_smooth_velocity(shape, seed=74, vmin=1500, vmax=3000)
    ma, mb = synth.random_field(shape, 75), synth.random_field(shape, 76)
    st = torch.cuda.current_stream()
    nan = float("nan")

    def poisoned(src):
        f = g.field(fill=nan)
        g.owned(f).copy_(src)
        return f

    kap = poisoned(g.owned(g.kappa_from_velocity(v)))
    mu_a = poisoned(torch.from_numpy(ma.astype(np.float32)).cuda())
    mu_b_host = torch.from_numpy(mb.astype(np.float32)).cuda()
    work = g.field()

    def run(in_place):
        mu_b = poisoned(mu_b_host)
        out = mu_b if in_place else g.field(fill=nan)
        _abi.rtm_adjoint_step(g.c, out, mu_a, mu_b, kap, work, st)
        torch.cuda.synchronize()
        pad = g.padded(out).clone()
        pad[radius:radius + nz, radius:radius + ny, radius:radius + nx] = 0.0
        if not in_place:
            assert int(torch.isnan(pad).sum()) == pad.numel() - nx * ny * nz, "a ghost cell was written"
        return g.download(out)

    iv = _abi.rtm_get_option(_abi.RTM_OPT_INTERIOR_VARIANT)
    wv = _abi.rtm_get_option(_abi.RTM_OPT_WHOLE_VARIANT)
    try:
        _abi.rtm_set_option(_abi.RTM_OPT_INTERIOR_VARIANT, 3)          # the per-cell path
        ref = run(False)
        _abi.rtm_set_option(_abi.RTM_OPT_INTERIOR_VARIANT, iv)
        assert np.all(np.isfinite(ref)) and np.any(ref != 0)
        for var in (0, 1, 2, 4, 5):
            _abi.rtm_set_option(_abi.RTM_OPT_WHOLE_VARIANT, var)
            for zc in (0, 5):
                _abi.rtm_set_option(_abi.RTM_OPT_ZCHUNK, zc)
                for in_place in (False, True):
                    _say(f"adjoint tiled R={radius} variant {var} zchunk {zc} in place {in_place}")
                    assert np.array_equal(run(in_place), ref), (var, zc, in_place)
    finally:
        _abi.rtm_set_option(_abi.RTM_OPT_INTERIOR_VARIANT, iv)
        _abi.rtm_set_option(_abi.RTM_OPT_WHOLE_VARIANT, wv)
        _abi.rtm_set_option(_abi.RTM_OPT_ZCHUNK, 0)


@pytest.mark.parametrize("n,nchunks", [(1, 1024), (1000, 7), (4_915_201, 1024)])
def test_misfit_residual_chunks(n, nchunks):
    """Chunked residual and misfit: resid exact, the FP64 misfit within rounding of the numpy sum,
    the same bits on every call."""
    import torch

    from paper_1603_03971_amd import _abi

    rng = np.random.default_rng(n)
    d = rng.standard_normal(n).astype(np.float32)
    obs = rng.standard_normal(n).astype(np.float32)
    dt, ot = torch.from_numpy(d).cuda(), torch.from_numpy(obs).cuda()
    part = torch.full((nchunks,), float("nan"), dtype=torch.float64, device="cuda")
    vals = []
    for _ in range(2):
        resid = torch.empty_like(dt)
        mis = torch.zeros(1, dtype=torch.float64, device="cuda")
        _abi.rtm_misfit_residual_chunks(dt, ot, resid, n, part, nchunks, mis, torch.cuda.current_stream())
        torch.cuda.synchronize()
        vals.append(float(mis.item()))
    r = d - obs
    assert np.array_equal(resid.cpu().numpy(), r)
    want = 0.5 * float(np.sum(r.astype(np.float64) ** 2))
    assert abs(vals[0] - want) <= 1e-12 * want
    assert vals[0] == vals[1]


def test_gradient_kernel_matches_oracle():
    import torch

    from paper_1603_03971_amd import _abi

    shape = (21, 30, 37)
    g = _grid(shape)
    u, mu, g0 = (synth.random_field(shape, s) for s in (81, 82, 83))
    grad = g.upload(g0)
    _abi.rtm_gradient_accumulate(g.c, grad, g.upload(u), g.upload(mu), torch.cuda.current_stream())
    torch.cuda.synchronize()
    sp = [oracle.sponge_profile(n, 6) for n in (shape[2], shape[1], shape[0])]
    gg = sp[2][:, None, None] * sp[1][None, :, None] * sp[0][None, None, :]
    u32, mu32 = u.astype(np.float32).astype(np.float64), mu.astype(np.float32).astype(np.float64)
    ref = g0.astype(np.float32) + gg * mu32 * oracle.laplacian(u32, 4)
    assert oracle.rel_l2(g.download(grad), ref) <= 1e-6


def test_scaled_adjoint_kernels():
    """The pieces of the scaled recursion: grad += w L u against the oracle's Laplacian; the receiver
    factors kappa g and 1 / (kappa g) bit for bit against the same FP32 products on the host (0 for an
    index that is not an owned cell); the weighted gather; dJ/dv = 2 G / v bit for bit."""
    import torch

    from paper_1603_03971_amd import _abi

    shape = (21, 30, 37)
    nz, ny, nx = shape
    g = _grid(shape)
    st = torch.cuda.current_stream()
    u, w, g0 = (synth.random_field(shape, s) for s in (84, 85, 86))
    grad = g.upload(g0)
    _abi.rtm_gradient_accumulate_scaled(g.c, grad, g.upload(u), g.upload(w), st)
    torch.cuda.synchronize()
    u32, w32 = u.astype(np.float32).astype(np.float64), w.astype(np.float32).astype(np.float64)
    ref = g0.astype(np.float32) + w32 * oracle.laplacian(u32, 4)
    assert oracle.rel_l2(g.download(grad), ref) <= 1e-6

    v = synth.random_smooth_velocity(shape, seed=87, vmin=1500, vmax=3000).astype(np.float32)
    kap = g.kappa_from_velocity(v)
    cells = np.array([(0, 0, 0), (36, 29, 20), (5, 7, 3), (18, 1, 19), (2, 28, 10)])
    idx = np.concatenate([g.index(cells), [0, g.total - 1]])           # two indices of ghost cells
    idx_d = torch.from_numpy(idx).cuda()
    kg = torch.full((len(idx),), float("nan"), device="cuda")
    inv = torch.full((len(idx),), float("nan"), device="cuda")
    _abi.rtm_scaled_adjoint_factors(g.c, kap, idx_d, len(idx), kg, inv, st)
    gx, gy, gz = (t.cpu().numpy() for t in (g.gx, g.gy, g.gz))
    kh = g.download(kap)
    want = np.array([kh[k, j, i] * ((gx[i] * gy[j]) * gz[k]) for i, j, k in cells], dtype=np.float32)
    got_kg, got_inv = kg.cpu().numpy(), inv.cpu().numpy()
    np.testing.assert_array_equal(got_kg[:len(cells)], want)
    np.testing.assert_array_equal(got_inv[:len(cells)], (np.float32(1.0) / want).astype(np.float32))
    assert np.all(got_kg[len(cells):] == 0) and np.all(got_inv[len(cells):] == 0)

    field = g.upload(w)
    out = torch.empty(len(cells), device="cuda")
    wt = torch.from_numpy(np.linspace(-2, 3, len(cells)).astype(np.float32)).cuda()
    _abi.rtm_record_weighted(g.c, field, idx_d, wt, out, len(cells), st)
    wh = w.astype(np.float32)
    np.testing.assert_array_equal(out.cpu().numpy(),
                                  wt.cpu().numpy() * np.array([wh[k, j, i] for i, j, k in cells], dtype=np.float32))

    G = g.upload(g0)
    gv = torch.empty(shape, device="cuda")
    _abi.rtm_velocity_gradient_scaled(g.c, gv, G, torch.from_numpy(v).cuda(), st)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(gv.cpu().numpy(), (np.float32(2.0) * g0.astype(np.float32)) / v)


def _problem(shape, nsteps, nshots, seed, C=50, nrec_stride=3, true_model=None, adjoint="scaled"):
    """Shots at seeded surface positions with receivers every `nrec_stride` cells at depth 4."""
    import torch

    from paper_1603_03971_amd.adjoint import MisfitProblem, Shot

    nz, ny, nx = shape
    g = _grid(shape)
    src = synth.random_positions(nshots, nx, ny, k=5, seed=seed, margin=8)
    rec = synth.surface_receivers(nx, ny, k=4, stride=nrec_stride)
    wav = g.ricker(nsteps, 20.0)
    v_true = true_model if true_model is not None else synth.random_smooth_velocity(shape, seed + 1, 1800, 2800)
    shots = []
    for s in src:
        w = g.injection_weights([v_true[s[2], s[1], s[0]]])
        shots.append(Shot([s], w, rec))
    prob = MisfitProblem(g, nsteps, wav, shots, checkpoint_every=C, adjoint=adjoint)
    kt = g.kappa_from_velocity(v_true)
    for sh in shots:
        sh.observed = prob.model(kt, sh)
    torch.cuda.synchronize()
    return prob, v_true, src, rec, wav


@pytest.mark.parametrize("adjoint", ["scaled", "direct"])
def test_dot_product_fp32(adjoint):
    """<F x, y> = <x, F^T y> for the GPU forward map (source series -> traces) and its transpose, run
    as the scaled recursion (the forward kernel on w = kappa g mu) and as the direct one."""
    import torch

    shape = (40, 36, 44)
    nsteps = 90
    prob, v, src, rec, _ = _problem(shape, nsteps, 1, seed=90, C=25, adjoint=adjoint)
    g = prob.g
    kap = prob.kappa(torch.from_numpy(v.astype(np.float32)).cuda())
    shot = prob.shots[0]
    rng = np.random.default_rng(91)
    x = rng.standard_normal((nsteps, 1)).astype(np.float32)
    y = torch.from_numpy(rng.standard_normal((nsteps, len(rec))).astype(np.float32)).cuda()
    fx = prob.model(kap, shot, amp=x)
    misfit = torch.zeros(1, dtype=torch.float64, device="cuda")
    shot.observed = torch.zeros_like(fx)
    ckpt, _ = prob.forward(kap, shot, misfit)
    ysrc = torch.zeros((nsteps, 1), dtype=torch.float32, device="cuda")
    grad = g.field()
    prob.backward(kap, shot, ckpt, y, grad, y_src=ysrc)
    torch.cuda.synchronize()
    fty = ysrc.cpu().numpy().astype(np.float64) * shot.src_w.astype(np.float64)
    lhs = float(np.sum(fx.cpu().numpy().astype(np.float64) * y.cpu().numpy()))
    rhs = float(np.sum(x.astype(np.float64) * fty))
    rel = abs(lhs - rhs) / max(abs(lhs), abs(rhs))
    _say(f"dot product ({adjoint}): <Fx,y> {lhs:.9e} <x,F^T y> {rhs:.9e} rel {rel:.2e}")
    assert rel <= 1e-5


@pytest.fixture(scope="module")
def grad64():
    import torch

    shape = (64, 64, 64)
    nsteps, nshots = 200, 2
    prob, v_true, src, rec, wav = _problem(shape, nsteps, nshots, seed=100, C=50)
    v0 = synth.smooth(v_true, 6.0)
    _say("grad64: gpu gradient")
    J, gv = prob.misfit_and_gradient(torch.from_numpy(v0.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    return prob, v_true, v0, src, rec, wav, J, gv.cpu().numpy()


def test_gradient_matches_oracle_64(grad64):
    prob, v_true, v0, src, rec, wav, J, gv = grad64
    g = prob.g
    h, dt = g.h, g.dt
    shape = v0.shape
    sp = tuple(oracle.sponge_profile(n, 6) for n in (shape[2], shape[1], shape[0]))
    dto = oracle.stable_dt(4, h, 3000.0)
    assert abs(dto - dt) < 1e-15
    kt = oracle.kappa_field(v_true.astype(np.float32), dt, h)
    k0 = oracle.kappa_field(v0.astype(np.float32), dt, h)
    amp = oracle.ricker(np.arange(prob.nsteps) * dt, 20.0)[:, None]
    Jo, gk = 0.0, np.zeros(shape)
    for s in src:
        w = oracle.injection_weight([v_true[s[2], s[1], s[0]]], dt, h)
        obs = oracle.forward(kt, sp, prob.nsteps, src_ijk=[s], src_w=w, src_amp=amp, rec_ijk=rec, nthreads=16)["traces"]
        j, gks = oracle.gradient_kappa(k0, sp, prob.nsteps, src_ijk=[s], src_w=w, src_amp=amp, rec_ijk=rec,
                                       observed=obs, nthreads=16)
        Jo += j
        gk += gks
    gvo = 2.0 * v0.astype(np.float32) * (dt / h) ** 2 * gk
    e = oracle.rel_l2(gv, gvo)
    _say(f"grad64: J gpu {J:.9e} oracle {Jo:.9e}; dJ/dv rel-L2 {e:.2e}")
    assert abs(J - Jo) <= 1e-3 * Jo
    assert e <= 1e-3


def test_gradient_matches_finite_differences(grad64):
    """Central differences of the GPU misfit for a 1e-3 relative velocity perturbation on 64 seeded
    cells of the illuminated zone (between the surface shots and depth 30).  The difference is formed
    from the traces in FP64, J+ - J- = 1/2 <d+ - d-, d+ + d- - 2 d_obs>, so the two large misfits
    never cancel in floating point; what remains is the FP32 noise of the traces.  Each cell is
    perturbed with the sign of its gradient so that the 64 contributions add up instead of partly
    cancelling (any direction is a valid finite-difference direction)."""
    import torch

    prob, v_true, v0, src, rec, wav, J, gv = grad64
    rng = np.random.default_rng(110)
    cells = np.stack([rng.integers(8, 56, 64), rng.integers(8, 56, 64), rng.integers(6, 30, 64)], axis=1)
    sign = np.sign(gv[cells[:, 2], cells[:, 1], cells[:, 0]]).astype(np.float64)
    sign[sign == 0] = 1.0
    e = np.zeros_like(v0)
    e[cells[:, 2], cells[:, 1], cells[:, 0]] = sign * 1e-3 * v0[cells[:, 2], cells[:, 1], cells[:, 0]]
    fd = 0.0
    kp = prob.kappa(torch.from_numpy((v0 + e).astype(np.float32)).cuda())
    km = prob.kappa(torch.from_numpy((v0 - e).astype(np.float32)).cuda())
    for sh in prob.shots:
        dp = prob.model(kp, sh).cpu().numpy().astype(np.float64)
        dm = prob.model(km, sh).cpu().numpy().astype(np.float64)
        obs = sh.observed.cpu().numpy().astype(np.float64)
        fd += 0.5 * float(np.sum((dp - dm) * (dp + dm - 2.0 * obs)))
    fd /= 2.0
    an = float(np.sum(gv.astype(np.float64) * e))
    rel = abs(fd - an) / abs(an)
    _say(f"FD: {fd:.6e} adjoint {an:.6e} rel {rel:.2e}")
    assert rel <= 1e-2


def test_scaled_and_direct_gradients_agree():
    """The scaled recursion (forward kernel on w) and the direct one (rtm_adjoint_step on mu) give the
    same misfit bits (same forward runs) and the same gradient to FP32 rounding."""
    import torch

    shape = (36, 32, 40)
    a = _problem(shape, 80, 2, seed=140, C=20, adjoint="scaled")
    b = _problem(shape, 80, 2, seed=140, C=20, adjoint="direct")
    v0 = torch.from_numpy(synth.smooth(a[1], 4.0).astype(np.float32)).cuda()
    Ja, ga = a[0].misfit_and_gradient(v0)
    Jb, gb = b[0].misfit_and_gradient(v0)
    e = oracle.rel_l2(ga.cpu().numpy(), gb.cpu().numpy())
    _say(f"scaled vs direct gradient rel-L2 {e:.2e}")
    assert Ja == Jb
    assert e <= 1e-5


def test_checkpoint_interval_invariance():
    """The recomputation schedule does not change the result: the gradient is bitwise the same for
    any checkpoint interval."""
    import torch

    shape = (30, 28, 33)
    a = _problem(shape, 70, 1, seed=120, C=7)
    b = _problem(shape, 70, 1, seed=120, C=1000)
    v0 = synth.smooth(a[1], 4.0)
    va = torch.from_numpy(v0.astype(np.float32)).cuda()
    Ja, ga = a[0].misfit_and_gradient(va)
    Jb, gb = b[0].misfit_and_gradient(va)
    assert Ja == Jb
    assert torch.equal(ga, gb)


def test_autograd_function():
    import torch

    from paper_1603_03971_amd.adjoint import velocity_misfit

    shape = (30, 28, 33)
    prob, v_true, *_ = _problem(shape, 60, 2, seed=130, C=20)
    v = torch.from_numpy(synth.smooth(v_true, 4.0).astype(np.float32)).cuda().requires_grad_(True)
    J = velocity_misfit(v, prob)
    J.backward()
    J2, gv = prob.misfit_and_gradient(v.detach())
    assert abs(float(J) - J2) <= 1e-12 * J2
    assert torch.equal(v.grad, gv)
    assert float(J) > 0 and float(v.grad.abs().max()) > 0
