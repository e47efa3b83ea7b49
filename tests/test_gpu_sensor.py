"""The learned-sensor form on the GPU: features and TENO labels against the
oracle, the network's FP32 forward / backward and Adam against the FP64 MLP
oracle, the MFMA inference path, the routed flux in its two limits (all
cheap = the oracle's cheap flux everywhere; all full = the plain residual),
and a trained network's error and gain against the plain form."""
import numpy as np
import pytest

from oracle import mlp
from oracle import oracle as O
from paper_2007_14933_amd import inputs as I
from parity_util import flux_scale, say

pytestmark = pytest.mark.gpu


def iface_stencils(prob, U, d):
    """(n, 6, nc) stencils of direction d in the library's label order
    (x fastest over the interface grid, extent n_d + 1 along d)."""
    nd = prob.ndim
    E = [prob.n[e] + (1 if e == d else 0) if e < nd else 1 for e in range(3)]
    kk, jj, ii = np.meshgrid(np.arange(E[2]), np.arange(E[1]), np.arange(E[0]), indexing="ij")
    pos = [ii.ravel(), jj.ravel(), kk.ravel()]
    pos[d] = pos[d] - 1
    out = []
    for k in range(6):
        q = [pos[e].copy() for e in range(3)]
        q[d] = q[d] - 2 + k
        ix = [q[e] + (3 if e < nd else 0) for e in range(3)]
        out.append(U[:, ix[2], ix[1], ix[0]].T)
    return np.stack(out, axis=1)


def state_after(prob, nsteps):
    from parity_util import oracle_run
    U, _ = oracle_run(prob, nsteps)
    return O.apply_bc(prob, U)


def feature_sensitivity(prob, d, Uk, S, fo, draws=4, seed=3):
    """Largest change of the oracle's features when the stencil states are
    perturbed by about one ulp (relative 2.2e-16)."""
    rng = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(draws):
        f2, _ = O.features(prob, d, Uk * (1.0 + 2.2e-16 * rng.standard_normal(Uk.shape)), S)
        worst = max(worst, float(np.abs(f2 - fo).max()))
    return worst


@pytest.mark.parametrize("case", ["riemann2d_48", "smooth3d_10"])
def test_features_and_labels_match_oracle(case):
    import torch
    from paper_2007_14933_amd import sensor as SN
    from paper_2007_14933_amd.solver import Solver
    if case == "riemann2d_48":
        prob = I.riemann2d(48, 3)
        U = state_after(prob, 30)
    else:
        prob = I.smooth_random(3, (10, 9, 8), seed=2, amp=0.3).with_(bc=((I.PERIODIC,) * 2, (I.EXTRAPOLATE,) * 2,
                                                                     (I.PERIODIC,) * 2))
        U = O.apply_bc(prob, prob.U0.copy())
    say("[gpu sensor] labels", case)
    s = Solver(prob.with_(U0=U))
    f, l = SN.collect(s)
    f, l = f.cpu().numpy(), l.cpu().numpy()
    off = 0
    nbad = 0
    nnoise = 0
    for d in range(prob.ndim):
        st = iface_stencils(prob, U, d)
        for t in range(len(st)):
            S = np.eye(3)[d][: prob.ndim]
            fo, lo = O.features(prob, d, st[t], S)
            # FP64 features rounded to float32; where the stencil is uniform
            # to within rounding the indicators are rounding noise, so the
            # bar there is the oracle's own response to one-ulp relative
            # perturbations of the stencil states (margin 8)
            diff = np.abs(f[off + t] - fo).max()
            if diff > 1e-6:
                sens = feature_sensitivity(prob, d, st[t], S, fo)
                nnoise += 1
                assert diff <= 1e-6 + 8.0 * sens, (d, t, f[off + t], fo, sens)
            assert np.all(np.isfinite(f[off + t])) and f[off + t][:4].sum() <= 1.0 + 1e-6
            nbad += int(l[off + t] != lo)
        off += len(st)
    say("   interfaces %d, label disagreements %d, smooth fraction %.3f, features at rounding-noise level %d"
        % (off, nbad, l.mean(), nnoise))
    assert off == len(l) and nbad == 0
    del torch


def _mlp_data(n=3000, seed=5):
    rng = np.random.default_rng(seed)
    theta = mlp.bf16_round(mlp.init(seed) + 0.05 * rng.normal(size=mlp.NPARAM))
    X = np.concatenate([rng.dirichlet(np.ones(4), n), rng.uniform(0, 0.5, (n, 6))], axis=1).astype(np.float32)
    y = (rng.uniform(size=n) < 0.6).astype(np.uint8)
    return theta, X, y


def test_mlp_forward_backward_adam_match_oracle():
    import torch
    from paper_2007_14933_amd import sensor as SN
    say("[gpu sensor] mlp fwd/bwd/adam")
    theta, X, y = _mlp_data()
    tr = SN.Trainer()
    tr.w.copy_(torch.from_numpy(mlp.bf16_bits(theta).view(np.int16)).cuda())
    tr.master.copy_(torch.from_numpy(theta.astype(np.float32)).cuda())
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    z = tr.forward(Xd).cpu().numpy()
    zo, _ = mlp.forward(theta, X.astype(np.float64))
    assert np.abs(z - zo).max() <= 1e-5 * (1 + np.abs(zo).max())
    g, L = tr.grad_loss(Xd, yd)
    g = g.cpu().numpy()
    go = mlp.grad(theta, X.astype(np.float64), y)
    Lo = mlp.loss(theta, X.astype(np.float64), y)
    say("   max|dz| %.2e  max|dg|/max|g| %.2e  dloss %.2e" % (np.abs(z - zo).max(), np.abs(g - go).max() / np.abs(go).max(),
                                                           abs(float(L.item()) - Lo)))
    assert np.abs(g - go).max() <= 1e-5 * np.abs(go).max()
    assert abs(float(L.item()) - Lo) <= 1e-6 * abs(Lo)
    # one Adam step from zero moments
    tr.t = 0
    tr.step(Xd, yd, lr=1e-3)
    th1, _, _ = mlp.adam(theta, np.zeros(mlp.NPARAM), np.zeros(mlp.NPARAM), go, 1, lr=1e-3)
    m1 = tr.master.cpu().numpy()
    assert np.abs(m1 - th1).max() <= 2e-6 * max(1.0, np.abs(th1).max())
    assert np.array_equal(tr.w.cpu().numpy().view(np.uint16), mlp.bf16_bits(m1))


def test_mlp_mfma_inference_matches_oracle():
    import torch
    from paper_2007_14933_amd import sensor as SN
    say("[gpu sensor] mfma inference")
    theta, X, y = _mlp_data(n=5000, seed=9)
    tr = SN.Trainer()
    tr.w.copy_(torch.from_numpy(mlp.bf16_bits(theta).view(np.int16)).cuda())
    z = tr.forward(torch.from_numpy(X).cuda(), inference=True).cpu().numpy()
    zo, _ = mlp.forward(theta, X.astype(np.float64), round_activations=True)
    err = np.abs(z - zo)
    say("   max|dz| %.3e  median %.3e  sign agreement %.5f" % (err.max(), np.median(err), np.mean((z >= 0) == (zo >= 0))))
    assert np.median(err) <= 1e-3 * (1 + np.median(np.abs(zo)))
    assert err.max() <= 5e-2 * (1 + np.abs(zo).max())
    assert np.mean((z >= 0) == (zo >= 0)) >= 0.995


def const_net(b3):
    theta = np.zeros(mlp.NPARAM)
    theta[-1] = b3
    return mlp.bf16_bits(theta)


def oracle_cheap_residual(prob, U):
    S, J = O.metrics(prob)
    nd = prob.ndim
    R = np.zeros(O.int_shape(prob))
    Ji = O.interior(prob, J[None])[0]
    for d in range(nd):
        st = iface_stencils(prob, U, d)
        F = np.stack([O.cheap_flux(prob, d, st[t], np.eye(3)[d][:nd]) for t in range(len(st))])
        E = [prob.n[e] + (1 if e == d else 0) if e < nd else 1 for e in range(3)]
        F = F.reshape(E[2], E[1], E[0], nd + 2)
        ax = 2 - d
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[ax] = slice(1, None)
        lo[ax] = slice(0, -1)
        dF = np.moveaxis(F[tuple(hi)] - F[tuple(lo)], -1, 0)
        # separable uniform meshes: J |S_d| = 1 / h_d
        h = float(prob.coords1d[d][1] - prob.coords1d[d][0])
        R -= dF / h
    return R, S, J


@pytest.mark.parametrize("mixed", [0, 1])
def test_routed_limits(mixed):
    """All interfaces routed cheap: the oracle's cheap flux everywhere (FP32
    deviations in the precision form); all routed full: the plain FP64
    residual (the routed forms fall back to the FP64 full flux)."""
    from paper_2007_14933_amd.solver import Solver
    prob = I.riemann2d(40, 11)
    U = state_after(prob, 20)
    p2 = prob.with_(U0=U)
    say("[gpu sensor] routed limits, mixed =", mixed)
    s = Solver(p2, sensor=1, form=mixed)
    s.set_sensor(const_net(30.0), 0.5)
    Rg = s.residual().cpu().numpy()
    sm, tot = s.sensor_stats()
    assert sm == tot
    Rc, S, J = oracle_cheap_residual(p2, U)
    sc = flux_scale(p2, U, J, S)
    err = np.abs(Rg - Rc).max(axis=(1, 2, 3)) / sc
    say("   all-cheap residual |diff| / flux scale:", err)
    assert err.max() <= (1e-13 if not mixed else 2e-6)
    s2 = Solver(p2, sensor=1, form=mixed)
    s2.set_sensor(const_net(-30.0), 0.5)
    Rf = s2.residual().cpu().numpy()
    assert s2.sensor_stats()[0] == 0
    # the routed forms' full flux is the FP64 one in both precisions
    Rp = Solver(p2).residual().cpu().numpy()
    assert np.abs(Rf - Rp).max() <= 1e-13 * np.abs(Rp).max()


def jump_net():
    """Smooth unless one of the six log-jump features is sizeable:
    z = 4 - 40 relu(relu(sum of jumps))."""
    theta = np.zeros(mlp.NPARAM)
    for i in range(4, 10):
        theta[i * 32] = 1.0
    theta[352] = 1.0
    theta[1408] = -40.0
    theta[1440] = 4.0
    return mlp.bf16_bits(theta)


@pytest.mark.parametrize("dilate", [0, 1, 2])
def test_routing_dilation(dilate):
    """Sod's initial jump: the interfaces whose stencil sees the jump are
    routed full, and with dilation d also the d interfaces on each side;
    every other interface takes the cheap flux.  The residual matches the
    oracle's fluxes chosen the same way."""
    from paper_2007_14933_amd.solver import Solver
    prob = I.sod(80).with_(scheme=I.TENO5)
    U = O.apply_bc(prob, prob.U0.copy())
    say("[gpu sensor] dilation", dilate)
    s = Solver(prob.with_(U0=U), sensor=1)
    s.set_sensor(jump_net(), 0.5, dilate=dilate)
    Rg = s.residual().cpu().numpy()
    st = iface_stencils(prob, U, 0)
    smooth = np.array([O.features(prob, 0, st[t], [1.0])[0][4:].max() == 0.0 for t in range(len(st))])
    route = smooth.copy()
    for o in range(1, dilate + 1):
        route[o:] &= smooth[:-o]
        route[:-o] &= smooth[o:]
    F = np.stack([O.cheap_flux(prob, 0, st[t], [1.0]) if route[t] else O.iface_flux(prob, 0, st[t], [1.0])[0]
                  for t in range(len(st))])
    h = float(prob.coords1d[0][1] - prob.coords1d[0][0])
    Ro = -(F[1:] - F[:-1]).T / h
    S, J = O.metrics(prob)
    err = np.abs(Rg.reshape(Ro.shape) - Ro).max(axis=1) / flux_scale(prob, U, J, S)
    sm, tot = s.sensor_stats()
    say("   routed cheap %d of %d (oracle %d); residual |diff| / flux scale %s" % (sm, tot, int(smooth.sum()), err))
    assert sm == int(smooth.sum()) and (~route).sum() == 3 + 2 * dilate
    assert err.max() <= 1e-13


@pytest.mark.parametrize("case", ["riemann2d_48", "smooth3d_10"])
def test_routing_masks_match_oracle_decisions(case):
    """Every interface's routing decision of the sensor kernels (per interface
    along x, marching along y and z) equals the oracle's: oracle features,
    the FP64 network on bfloat16-rounded inputs and activations, P(smooth) >=
    threshold.  Interfaces whose oracle logit lies within 0.02 of the cut are
    excluded (the kernels' FP32 features and MFMA sums may round either way
    there); they must stay a small minority."""
    from paper_2007_14933_amd import sensor as SN
    from paper_2007_14933_amd.solver import Solver
    if case == "riemann2d_48":
        prob = I.riemann2d(48, 3)
        U = state_after(prob, 30)
    else:
        prob = I.smooth_random(3, (70, 9, 8), seed=2, amp=0.3)
        U = O.apply_bc(prob, prob.U0.copy())
    # scaled random weights: logits spread over tens of units; b3 puts the
    # cut near the median so that both classes occur
    w = SN.init_weights(4) * 3.0
    w[1440] = 3.2 if case == "riemann2d_48" else 15.4
    bits = SN.bf16_bits(w)
    theta = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    thr = 0.5
    s = Solver(prob.with_(U0=U), sensor=1)
    s.set_sensor(bits, thr, dilate=0)
    s.sensor_update()
    sm, tot = s.sensor_stats()
    zc = np.log(thr / (1 - thr))
    ntot = nclear = nsmooth = 0
    for d in range(prob.ndim):
        st = iface_stencils(prob, U, d)
        F = np.array([O.features(prob, d, st[t], np.eye(3)[d][:prob.ndim])[0] for t in range(len(st))])
        z, _ = mlp.forward(theta, F, round_activations=True)
        m = s.sensor_masks(d)
        assert m.shape == z.shape and set(np.unique(m)) <= {0, 1}
        clear = np.abs(z - zc) > 0.02
        want = z >= zc
        bad = np.flatnonzero(clear & (m.astype(bool) != want))
        say("[gpu sensor] %s dir %d: %d interfaces, %d away from the cut, %d routed (oracle %d), %d disagree"
            % (case, d, len(z), int(clear.sum()), int(m.sum()), int(want.sum()), len(bad)))
        assert len(bad) == 0, bad[:10]
        ntot += len(z)
        nclear += int(clear.sum())
        nsmooth += int(m.sum())
    assert tot == ntot and sm == nsmooth
    assert nclear >= 0.98 * ntot
    assert 0 < nsmooth < ntot  # both classes occur


@pytest.fixture(scope="module")
def trained_routing_run():
    """Train the network on method-made labels (small run), choose the
    routing (threshold, dilation) on held-out shock-vortex seeds, then run
    the measured shock-vortex field (seed 42, 256 x 128) routed and plain to
    its end time."""
    import torch
    from paper_2007_14933_amd import sensor as SN
    from paper_2007_14933_amd.solver import Solver
    say("[gpu sensor] train small network")
    torch.manual_seed(0)
    X, y = SN.generate(nprob=6, N=128, seed=300, log=say)
    Xv, yv = SN.generate(nprob=2, N=128, seed=1300, log=None)
    tr = SN.Trainer(seed=0)
    tr.fit(X, y, epochs=8, batch=512, log=say)
    zv = tr.forward(Xv, inference=True)
    _, rec = SN.pick_threshold(zv, yv)
    acc = float(((zv >= 0) == (yv == 1)).float().mean().item())
    say("   samples %d, held-out accuracy %.4f, smooth recall at 0.1%% false-smooth %.3f" % (len(y), acc, rec))
    thr, _, _, dil = SN.pick_threshold_by_error(tr.weights_bits(), SN.heldout_problems(256, 128, (1000, 1001)),
                                                 log=say)
    prob = I.shock_vortex(256, 128, seed=42)
    res = {}
    for name, kw in (("plain", {}), ("routed", {"sensor": 1})):
        s = Solver(prob, **kw)
        if kw:
            s.set_sensor(tr.weights_bits(), thr, dilate=dil)
        s.profile(True)
        s.run(10 ** 9, cfl=prob.cfl, t_end=prob.t_end)
        s.check()
        prof = s.profile_read()
        res[name] = {"rho": s.interior()[0], "sweep_ms": sum(prof["sweep_%s" % a][1] for a in "xy"),
                     "sensor_ms": prof["sensor"][1], "stats": s.sensor_stats() if kw else None,
                     "steps": s.nsteps_done}
    a, b = res["routed"]["rho"], res["plain"]["rho"]
    res["l1"] = np.abs(a - b).mean() / np.abs(b).mean()
    res["acc"], res["thr"] = acc, thr
    sm, tot = res["routed"]["stats"]
    say("   threshold %.3f, %d steps: rel L1(rho) routed vs plain %.3e; smooth fraction %.3f; "
        "sweep ms plain %.2f routed %.2f (+ sensor %.2f)"
        % (thr, res["plain"]["steps"], res["l1"], sm / tot, res["plain"]["sweep_ms"], res["routed"]["sweep_ms"],
           res["routed"]["sensor_ms"]))
    return res


def test_trained_sensor_error(trained_routing_run):
    """The trained network separates the classes well above chance, and the
    routed run stays within the 1e-4 relative L1 density bar of plain."""
    r = trained_routing_run
    assert r["acc"] > 0.6  # balanced classes: well above chance
    assert r["l1"] <= 1e-4
    sm, tot = r["routed"]["stats"]
    assert sm > 0  # some interfaces do take the cheap flux


@pytest.mark.xfail(strict=True, reason=(
    "measured on MI355X: the routed sweeps plus the sensor are slower than plain TENO5 sweeps -- "
    "only 5-12 % of the shock-vortex interfaces are routed cheap by the network trained here, the cheap "
    "flux is about 35 % cheaper than TENO5 per interface (the Roe state, eigen-projection, per-point "
    "loads and the register window stay), and features plus inference cost about a quarter of a sweep"))
def test_trained_sensor_gain(trained_routing_run):
    """What the trained network gains over the method without it: routed
    sweeps plus the sensor against the plain sweeps of the same run."""
    r = trained_routing_run
    assert r["routed"]["sweep_ms"] + r["routed"]["sensor_ms"] < r["plain"]["sweep_ms"]
