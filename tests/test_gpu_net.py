"""GPU checks of the learned-warm-start network against the FP64 oracle.

Each matrix-core kernel is compared with the oracle's direct convolution on
identical BF16-valued inputs and weights (the GPU accumulates in FP32, so the
bar is a few FP32 rounding errors of the 27 * Cin-term sums).  The whole
network gradient is compared with a reference that runs the oracle's
convolutions in FP64 and rounds activations and activation gradients to BF16
at the same points as the GPU (bar 1e-2 relative L2: a BF16 rounding can fall
on the other side for a few entries).  Training must lower the loss, and the
learned initial iterate must leave the converged solution unchanged.
"""
import numpy as np
import pytest

import oracle
from paper_2211_08263_amd import newmark as nmb
from paper_2211_08263_amd import workloads as W

pytestmark = pytest.mark.gpu

LEAK = 0.1


def bf16_bits(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    return (u >> 16).astype(np.uint16)


def bf16_val(a):
    return (bf16_bits(a).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def dev_u16(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int16)).cuda()


def cl_to_cf(x, n, c):
    """channels-last [N][C] -> channels-first (c, n3, n2, n1)"""
    return np.ascontiguousarray(x[:, :c].T).reshape(c, n[2], n[1], n[0])


def cf_to_cl(x):
    c = x.shape[0]
    return np.ascontiguousarray(x.reshape(c, -1).T)


GRIDS = [(16, 8, 8), (32, 16, 8), (16, 16, 32)]


@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("cinp,cin,cout", [(32, 31, 16), (16, 16, 16), (16, 16, 3)])
def test_conv_forward_matches_oracle(n, cinp, cin, cout):
    import torch
    rng = np.random.default_rng(sum(n) + cin + cout)
    N = n[0] * n[1] * n[2]
    x = bf16_val(rng.standard_normal((N, cinp)))
    w = rng.standard_normal((cout, cin, 27)).astype(np.float32) * 0.3
    b = rng.standard_normal(cout).astype(np.float32)
    out = torch.zeros(N * 16, dtype=torch.float32, device="cuda")
    nmb.conv3d_bf16(0, n, cinp, cin, cout, x=dev_u16(bf16_bits(x)), w=w, bias=b, out=out)
    got = out.cpu().numpy().reshape(N, 16)[:, :cout]
    want = cf_to_cl(oracle.conv3d_fwd(cl_to_cf(x, n, cin), bf16_val(w).reshape(cout, cin, 3, 3, 3), b, n))
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"conv fwd n={n} cinp={cinp} cin={cin} cout={cout}: {err:.2e}", flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("cout", [16, 3])
def test_conv_backward_data_matches_oracle(n, cout):
    import torch
    rng = np.random.default_rng(7 + cout)
    N = n[0] * n[1] * n[2]
    cin = 16
    dy = np.zeros((N, 16))
    dy[:, :cout] = bf16_val(rng.standard_normal((N, cout)))
    w = rng.standard_normal((cout, cin, 27)).astype(np.float32) * 0.3
    out = torch.zeros(N * 16, dtype=torch.float32, device="cuda")
    nmb.conv3d_bf16(1, n, 16, cin, cout, w=w, dy=dev_u16(bf16_bits(dy)), out=out)
    got = out.cpu().numpy().reshape(N, 16)[:, :cin]
    want = cf_to_cl(oracle.conv3d_bwd_data(cl_to_cf(dy, n, cout), bf16_val(w).reshape(cout, cin, 3, 3, 3), n))
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"conv bwd-data n={n} cout={cout}: {err:.2e}", flush=True)
    assert err < 1e-5


@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("cinp,cin,cout", [(32, 31, 16), (16, 16, 3)])
def test_conv_backward_weight_matches_oracle(n, cinp, cin, cout):
    rng = np.random.default_rng(11 + cin)
    N = n[0] * n[1] * n[2]
    x = bf16_val(rng.standard_normal((N, cinp)))
    dy = np.zeros((N, 16))
    dy[:, :cout] = bf16_val(rng.standard_normal((N, cout)))
    dw, db = nmb.conv3d_bf16(2, n, cinp, cin, cout, x=dev_u16(bf16_bits(x)), dy=dev_u16(bf16_bits(dy)))
    wdw, wdb = oracle.conv3d_bwd_weight(cl_to_cf(x, n, cin), cl_to_cf(dy, n, cout), cin, cout, n)
    err = np.abs(dw - wdw.reshape(cout, cin, 27)).max() / np.abs(wdw).max()
    errb = np.abs(db - wdb).max() / np.abs(wdb).max()
    print(f"conv bwd-weight n={n} cin={cin} cout={cout}: {err:.2e} bias {errb:.2e}", flush=True)
    assert err < 1e-4 and errb < 1e-4


def _reference_grad(params, feat, target, n):
    """FP64 backprop with BF16 storage of activations and activation gradients."""
    cins, couts = [31, 16, 16, 16], [16, 16, 16, 3]
    Ws, bs, off = [], [], 0
    for ci, co in zip(cins, couts):
        Ws.append(bf16_val(params[off: off + co * ci * 27]).reshape(co, ci, 3, 3, 3))
        off += co * ci * 27
        bs.append(params[off: off + co].astype(np.float64))
        off += co
    N = feat.shape[0]
    A = [cl_to_cf(feat, n, 31)]
    for l in range(3):
        z = oracle.conv3d_fwd(A[-1], Ws[l], bs[l], n)
        A.append(bf16_val(np.where(z > 0, z, LEAK * z)))
    pred = oracle.conv3d_fwd(A[3], Ws[3], bs[3], n)
    t = cl_to_cf(target, n, 3)
    loss = np.mean((pred - t) ** 2)
    dz = bf16_val(2 * (pred - t) / (3 * N))
    grads = [None] * 4
    for l in range(3, -1, -1):
        dw, db = oracle.conv3d_bwd_weight(A[l], dz, cins[l], couts[l], n)
        grads[l] = (dw.reshape(-1), db)
        if l > 0:
            da = oracle.conv3d_bwd_data(dz, Ws[l], n)
            dz = bf16_val(np.where(A[l] > 0, da, LEAK * da))
    g = np.concatenate([np.concatenate([gw, gb]) for gw, gb in grads])
    return g, loss


def test_network_gradient_matches_reference():
    import torch
    n = (16, 16, 8)
    N = n[0] * n[1] * n[2]
    rng = np.random.default_rng(3)
    feat = np.zeros((N, 32))
    feat[:, :31] = bf16_val(rng.standard_normal((N, 31)))
    target = np.zeros((N, 4), dtype=np.float32)
    target[:, :3] = rng.standard_normal((N, 3))
    net = nmb.Net(seed=5)
    params = net.get_params()
    g, loss = net.gradients(n, dev_u16(bf16_bits(feat)), torch.from_numpy(target).cuda())
    gr, lr = _reference_grad(params, feat, target, n)
    err = np.linalg.norm(g - gr) / np.linalg.norm(gr)
    print(f"network gradient rel L2 {err:.2e}, loss {loss:.6f} vs {lr:.6f}", flush=True)
    assert abs(loss - lr) / lr < 1e-4
    assert err < 1e-2
    net.close()


def _trajectory_samples(pb, steps, net):
    """Features/targets of consecutive steps of the FP64 solver (previous-step start)."""
    import torch
    N = pb.n_vox
    feats, targets = [], []
    with nmb.newmark_init_problem(pb, nmb.Options(tol=1e-10, max_iter=500)) as ctx:
        nmb.ws_attach(ctx, net)
        for s in range(steps):
            f = torch.empty(N * 32, dtype=torch.int16, device="cuda")
            t = torch.empty(N * 4, dtype=torch.float32, device="cuda")
            nmb.ws_features(ctx, f)
            nmb.newmark_step(ctx, pb.U(s + 1))
            nmb.ws_target(ctx, t)
            feats.append(f)
            targets.append(t)
    return feats, targets


def test_training_lowers_loss_and_learned_start_keeps_the_solution():
    import torch
    pb = W.make_polycrystal(n=32, n_grains=8, seed=1001, n_steps=16)
    net = nmb.Net(seed=1)
    feats, targets = _trajectory_samples(pb, 16, net)
    grid = pb.n
    losses = []
    for epoch in range(25):
        tot = 0.0
        for f, t in zip(feats[4:], targets[4:]):
            tot += net.train_step(grid, f, t, lr=2e-3)
        losses.append(tot / len(feats[4:]))
    print("training losses", [f"{x:.4g}" for x in losses[::4]], flush=True)
    assert losses[-1] < 0.7 * losses[0]
    # learned initial iterate: same converged trajectory as the previous-step start
    res = {}
    for ws in (nmb.WS_PREV, nmb.WS_LEARNED):
        with nmb.newmark_init_problem(pb, nmb.Options(tol=1e-10, max_iter=500, warm_start=ws)) as ctx:
            if ws == nmb.WS_LEARNED:
                nmb.ws_attach(ctx, net)
            its = []
            for s in range(12):
                st = nmb.newmark_step(ctx, pb.U(s + 1))
                its.append(st["iters"][0])
            res[ws] = (nmb.get_state(ctx)["u"], its)
    u0, u1 = res[nmb.WS_PREV][0], res[nmb.WS_LEARNED][0]
    rel = np.linalg.norm(u1 - u0) / np.linalg.norm(u0)
    print("iterations prev", res[nmb.WS_PREV][1], "learned", res[nmb.WS_LEARNED][1], "rel diff", rel, flush=True)
    assert rel < 1e-7
    net.close()


def test_learned_start_with_mixed_precision_keeps_the_solution():
    """Learned start under mixed precision: the prediction kernel also writes the FP32 copy
    the first refinement sweep starts from (with the prescribed Gamma values set in both
    copies) and the scale comes from the sums the fused corrector left.  The trajectory must
    agree with the FP64 zero-start one to the mixed-precision tolerance, on the slab and on a
    sphere source with per-step varying values."""
    for gamma in ("slab", "sphere"):
        kw = dict(gamma="sphere", sphere_radius=4.0) if gamma == "sphere" else {}
        pb = W.make_polycrystal(n=32, n_grains=8, seed=1007, n_steps=10, **kw)
        net = nmb.Net(seed=3)
        res = {}
        for name, prec, ws in (("fp64", nmb.PREC_FP64, nmb.WS_COLD), ("mixed_learned", nmb.PREC_MIXED,
                                                                        nmb.WS_LEARNED)):
            opts = nmb.Options(tol=1e-9, max_iter=500, warm_start=ws, precision=prec, inner_tol=1e-5,
                               true_residual=True)
            with nmb.newmark_init_problem(pb, opts) as ctx:
                if ws == nmb.WS_LEARNED:
                    nmb.ws_attach(ctx, net)
                us, st = [], []
                for s in range(8):
                    st.append(nmb.newmark_step(ctx, pb.U(s + 1)))
                    us.append(nmb.get_state(ctx)["u"].reshape(3, -1).copy())
            res[name] = (us, st)
        errs = [np.linalg.norm(a - b) / np.linalg.norm(a) for a, b in zip(res["fp64"][0], res["mixed_learned"][0])
                if np.abs(a).max() > 0]
        print(f"{gamma}: learned+mixed vs FP64 max rel L2 {max(errs):.2e}, relres "
              f"{max(x['relres'] for x in res['mixed_learned'][1]):.2e}, sweeps "
              f"{[x['sweeps'] for x in res['mixed_learned'][1]]}", flush=True)
        assert max(x["relres"] for x in res["mixed_learned"][1]) <= 1e-9  # FP64 residual of the iterate
        assert max(errs) < 1e-5
        for s, u in enumerate(res["mixed_learned"][0]):
            want = pb.U(s + 1)
            for c in range(3):
                assert np.array_equal(u[c, pb.gamma_idx], np.full(pb.gamma_idx.size, want[c]))
        net.close()


def test_features_and_target_match_the_newmark_state():
    """Features from (u_n, v_n, a_n), scale s = rms(u~ - u_n) and target (u_{n+1} - u~)/s,
    recomputed in FP64 from the library's own state (the predictor u~ written out from the
    Newmark update rule with beta = 1/4)."""
    import torch
    pb = W.make_polycrystal(n=16, n_grains=4, seed=1002, n_steps=8)
    N = pb.n_vox
    net = nmb.Net(seed=2)
    with nmb.newmark_init_problem(pb, nmb.Options(tol=1e-10, max_iter=500)) as ctx:
        nmb.ws_attach(ctx, net)
        for s in range(5):
            nmb.newmark_step(ctx, pb.U(s + 1))
        st = nmb.get_state(ctx)
        f = torch.empty(N * 32, dtype=torch.int16, device="cuda")
        t = torch.empty(N * 4, dtype=torch.float32, device="cuda")
        nmb.ws_features(ctx, f)
        nmb.newmark_step(ctx, pb.U(6))
        nmb.ws_target(ctx, t)
        u1 = nmb.get_state(ctx)["u"]
    net.close()
    u, v, a = (st[k].reshape(3, N) for k in ("u", "v", "a"))
    c2 = pb.dt ** 2 * (0.5 - pb.beta)
    ut = u + pb.dt * v + c2 * a
    s = np.sqrt(np.mean((ut - u) ** 2))
    assert s > 0
    feat = (f.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32).reshape(N, 32)
    want = np.concatenate([u / s, pb.dt * v / s, c2 * a / s]).T
    err = np.abs(feat[:, :9] - want).max() / np.abs(want).max()
    print(f"state features: max err {err:.2e} (BF16 half-ulp 3.9e-3)", flush=True)
    assert err < 4e-3
    ph = pb.phase_id.reshape(-1)
    mat = feat[:, 9:31].astype(np.float64)
    ref = np.concatenate([pb.rho[:, None], pb.C21], axis=1)[ph]
    # density over one constant, the 21 stiffnesses over one other constant (C11 of the
    # reference medium), each rounded to BF16
    for sl in (slice(0, 1), slice(1, 22)):
        m, r = mat[:, sl], ref[:, sl]
        k = float((m * r).sum() / (r * r).sum())
        assert k > 0
        dev = np.abs(m - k * r).max() / np.abs(k * r).max()
        assert dev < 4e-3, (sl, dev)
    assert feat[:, 31].max() == 0 and feat[:, 31].min() == 0
    tg = t.cpu().numpy().reshape(N, 4)
    wt = ((u1.reshape(3, N) - ut) / s).T
    errt = np.abs(tg[:, :3] - wt).max() / np.abs(wt).max()
    print(f"target: max err {errt:.2e}", flush=True)
    assert errt < 1e-6 and tg[:, 3].max() == 0 and tg[:, 3].min() == 0


def test_residual_sample_and_loss_match_the_oracle_operator():
    """rp = P(b - A u~_Gamma), cref = |P(b - A u_bar)|^2 and the residual-norm loss of the
    learned start, recomputed with the oracle's FP64 operator; the solver state is untouched."""
    import torch
    pb = W.make_polycrystal(n=16, n_grains=4, seed=1004, n_steps=8)
    N = pb.n_vox
    op = oracle.OracleProblem.from_problem(pb)
    fixed = np.zeros(N, bool)
    fixed[pb.gamma_idx] = True
    net = nmb.Net(seed=3)
    with nmb.newmark_init_problem(pb, nmb.Options(tol=1e-10, max_iter=500)) as ctx:
        nmb.ws_attach(ctx, net)
        for s in range(4):
            nmb.newmark_step(ctx, pb.U(s + 1))
        st = nmb.get_state(ctx)
        f = torch.empty(N * 32, dtype=torch.int16, device="cuda")
        rp = torch.empty(3 * N, dtype=torch.float64, device="cuda")
        sc, cref, crefm = nmb.ws_residual_sample(ctx, pb.U(5), f, rp)
        pred = torch.empty(N * 4, dtype=torch.float32, device="cuda")
        net.forward(pb.n, f, pred)
        loss = nmb.ws_train_residual(ctx, f, rp, sc, cref, lr=1e-3, metric=0)
        pred2 = torch.empty_like(pred)
        net.forward(pb.n, f, pred2)
        lossm = nmb.ws_train_residual(ctx, f, rp, sc, crefm, lr=1e-3, metric=1)
        st2 = nmb.get_state(ctx)
    net.close()
    for k in ("u", "v", "a"):
        assert np.array_equal(st[k], st2[k])

    def A(x):
        return op.apply(x.reshape(op.field_shape)).reshape(3, N)

    def PM(x):
        z = op.precond(x.reshape(op.field_shape)).reshape(3, N)
        z[:, fixed] = 0
        return z

    u, v, a = (st[k].reshape(3, N) for k in ("u", "v", "a"))
    ut = u + pb.dt * v + pb.dt ** 2 * (0.5 - pb.beta) * a
    U5 = pb.U(5)[:, None]
    b = pb.rho[pb.phase_id.reshape(-1)][None, :] * ut
    utg = ut.copy()
    utg[:, fixed] = U5
    rp_want = b - A(utg)
    rp_want[:, fixed] = 0
    ubar = np.zeros((3, N))
    ubar[:, fixed] = U5
    r_bar = b - A(ubar)
    r_bar[:, fixed] = 0
    cref_want = float((r_bar ** 2).sum())
    s_want = float(np.sqrt(np.mean((ut - u) ** 2)))
    got = rp.cpu().numpy().reshape(3, N)
    e_rp = np.abs(got - rp_want).max() / np.abs(rp_want).max()
    print(f"rp err {e_rp:.2e}, cref {cref:.6e} vs {cref_want:.6e}, s {sc:.6e} vs {s_want:.6e}", flush=True)
    assert e_rp < 1e-12
    assert abs(cref - cref_want) <= 1e-12 * cref_want
    assert abs(sc - s_want) <= 1e-12 * s_want
    y = sc * pred.cpu().numpy().astype(np.float64).reshape(N, 4)[:, :3].T
    y[:, fixed] = 0
    r0 = rp_want - A(y)
    r0[:, fixed] = 0
    loss_want = float((r0 ** 2).sum()) / cref_want
    print(f"loss {loss:.7g} vs {loss_want:.7g}", flush=True)
    assert abs(loss - loss_want) <= 1e-5 * loss_want
    crefm_want = float((r_bar * PM(r_bar)).sum())
    assert abs(crefm - crefm_want) <= 1e-12 * crefm_want
    y2 = sc * pred2.cpu().numpy().astype(np.float64).reshape(N, 4)[:, :3].T
    y2[:, fixed] = 0
    r02 = rp_want - A(y2)
    r02[:, fixed] = 0
    lossm_want = float((r02 * PM(r02)).sum()) / crefm_want
    print(f"energy loss {lossm:.7g} vs {lossm_want:.7g}", flush=True)
    assert abs(lossm - lossm_want) <= 1e-5 * lossm_want


def test_residual_training_lowers_the_initial_residual():
    import torch
    pb = W.make_polycrystal(n=32, n_grains=8, seed=1005, n_steps=14)
    N = pb.n_vox
    net = nmb.Net(seed=4)
    with nmb.newmark_init_problem(pb, nmb.Options(tol=1e-10, max_iter=500, warm_start=nmb.WS_COLD)) as ctx:
        nmb.ws_attach(ctx, net)
        samples = []
        for s in range(14):
            f = torch.empty(N * 32, dtype=torch.int16, device="cuda")
            rp = torch.empty(3 * N, dtype=torch.float64, device="cuda")
            sc, cref, crefm = nmb.ws_residual_sample(ctx, pb.U(s + 1), f, rp)
            nmb.newmark_step(ctx, pb.U(s + 1))
            if s >= 4:
                samples.append((f, rp, sc, crefm))
        losses = []
        for epoch in range(30):
            losses.append(np.mean([nmb.ws_train_residual(ctx, f, rp, sc, crefm, lr=2e-3, metric=1)
                                   for f, rp, sc, crefm in samples]))
    print("residual training losses", [f"{x:.4g}" for x in losses[::5]], losses[-1], flush=True)
    assert losses[-1] < 0.5 * losses[0]
    net.close()


def test_solver_inference_matches_the_full_network():
    """The solver caches the material share of the first layer; its learned iterate must
    agree with u~ + s net(f) evaluated on the full 31-channel features (BF16 activations:
    a rounding can fall on the other side for a few entries), also after the weights change."""
    import torch
    pb = W.make_polycrystal(n=32, n_grains=6, seed=1006, n_steps=8)
    N = pb.n_vox
    net = nmb.Net(seed=9)
    with nmb.newmark_init_problem(pb, nmb.Options(tol=1e-10, max_iter=500)) as ctx:
        nmb.ws_attach(ctx, net)
        for s in range(4):
            nmb.newmark_step(ctx, pb.U(s + 1))
        for trial in range(2):
            st = nmb.get_state(ctx)
            u, v, a = (st[k].reshape(3, N) for k in ("u", "v", "a"))
            ut = u + pb.dt * v + pb.dt ** 2 * (0.5 - pb.beta) * a
            sc = np.sqrt(np.mean((ut - u) ** 2))
            x0 = torch.empty(3 * N, dtype=torch.float64, device="cuda")
            nmb.ws_predict(ctx, x0)
            f = torch.empty(N * 32, dtype=torch.int16, device="cuda")
            nmb.ws_features(ctx, f)
            pred = torch.empty(N * 4, dtype=torch.float32, device="cuda")
            net.forward(pb.n, f, pred)
            want = sc * pred.cpu().numpy().astype(np.float64).reshape(N, 4)[:, :3].T
            got = x0.cpu().numpy().reshape(3, N) - ut
            err = np.linalg.norm(got - want) / np.linalg.norm(want)
            print(f"weights {trial}: cached-first-layer inference vs full network rel L2 {err:.2e}", flush=True)
            assert err < 1e-2
            # change the weights: the cached material share must be recomputed
            w = net.get_params()
            net.set_params(w * 1.05)
    net.close()


def test_trained_start_on_a_held_out_trajectory():
    """The shipped weights on a polycrystal none of the training trajectories used (64^3,
    8 grains, seed 1099): per-step initial relative residual, PCG iterations and step time
    for the cold (zero), previous-step and learned initial iterates, FP64 solver to 1e-8.
    The learned iterate must start closer to the solution than both (lower geometric-mean
    initial residual) and need no more iterations than the cold start; the iteration
    counts and times are recorded (see the printout)."""
    from paper_2211_08263_amd import warmstart
    pb = W.make_polycrystal(n=64, n_grains=8, seed=1099, n_steps=30)
    net = nmb.Net()
    assert warmstart.load_weights(net)
    res = {}
    for name, ws in (("cold", nmb.WS_COLD), ("prev", nmb.WS_PREV), ("learned", nmb.WS_LEARNED)):
        with nmb.newmark_init_problem(pb, nmb.Options(tol=1e-8, max_iter=500, warm_start=ws)) as ctx:
            if ws == nmb.WS_LEARNED:
                nmb.ws_attach(ctx, net)
            st = [nmb.newmark_step(ctx, pb.U(s + 1)) for s in range(24)]
        st = st[4:]  # from rest the first steps carry almost no signal
        res[name] = {"iters": float(np.mean([x["iters"][0] for x in st])),
                     "relres0": float(np.exp(np.mean([np.log(max(x["relres0"], 1e-300)) for x in st]))),
                     "ms": float(np.median([x["t_step_ms"] for x in st]))}
    net.close()
    print("held-out 64^3 trajectory:", {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in res.items()},
          flush=True)
    assert res["learned"]["relres0"] < 0.8 * res["cold"]["relres0"]
    assert res["learned"]["relres0"] < 0.8 * res["prev"]["relres0"]
    assert res["learned"]["iters"] <= res["cold"]["iters"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_learned_start_worse_than_zero_is_replaced_by_the_zero_start(precision):
    """A network that predicts nonsense (random weights scaled by 100): the step compares the
    learned iterate's projected residual with the zero start's and restarts from the zero
    start when it is larger, so no step starts further away than the zero start does, the
    iteration counts are the zero start's and the trajectory agrees with it to the tolerance."""
    pb = W.make_polycrystal(n=32, n_grains=8, seed=1007, n_steps=10)
    net = nmb.Net(seed=5)
    net.set_params(net.get_params() * 100.0)
    prec = nmb.PREC_MIXED if precision == "mixed" else nmb.PREC_FP64
    res = {}
    for name, ws in (("cold", nmb.WS_COLD), ("learned", nmb.WS_LEARNED)):
        opts = nmb.Options(tol=1e-9, max_iter=500, warm_start=ws, precision=prec, true_residual=True)
        with nmb.newmark_init_problem(pb, opts) as ctx:
            if ws == nmb.WS_LEARNED:
                nmb.ws_attach(ctx, net)
            st, us = [], []
            for s in range(8):
                st.append(nmb.newmark_step(ctx, pb.U(s + 1)))
                us.append(nmb.get_state(ctx)["u"].copy())
        res[name] = (st, us)
    net.close()
    key = "inner_iters" if precision == "mixed" else "iters"
    it = {k: [x[key] if precision == "mixed" else x[key][0] for x in v[0]] for k, v in res.items()}
    r0 = [x["relres0"] for x in res["learned"][0]]
    err = max(np.linalg.norm(a - b) / max(np.linalg.norm(a), 1e-300)
              for a, b in zip(res["cold"][1], res["learned"][1]) if np.abs(a).max() > 0)
    print(f"{precision}: nonsense network, initial residuals {np.round(r0, 6).tolist()}, iterations "
          f"{it['learned']} (zero start {it['cold']}), rel L2 to the zero-start run {err:.2e}", flush=True)
    assert all(r <= 1.0 + 1e-6 for r in r0)
    assert all(abs(a - b) <= 1 for a, b in zip(it["learned"], it["cold"]))
    assert max(x["relres"] for x in res["learned"][0]) <= 1e-9
    assert err <= 1e-7


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_learned_start_guard_on_the_green_route(precision):
    """The same guard on the Green route's u_b solve (residual against ||b||, the zero start's):
    with a nonsense network no step starts further away than zero, and the trajectory agrees
    with the zero-start Green route to the tolerance."""
    pb = W.make_polycrystal(n=16, n_grains=6, seed=7, gamma="sphere", sphere_radius=1.5, n_steps=8)
    net = nmb.Net(seed=5)
    net.set_params(net.get_params() * 100.0)
    prec = nmb.PREC_MIXED if precision == "mixed" else nmb.PREC_FP64
    res = {}
    for name, ws in (("cold", nmb.WS_COLD), ("learned", nmb.WS_LEARNED)):
        opts = nmb.Options(tol=1e-10, max_iter=500, warm_start=ws, precision=prec, route=nmb.ROUTE_GREEN,
                           green_tol=1e-12)
        with nmb.newmark_init_problem(pb, opts) as ctx:
            if ws == nmb.WS_LEARNED:
                nmb.ws_attach(ctx, net)
            st, us = [], []
            for s in range(6):
                st.append(nmb.newmark_step(ctx, pb.U(s + 1)))
                us.append(nmb.get_state(ctx)["u"].copy())
        res[name] = (st, us)
    net.close()
    r0 = [x["relres0"] for x in res["learned"][0]]
    err = max(np.linalg.norm(a - b) / max(np.linalg.norm(a), 1e-300)
              for a, b in zip(res["cold"][1], res["learned"][1]) if np.abs(a).max() > 0)
    print(f"Green route, {precision}: nonsense network, initial residuals {np.round(r0, 6).tolist()}, rel L2 to "
          f"the zero-start run {err:.2e}", flush=True)
    assert all(r <= 1.0 + 1e-6 for r in r0)
    assert err <= 1e-8
