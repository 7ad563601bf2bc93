"""GPU adjoint (HIP rollout forward + hand-written backward, through ClothRollout) against
the FP64 oracle.

The gradient is that of the current smooth piece of the rollout: every substep's contact
sets held fixed.  With collision, a resting node sits exactly at the thickness after every
push, so FP32 and FP64 runs take different contact decisions at many nodes and their
rollouts lie on different smooth pieces.  The references are therefore built on the GPU's
own piece: its trajectory is recorded substep by substep with the contact sets its step
uses (cloth_debug_contacts), every set is checked against the oracle's distances at the
FP64 prediction from the GPU state (it must hold every triangle within th - 1e-6 m and only
triangles within th + 1e-6 m), and then
  - the oracle's substep adjoint with those sets is run backwards along the trajectory
    (the FP64 reference adjoint), and
  - central differences (h = 1e-3 relative) of the FP64 oracle rollout with those sets
    held fixed give the derivative of the same piece directly.
Without collision the trajectories agree and the GPU gradient is also checked against
central differences of the plain FP64 oracle forward.  Bar: 1e-3 relative (normwise for
whole gradients; per entry, with a floor of 1e-3 of the largest entry, for differences)."""
import numpy as np
import pytest

import oracle
from paper_2507_11794_amd import cloth as B
from paper_2507_11794_amd import workloads as W

pytestmark = pytest.mark.gpu


def h32(inp):
    return float(np.float32(np.float32(inp.dt) / np.float32(inp.n_substeps)))


def _rollout(sim, k, c, v0, n_steps, ckpt, out_steps):
    from paper_2507_11794_amd.rollout import ClothRollout
    inp = sim.inp
    return ClothRollout.apply(sim, k, c, v0, inp.dt, inp.n_substeps, n_steps, ckpt, out_steps)


def _gpu_grads(inp, n_steps, target, ckpt=20, v0=None):
    import torch
    dev = torch.device("cuda")
    with B.Cloth(inp) as sim:
        k = torch.tensor(inp.k, device=dev, requires_grad=True)
        c = torch.tensor(inp.c, device=dev, requires_grad=True)
        v = torch.tensor(inp.v0 if v0 is None else v0, device=dev, requires_grad=True)
        x = _rollout(sim, k, c, v, n_steps, ckpt, [n_steps])
        tgt = torch.tensor(target, dtype=torch.float32, device=dev)
        loss = ((x[0] - tgt) ** 2).sum(dim=1).mean()
        loss.backward()
        torch.cuda.synchronize()
        return (k.grad.cpu().numpy().astype(np.float64), c.grad.cpu().numpy().astype(np.float64),
                v.grad.cpu().numpy().astype(np.float64), x[0].detach().cpu().numpy())


def _record_gpu_trajectory(inp, n_steps, cap=16):
    """Step the GPU substep by substep: the state before every substep, the contact sets
    that substep uses (CSR, caller node order) and the final positions."""
    h = h32(inp)
    xs, vs, sets = [], [], []
    with B.Cloth(inp) as sim:
        for _ in range(n_steps * inp.n_substeps):
            x, v = sim.read_state()
            xs.append(x)
            vs.append(v)
            sets.append(sim.debug_contacts(h, cap=cap, csr=True) if inp.thickness > 0 else
                        (np.zeros(inp.n_nodes + 1, dtype=np.int32), np.zeros(0, np.int32)))
            sim.step(dt=h, n_substeps=1, n_steps=1)
        xT, _ = sim.read_state()
    return xs, vs, sets, xT


def _check_contact_sets(m, xs, vs, sets, h, border=1e-6):
    """Every substep's GPU contact sets against the oracle at the FP64 prediction from the
    GPU's state: sure contacts (distance < th - border) all listed, nothing listed beyond
    th + border, nothing on pinned nodes.  Returns (listed contacts, near-threshold ones)."""
    listed = near = 0
    for s, (x, v, cs) in enumerate(zip(xs, vs, sets)):
        xp, _ = m.predict(x, v, h)
        st, nb = m.check_contacts(xp, cs, border)
        bad = np.nonzero(st)[0]
        assert bad.size == 0, ("substep", s, "invalid contact sets at nodes", bad[:8].tolist(),
                               st[bad[:8]].tolist())
        listed += int(cs[0][-1])
        near += nb
    return listed, near


def _oracle_adjoint_on_gpu_trajectory(m, inp, xs, vs, sets, xT, target):
    """The oracle's substep adjoint with the GPU's contact sets, run backwards along the
    GPU's trajectory."""
    h = h32(inp)
    xb = (2.0 / inp.n_nodes) * (xT.astype(np.float64) - target)
    vb = np.zeros_like(xb)
    gk, gc = np.zeros(inp.n_springs), np.zeros(inp.n_springs)
    for n in range(len(xs) - 1, -1, -1):
        xb, vb, kb, cb = m.substep_vjp_given(xs[n], vs[n], h, sets[n], xb, vb)
        gk += kb
        gc += cb
    return gk, gc, vb


def _target(inp, n_steps, seed=11):
    rng = np.random.default_rng(seed)
    m = oracle.Model.from_inputs(inp)
    m.set_params(k=inp.k.astype(np.float64) * (1 + 0.1 * rng.normal(size=inp.n_springs)))
    x, _ = m.run(inp.x0, inp.v0, h32(inp), n_steps * inp.n_substeps)
    return x


def _normwise(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_forward_matches_plain_stepping_bitwise():
    import torch
    inp = W.small_collision_scene(n=14, freq=5, drop=0.165, spacing=0.02)
    dev = torch.device("cuda")
    with B.Cloth(inp) as plain:
        plain.step(n_steps=60)
        xp, _ = plain.read_state()
    with B.Cloth(inp) as sim:
        k = torch.tensor(inp.k, device=dev)
        c = torch.tensor(inp.c, device=dev)
        v0 = torch.zeros((inp.n_nodes, 3), device=dev)
        x = _rollout(sim, k, c, v0, 60, 20, [0, 30, 60])
        torch.cuda.synchronize()
        assert np.array_equal(x[2].cpu().numpy(), xp)
        assert np.array_equal(x[0].cpu().numpy(), inp.x0)


def _scene(name):
    if name == "small":
        inp = W.small_collision_scene(n=14, freq=5, drop=0.165, spacing=0.02)
        return inp, 60, _target(inp, 60)
    # 64x64 cloth over a 2,000-triangle sphere, 200 frames x 4 substeps, checkpoints every
    # 20 frames; the target is the oracle's forward pass with the workload's perturbed
    # stiffness k_hat = k (1 + 0.1 xi)
    inp, k_hat = W.config4()
    m = oracle.Model.from_inputs(inp, k=k_hat.astype(np.float64))
    x, _ = m.run(inp.x0, inp.v0, h32(inp), inp.n_steps * inp.n_substeps)
    return inp, inp.n_steps, x


_RUNS = {}


def _run(name):
    """GPU gradients of the scene's loss plus the recorded GPU trajectory and its validated
    contact sets (computed once per scene)."""
    if name not in _RUNS:
        inp, n_steps, target = _scene(name)
        gk, gc, gv, xT = _gpu_grads(inp, n_steps, target)
        xs, vs, sets, xT2 = _record_gpu_trajectory(inp, n_steps)
        assert np.array_equal(xT, xT2)  # the rollout steps exactly as plain stepping
        m = oracle.Model.from_inputs(inp)
        listed, near = _check_contact_sets(m, xs, vs, sets, h32(inp))
        print(f"{name}: {len(xs)} substeps, {listed} contacts listed by the GPU, all valid "
              f"({near} within 1e-6 m of the thickness)")
        _RUNS[name] = dict(inp=inp, n_steps=n_steps, target=target, g=(gk, gc, gv), xs=xs,
                           vs=vs, sets=sets, xT=xT, m=m, listed=listed)
    return _RUNS[name]


@pytest.mark.parametrize("scene", ["small", "config4"])
def test_gradients_match_oracle_adjoint_on_gpu_contact_sets(scene):
    r = _run(scene)
    assert r["listed"] > 100
    rk, rc, rv = _oracle_adjoint_on_gpu_trajectory(r["m"], r["inp"], r["xs"], r["vs"],
                                                   r["sets"], r["xT"], r["target"])
    for name, a, b in zip(("k", "c", "v0"), r["g"], (rk, rc, rv)):
        err = _normwise(a, b)
        print(f"{scene} {name}: normwise relative error {err:.2e} (|g| = {np.linalg.norm(b):.3e})")
        assert err <= 1e-3, name


def _oracle_adjoint_on_given_trajectory(m, inp, sets, target):
    """The FP64 trajectory of the smooth piece with the given contact sets, from the initial
    state, and the oracle's substep adjoint run backwards along it: the derivative that
    central differences of run_given approximate."""
    h = h32(inp)
    x, v = inp.x0.astype(np.float64), inp.v0.astype(np.float64)
    xs, vs = [], []
    for cs in sets:
        xs.append(x)
        vs.append(v)
        x, v = m.substep_given(x, v, h, cs)
    xb = (2.0 / inp.n_nodes) * (x - target)
    vb = np.zeros_like(xb)
    gk, gc = np.zeros(inp.n_springs), np.zeros(inp.n_springs)
    for n in range(len(sets) - 1, -1, -1):
        xb, vb, kb, cb = m.substep_vjp_given(xs[n], vs[n], h, sets[n], xb, vb)
        gk += kb
        gc += cb
    return gk, gc, vb


def test_config4_gradients_match_central_differences_with_collision():
    """15 entries each of k, c and v0: central differences of the FP64 oracle rollout with
    the GPU's validated contact sets held fixed, i.e. of the smooth piece the GPU's gradient
    differentiates (no FD sample can flip a contact: the sets are fixed).  The step is 1e-3
    of the entry (of 0.01 m/s for the zero v0) first; the 800-substep rollout over the
    surface is strongly curved in some entries (the difference's error falls with the square
    of the step), so where the 1e-3 step misses the bar below it is retaken at 1e-4, 1e-5
    and 1e-6 (a wrong derivative misses at every step: the differences converge to it).

    The FD differentiates the piece along its FP64 trajectory from the initial state; the
    GPU differentiates it along its own FP32 trajectory, whose small rounding differences
    the 800 substeps of contact amplify.  So, per sampled entry:
      (a) the FP64 adjoint along the FP64 trajectory of the piece (a) matches the
          difference to 1e-3 relative (floor 1e-6 of its largest entry);
      (b) the GPU gradient (g) matches the FP64 adjoint along the GPU's own states (b) to
          1e-3 of max(|b|, 1e-3 of b's largest entry);
      (c) the GPU gradient matches the difference to 1e-3 of max(|difference|, the largest
          gradient entry) -- the bar of the test without collision -- plus |a - b|, the
          part the two trajectories account for (an oracle quantity: both adjoints are the
          oracle's)."""
    r = _run("config4")
    inp, m, target, sets = r["inp"], r["m"], r["target"], r["sets"]
    h = h32(inp)
    k0, c0 = inp.k.astype(np.float64), inp.c.astype(np.float64)
    v00 = inp.v0.astype(np.float64)
    gk, gc, gv = r["g"]
    ak, ac, av = _oracle_adjoint_on_given_trajectory(m, inp, sets, target)
    bk, bc, bv = _oracle_adjoint_on_gpu_trajectory(m, inp, r["xs"], r["vs"], sets, r["xT"],
                                                   target)

    def loss(k, c, v):
        m.set_params(k=k, c=c)
        x, _ = m.run_given(inp.x0, v, h, sets)
        return np.mean(np.sum((x - target) ** 2, axis=1))

    rng = np.random.default_rng(44)
    report, steps = {}, {}
    try:
        for name, theta, g, a, b, scale in (("k", k0, gk, ak, bk, 0.0), ("c", c0, gc, ac, bc, 0.0),
                                            ("v0", v00, gv, av, bv, 0.01)):
            gmax, amax, bmax = np.abs(g).max(), np.abs(a).max(), np.abs(b).max()
            worst = np.zeros(4)
            for i in rng.choice(theta.size, 15, replace=False):
                for eps in (1e-3, 1e-4, 1e-5, 1e-6):
                    step = eps * max(abs(theta.flat[i]), scale)
                    vals = []
                    for sgn in (1, -1):
                        t = theta.copy()
                        t.flat[i] += sgn * step
                        args = {"k": (t, c0, v00), "c": (k0, t, v00), "v0": (k0, c0, t)}[name]
                        vals.append(loss(*args))
                    fd = (vals[0] - vals[1]) / (2 * step)
                    e_a = abs(fd - a.flat[i]) / max(abs(fd), 1e-6 * amax)
                    if e_a <= 1e-3:
                        break
                steps[(name, eps)] = steps.get((name, eps), 0) + 1
                e_b = abs(g.flat[i] - b.flat[i]) / max(abs(b.flat[i]), 1e-3 * bmax)
                traj = abs(a.flat[i] - b.flat[i])
                e_c = (abs(fd - g.flat[i]) - traj) / max(abs(fd), gmax)
                e_fd = abs(fd - g.flat[i]) / max(abs(fd), gmax)
                worst = np.maximum(worst, [e_a, e_b, e_c, e_fd])
                assert e_a <= 1e-3, ("FP64 adjoint vs FD", name, int(i), fd, float(a.flat[i]))
                assert e_b <= 1e-3, ("GPU vs FP64 adjoint on its states", name, int(i),
                                     float(g.flat[i]), float(b.flat[i]))
                assert e_c <= 1e-3, ("GPU vs FD", name, int(i), fd, float(g.flat[i]), traj, gmax)
            report[name] = worst
    finally:
        m.set_params(k=k0, c=c0)
    for name, w in report.items():
        print(f"config4 {name}: (a) FP64 adjoint vs FD {w[0]:.2e}; (b) GPU vs FP64 adjoint on "
              f"the GPU's states {w[1]:.2e}; (c) GPU vs FD beyond the trajectory term {w[2]:.2e} "
              f"(without it {w[3]:.2e}) of max(|fd|, |g|max)")
    print("entries per difference step", steps)


def test_gradients_match_central_differences_without_collision():
    inp = W.config0(n=16, n_steps=40)
    n_steps = inp.n_steps
    target = _target(inp, n_steps)
    rng = np.random.default_rng(4)
    v0 = (0.05 * rng.normal(size=(inp.n_nodes, 3))).astype(np.float32)
    gk, gc, gv, _ = _gpu_grads(inp, n_steps, target, ckpt=7, v0=v0)
    m = oracle.Model.from_inputs(inp)
    h = h32(inp)
    n_sub = n_steps * inp.n_substeps
    k0, c0, v00 = inp.k.astype(np.float64), inp.c.astype(np.float64), v0.astype(np.float64)

    def loss(k, c, v):
        m.set_params(k=k, c=c)
        x, _ = m.run(inp.x0, v, h, n_sub)
        return np.mean(np.sum((x - target) ** 2, axis=1))

    for name, theta, g, scale in (("k", k0, gk, 50.0), ("c", c0, gc, 0.05), ("v0", v00, gv, 0.1)):
        gmax = np.abs(g).max()
        for i in rng.choice(theta.size, 15, replace=False):
            step = 1e-3 * max(abs(theta.flat[i]), scale)
            vals = []
            for sgn in (1, -1):
                t = theta.copy()
                t.flat[i] += sgn * step
                args = {"k": (t, c0, v00), "c": (k0, t, v00), "v0": (k0, c0, t)}[name]
                vals.append(loss(*args))
            fd = (vals[0] - vals[1]) / (2 * step)
            assert abs(fd - g.flat[i]) <= 1e-3 * max(abs(fd), gmax), (name, int(i), fd, g.flat[i])
    m.set_params(k=k0, c=c0)


def test_gradients_independent_of_checkpoint_interval():
    import torch
    inp = W.small_collision_scene(n=14, freq=5, drop=0.165, spacing=0.02)
    dev = torch.device("cuda")
    grads = []
    for ckpt in (1, 7, 20, 60):
        with B.Cloth(inp) as sim:
            k = torch.tensor(inp.k, device=dev, requires_grad=True)
            c = torch.tensor(inp.c, device=dev, requires_grad=True)
            v0 = torch.zeros((inp.n_nodes, 3), device=dev, requires_grad=True)
            x = _rollout(sim, k, c, v0, 60, ckpt, [30, 60])
            w = torch.linspace(-1, 1, x.numel(), device=dev).reshape(x.shape)
            (x * w).sum().backward()
            grads.append([t.grad.cpu().numpy() for t in (k, c, v0)])
    for g in grads[1:]:
        for a, b in zip(g, grads[0]):
            assert np.array_equal(a, b)


def test_gradients_independent_of_the_hit_list_length():
    """The contact search with no hit list, short lists that often overflow to the unlisted
    search, the default and the longest list (which the adjoint's kernels cap at 63 so four
    wavefronts' lists fit 64 KiB) finds the same contacts in the same order, and a forward
    pass on the four-lane kernel steps the same bits: gradients are bit-identical."""
    import torch
    inp = W.small_collision_scene(n=14, freq=5, drop=0.165, spacing=0.02)
    dev = torch.device("cuda")
    grads = []
    for cfg in (dict(hit_slots=32), dict(hit_slots=0), dict(hit_slots=2), dict(hit_slots=64),
                dict(kernel=B.CLOTH_KERNEL_LANES4, hit_slots=8, block_threads=64),
                dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=64),
                dict(kernel=B.CLOTH_KERNEL_GRID, block_threads=128)):
        with B.Cloth(inp) as sim:
            sim.set_launch(**cfg)
            k = torch.tensor(inp.k, device=dev, requires_grad=True)
            c = torch.tensor(inp.c, device=dev, requires_grad=True)
            v0 = torch.zeros((inp.n_nodes, 3), device=dev, requires_grad=True)
            x = _rollout(sim, k, c, v0, 60, 20, [30, 60])
            w = torch.linspace(-1, 1, x.numel(), device=dev).reshape(x.shape)
            (x * w).sum().backward()
            grads.append([t.grad.cpu().numpy() for t in (k, c, v0)])
    assert np.any(grads[0][0] != 0)
    for g in grads[1:]:
        for a, b in zip(g, grads[0]):
            assert np.array_equal(a, b)


def test_backward_without_forward_is_a_state_error():
    inp = W.small_collision_scene(n=8, freq=3)
    with B.Cloth(inp) as sim:
        with pytest.raises(B.ClothError) as ei:
            B.cloth_rollout_backward(sim.h, 0, 0, 0, 0)
        assert ei.value.status == B.CLOTH_ESTATE
