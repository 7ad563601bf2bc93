"""GPU adjoint (HIP rollout forward + hand-written backward, through ClothRollout) against
the FP64 oracle.

With collision, a resting node sits exactly at the thickness after every push, so FP32 and
FP64 runs take different contact decisions at many nodes and their rollouts lie on different
smooth pieces.  The reference adjoint is therefore the oracle's adjoint evaluated on the
GPU's own trajectory with the GPU's own contact sets (cloth_debug_contacts), which isolates
the adjoint arithmetic.  Without collision the trajectories agree and the GPU gradient is
also checked against central differences of the FP64 oracle forward (h = 1e-3 relative).
Bar: 1e-3 relative (normwise for whole gradients; per entry, with a floor of 1e-3 of the
largest entry, for differences)."""
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


def _oracle_adjoint_on_gpu_trajectory(inp, n_steps, target):
    """Step the GPU substep by substep, recording its states and contact sets, then run the
    oracle's substep adjoint backwards along them."""
    h = h32(inp)
    n_sub = n_steps * inp.n_substeps
    xs, vs, cs = [], [], []
    with B.Cloth(inp) as sim:
        for _ in range(n_sub):
            x, v = sim.read_state()
            xs.append(x)
            vs.append(v)
            cs.append(sim.debug_contacts(h) if inp.thickness > 0 else [[]] * inp.n_nodes)
            sim.step(dt=h, n_substeps=1, n_steps=1)
        xT, _ = sim.read_state()
    m = oracle.Model.from_inputs(inp)
    xb = (2.0 / inp.n_nodes) * (xT.astype(np.float64) - target)
    vb = np.zeros_like(xb)
    gk, gc = np.zeros(inp.n_springs), np.zeros(inp.n_springs)
    contacts = 0
    for n in range(n_sub - 1, -1, -1):
        contacts += sum(1 for c in cs[n] if c)
        xb, vb, kb, cb = m.substep_vjp_given(xs[n], vs[n], h, cs[n], xb, vb)
        gk += kb
        gc += cb
    return gk, gc, vb, xT, contacts


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


@pytest.mark.parametrize("scene", ["small", "config4"])
def test_gradients_match_oracle_adjoint_on_gpu_contact_sets(scene):
    if scene == "small":
        inp, n_steps = W.small_collision_scene(n=14, freq=5, drop=0.165, spacing=0.02), 60
    else:
        inp, _ = W.config4()
        n_steps = inp.n_steps  # 200 frames x 4 substeps, checkpoints every 20 frames
    target = _target(inp, n_steps)
    gk, gc, gv, xT = _gpu_grads(inp, n_steps, target)
    rk, rc, rv, xT2, contacts = _oracle_adjoint_on_gpu_trajectory(inp, n_steps, target)
    assert np.array_equal(xT, xT2)
    assert contacts > 100
    for name, a, b in (("k", gk, rk), ("c", gc, rc), ("v0", gv, rv)):
        err = _normwise(a, b)
        print(f"{scene} {name}: normwise relative error {err:.2e} (|g| = {np.linalg.norm(b):.3e})")
        assert err <= 1e-3, name


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
    wavefronts' lists fit 64 KiB) finds the same contacts in the same order: gradients are
    bit-identical."""
    import torch
    inp = W.small_collision_scene(n=14, freq=5, drop=0.165, spacing=0.02)
    dev = torch.device("cuda")
    grads = []
    for slots in (32, 0, 2, 64):
        with B.Cloth(inp) as sim:
            sim.set_launch(hit_slots=slots)
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
