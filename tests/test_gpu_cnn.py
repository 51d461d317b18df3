"""Warm-start network kernels against the float64 reference.

The GPU computes in bfloat16 (weights, activations and gradients rounded to
bfloat16, float32 accumulation); the reference is evaluated on the same
bfloat16-rounded weights and input.  Six layers of bfloat16 rounding bound
the relative error of the network output by a few 2^-8; tolerances are 2e-2
(output) and 5e-2 (gradients), far below the O(1) error of a wrong tap,
transposition or mask."""
import sys

import numpy as np
import pytest

from oracle import cnn
import _util as U

pytestmark = pytest.mark.gpu


def flat(params):
    return np.concatenate([np.concatenate([p["w"].reshape(-1), p["b"]]) for p in params]).astype(np.float32)


def unflat(v):
    out, i = [], 0
    for l in range(6):
        ci, co = cnn.CHANNELS[l], cnn.CHANNELS[l + 1]
        w = v[i:i + co * 9 * ci].reshape(co, 3, 3, ci).astype(np.float64)
        i += co * 9 * ci
        b = v[i:i + co].astype(np.float64)
        i += co
        out.append({"w": w, "b": b})
    return out


def random_params(seed, last_scale=0.1):
    rng = np.random.default_rng(seed)
    params = cnn.init_params(rng)
    params[-1]["w"] = rng.standard_normal(params[-1]["w"].shape) * last_scale / 17
    for p in params:
        p["b"] = rng.standard_normal(p["b"].shape) * 0.05
    return params


def images(seed, N, I1, I2):
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, (N, 3, I2, I1)).astype(np.float32)


def to_oracle(img):           # (3, I2, I1) -> (I1, I2, 3)
    return np.asarray(img, np.float64).transpose(2, 1, 0)


def banner(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("shape", [(2, 40, 22), (1, 128, 128)])
def test_forward_matches_reference(shape):
    import torch
    from paper_2603_00839_amd import rtg
    banner("cnn forward", shape)
    N, I1, I2 = shape
    params = random_params(0)
    net = rtg.WarmStartNet(flat(params))
    pq = unflat(U.bf16_round(flat(params)))
    C = images(1, N, I1, I2)
    X0 = net.forward(torch.from_numpy(C).cuda()).cpu().numpy()
    for n in range(N):
        c = to_oracle(C[n])
        ref_x0, _ = cnn.forward(pq, U.bf16_round(c).reshape(c.shape))
        f_ref = ref_x0 - U.bf16_round(c).reshape(c.shape)
        f_gpu = to_oracle(X0[n]) - c
        assert U.rel(f_gpu, f_ref) < 2e-2


def test_zero_last_layer_gives_observation_exactly():
    import torch
    from paper_2603_00839_amd import rtg
    banner("cnn zero last layer")
    params = cnn.init_params(np.random.default_rng(3))
    net = rtg.WarmStartNet(flat(params))
    C = torch.from_numpy(images(2, 2, 64, 20)).cuda()
    X0 = net.forward(C)
    assert torch.equal(X0, C)


def test_gradients_match_reference():
    import torch
    from paper_2603_00839_amd import rtg
    banner("cnn gradients")
    N, I1, I2 = 2, 48, 20
    params = random_params(4, last_scale=1.0)
    net = rtg.WarmStartNet(flat(params))
    pq = unflat(U.bf16_round(flat(params)))
    C = images(5, N, I1, I2)
    Y = C + 0.1 * np.random.default_rng(6).standard_normal(C.shape).astype(np.float32)
    loss = net.gradients(torch.from_numpy(C).cuda(), torch.from_numpy(Y).cuda())
    g_gpu = unflat(net.read_gradients())
    # reference: mean over the whole batch = average of per-image means
    g_ref = None
    sse = 0.0
    for n in range(N):
        c = to_oracle(C[n])
        x0, acts = cnn.forward(pq, U.bf16_round(c).reshape(c.shape))
        x0 = x0 - U.bf16_round(c).reshape(c.shape) + c          # residual uses the float32 C
        acts[0] = U.bf16_round(c).reshape(c.shape)
        y = to_oracle(Y[n])
        sse += float(np.sum((x0 - y) ** 2))
        # backward with the residual of the float32 C: dL/dX0 is the same formula
        acts_r = list(acts)
        acts_r[-1] = x0 - acts[0]
        gr = cnn.backward(pq, acts_r, y)
        gr = [{k: v / N for k, v in g.items()} for g in gr]
        g_ref = gr if g_ref is None else [{k: a[k] + b[k] for k in a} for a, b in zip(g_ref, gr)]
    np.testing.assert_allclose(float(loss.item()), sse, rtol=2e-2)
    for l in range(6):
        for k in ("w", "b"):
            r = U.rel(g_gpu[l][k], g_ref[l][k])
            print(f"layer {l} {k}: rel {r:.3e}", file=sys.stderr)
            assert r < 5e-2, (l, k, r)


def test_adam_step_matches_reference():
    import torch
    from paper_2603_00839_amd import rtg
    banner("cnn adam")
    params = random_params(7, last_scale=1.0)
    net = rtg.WarmStartNet(flat(params))
    C = torch.from_numpy(images(8, 1, 32, 16)).cuda()
    Y = C * 0.9
    net.gradients(C, Y)
    g = unflat(net.read_gradients())
    net.adam(1e-3)
    after = unflat(net.export())
    ref = [{k: v.copy() for k, v in p.items()} for p in unflat(flat(params))]
    opt = cnn.Adam(ref, lr=1e-3)
    opt.step(ref, g)
    for l in range(6):
        for k in ("w", "b"):
            np.testing.assert_allclose(after[l][k], ref[l][k], rtol=1e-5, atol=1e-7)


def test_training_reduces_the_loss():
    import torch
    from paper_2603_00839_amd import rtg
    banner("cnn training")
    params = cnn.init_params(np.random.default_rng(9))
    net = rtg.WarmStartNet(flat(params))
    rng = np.random.default_rng(10)
    C = torch.from_numpy(images(11, 4, 64, 64)).cuda()
    # a smooth target the network can learn: a fixed local average of C
    Y = (C + torch.roll(C, 1, dims=3) + torch.roll(C, -1, dims=3)) / 3.0
    losses = []
    for it in range(60):
        losses.append(float(net.train_step(C, Y.contiguous(), 3e-3).item()))
    print("losses", losses[0], losses[-1], file=sys.stderr)
    assert losses[-1] < 0.5 * losses[0]


def test_adam_four_steps_match_reference():
    """Four k_adam steps with a different gradient each (new data per step)
    and a changing learning rate, against the float64 Adam fed with the same
    gradients: the moments must decay and bias-correct across steps (from
    step 2 on the update is no longer lr g / |g|)."""
    import torch
    from paper_2603_00839_amd import rtg
    banner("cnn adam, four steps")
    params = random_params(12, last_scale=1.0)
    net = rtg.WarmStartNet(flat(params))
    ref = [{k: v.copy() for k, v in p.items()} for p in unflat(flat(params))]
    opt = cnn.Adam(ref)
    rng = np.random.default_rng(13)
    for k, lr in enumerate((1e-3, 2e-3, 5e-4, 1e-3)):
        C = torch.from_numpy(images(30 + k, 1, 32, 16)).cuda()
        Y = (C * float(rng.uniform(0.7, 1.1))).contiguous()
        net.gradients(C, Y)
        g = unflat(net.read_gradients())
        net.adam(lr)
        opt.step(ref, g, lr=lr)
    after = unflat(net.export())
    for l in range(6):
        for k in ("w", "b"):
            np.testing.assert_allclose(after[l][k], ref[l][k], rtol=1e-5, atol=1e-7)
