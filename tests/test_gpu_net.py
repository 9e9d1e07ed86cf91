"""GPU learned-preconditioner kernels checked against the FP64 network oracle.

Forward and adjoint layers, weight gradients, the loss and its gradient, the
whole network, Adam and the training step, in both field layouts ([nf][V][12]
and right-hand side fastest [V][12][nf]).  The GPU computes in FP32; the bar is
a relative error of 1e-5 for linear maps of one field and 1e-4 for the
reductions (weight gradients, loss), both far above FP32 rounding of sums over
27 hops and a few thousand sites and far below any indexing mistake (which
gives O(1) errors).
"""
import numpy as np
import pytest

from oracle import net as N
from paper_1311_5029_amd import inputs as I

from gpu_util import lib, rel

pytestmark = pytest.mark.gpu

TOL_MAP = 1e-5
TOL_RED = 1e-4


class NetLattice:
    def __init__(self, dims, eps=0.4, seed=81):
        import torch
        self.ok = lib()
        self.torch = torch
        self.dims = tuple(dims)
        self.V = int(np.prod(dims))
        self.U = I.random_su3_links(self.dims, eps, seed)
        self.P = N.all_transports(self.U)
        self.links = self.ok.to_device_complex(self.U)
        self.T = self.ok.empty_bytes(self.ok.ok_net_transports_bytes(self.dims))
        self.ok.ok_net_transports(self.dims, self.links, self.T)

    def up(self, f, inner=False):
        """Host fields (nf, Lt, Lz, Ly, Lx, 4, 3) -> FP32 device buffer in the chosen layout."""
        nf = f.shape[0]
        h = f.reshape(nf, self.V, 12)
        if inner:
            h = np.moveaxis(h, 0, -1)
        return self.ok.to_device_complex(np.ascontiguousarray(h), dtype="float32")

    def down(self, d, nf, inner=False):
        if inner:
            h = self.ok.to_host_complex(d, (self.V, 12, nf))
            h = np.moveaxis(h, -1, 0)
        else:
            h = self.ok.to_host_complex(d, (nf, self.V, 12))
        return np.ascontiguousarray(h).reshape((nf,) + I.lattice_shape(self.dims) + (4, 3))

    def params(self, A):
        return self.ok.to_device_complex(np.ascontiguousarray(A), dtype="float32")

    def sync(self):
        self.torch.cuda.synchronize()


@pytest.fixture(scope="module")
def nl():
    return NetLattice((4, 5, 6, 7))


def rand_A(shape, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


LAYOUTS = [(1, False), (3, False), (5, True), (12, True), (16, True)]
IDS = ["outer1", "outer3", "inner5", "inner12", "inner16"]


def test_each_hop_transport(nl):
    """One-hot layers (A_k = 1 on a single hop) give P_k(x) phi_{x+d_k} for every k: pins the
    transports, the neighbour of every hop and the backward daggers."""
    ok = nl.ok
    phi = I.gaussian_sources(nl.dims, 1, 91)
    d_in = nl.up(phi)
    out = nl.torch.empty_like(d_in)
    for k in range(27):
        A = np.zeros((27, 4, 4), complex)
        A[k] = np.eye(4)
        ok.ok_net_layer(nl.dims, nl.params(A), nl.T, d_in, out, 1, 0)
        nl.sync()
        got = nl.down(out, 1)
        assert rel(got, N.hop(nl.P, k, phi)) < TOL_MAP, k


@pytest.mark.parametrize("nf,inner", LAYOUTS, ids=IDS)
def test_layer_and_adjoint(nl, nf, inner):
    ok = nl.ok
    phi = I.gaussian_sources(nl.dims, nf, 92)
    A = rand_A((27, 4, 4), 93)
    d_in = nl.up(phi, inner)
    out = nl.torch.empty_like(d_in)
    flags = ok.OK_SPINOR_RHS_INNER if inner else 0
    ok.ok_net_layer(nl.dims, nl.params(A), nl.T, d_in, out, nf, flags)
    nl.sync()
    assert rel(nl.down(out, nf, inner), N.layer(nl.P, A, phi)) < TOL_MAP
    ok.ok_net_layer(nl.dims, nl.params(A), nl.T, d_in, out, nf, flags | ok.OK_NET_ADJOINT)
    nl.sync()
    assert rel(nl.down(out, nf, inner), N.layer_adjoint(nl.P, A, phi)) < TOL_MAP


@pytest.mark.parametrize("nf,inner", LAYOUTS, ids=IDS)
def test_weight_gradient(nl, nf, inner):
    ok = nl.ok
    phi = I.gaussian_sources(nl.dims, nf, 94)
    g = I.gaussian_sources(nl.dims, nf, 95)
    flags = ok.OK_SPINOR_RHS_INNER if inner else 0
    gA = nl.torch.empty(27 * 16 * 2, dtype=nl.torch.float32, device="cuda")
    work = ok.empty_bytes(ok.ok_net_workspace_bytes(nl.dims, 1, nf, 2))
    ok.ok_net_layer_wgrad(nl.dims, nl.T, nl.up(g, inner), nl.up(phi, inner), gA, nf, flags, work)
    nl.sync()
    got = ok.to_host_complex(gA, (27, 4, 4))
    want = N.layer_weight_grad(nl.P, g, phi)
    assert rel(got, want) < TOL_RED
    for k in (0, 5, 13, 26):
        assert rel(got[k], want[k]) < TOL_RED, k


def test_weight_gradient_bitwise_reproducible(nl):
    ok = nl.ok
    phi = nl.up(I.gaussian_sources(nl.dims, 3, 96))
    g = nl.up(I.gaussian_sources(nl.dims, 3, 97))
    work = ok.empty_bytes(ok.ok_net_workspace_bytes(nl.dims, 1, 3, 2))
    outs = []
    for _ in range(2):
        gA = nl.torch.empty(27 * 16 * 2, dtype=nl.torch.float32, device="cuda")
        ok.ok_net_layer_wgrad(nl.dims, nl.T, g, phi, gA, 3, 0, work)
        nl.sync()
        outs.append(gA.cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("inner", [False, True], ids=["outer", "inner"])
def test_loss_and_output_gradient(nl, inner):
    ok = nl.ok
    nf = 4
    out = I.gaussian_sources(nl.dims, nf, 98)
    psi = I.gaussian_sources(nl.dims, nf, 99)
    psi[2] *= 3.0
    flags = ok.OK_SPINOR_RHS_INNER if inner else 0
    d_out = nl.up(out, inner)
    gout = nl.torch.empty_like(d_out)
    loss = nl.torch.zeros(1, dtype=nl.torch.float64, device="cuda")
    work = ok.empty_bytes(ok.ok_net_workspace_bytes(nl.dims, 1, nf, 2))
    ok.ok_net_loss_grad(nl.dims, d_out, nl.up(psi, inner), gout, loss, nf, flags, work)
    nl.sync()
    norms = np.array([np.vdot(p, p).real for p in psi])
    diff = out.astype(np.complex64).astype(complex) - psi.astype(np.complex64).astype(complex)
    L = np.mean([np.vdot(d, d).real for d in diff] / norms)
    assert abs(loss.item() - L) / L < 1e-6
    want = diff / (nf * norms[:, None, None, None, None, None, None])
    assert rel(nl.down(gout, nf, inner), want) < TOL_MAP


@pytest.mark.parametrize("nf,inner", [(3, False), (6, True)], ids=["outer3", "inner6"])
def test_network_apply(nl, nf, inner):
    ok = nl.ok
    params = I.net_init_params(4, 0.5, 100, noise=0.1)
    net = ok.Net(4, nl.params(params), nl.T)
    phi = I.gaussian_sources(nl.dims, nf, 101)
    d_in = nl.up(phi, inner)
    out = nl.torch.empty_like(d_in)
    work = ok.empty_bytes(ok.ok_net_workspace_bytes(nl.dims, 4, nf, 0))
    ok.ok_net_apply(nl.dims, net, d_in, out, nf, ok.OK_SPINOR_RHS_INNER if inner else 0, work)
    nl.sync()
    assert rel(nl.down(out, nf, inner), N.forward(nl.P, params, phi)[-1]) < TOL_MAP


@pytest.mark.parametrize("nf,inner", [(2, False), (5, True)], ids=["outer2", "inner5"])
def test_loss_and_parameter_gradient(nl, nf, inner):
    ok = nl.ok
    params = I.net_init_params(3, 0.4, 102, noise=0.1)
    xi = I.gaussian_sources(nl.dims, nf, 103)
    psi = I.gaussian_sources(nl.dims, nf, 104)
    net = ok.Net(3, nl.params(params), nl.T)
    loss = nl.torch.zeros(1, dtype=nl.torch.float64, device="cuda")
    grad = nl.torch.empty(ok.ok_net_param_count(3), dtype=nl.torch.float32, device="cuda")
    work = ok.empty_bytes(ok.ok_net_workspace_bytes(nl.dims, 3, nf, 1))
    ok.ok_net_loss_and_grad(nl.dims, net, nl.up(xi, inner), nl.up(psi, inner), nf,
                            ok.OK_SPINOR_RHS_INNER if inner else 0, loss, grad, work)
    nl.sync()
    L, G = N.loss_and_grad(nl.P, params, xi, psi)
    assert abs(loss.item() - L) / L < TOL_RED
    got = ok.to_host_complex(grad, G.shape)
    assert rel(got, G) < TOL_RED
    for l in range(3):
        assert rel(got[l], G[l]) < TOL_RED, l


def test_adam_matches_oracle():
    ok = lib()
    import torch
    rng = np.random.default_rng(105)
    n = 3 * 27 * 16
    p = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    m = np.zeros(n, complex)
    v = np.zeros(n, complex)
    d_p, d_m, d_v = (ok.to_device_complex(a, dtype="float32") for a in (p, m, v))
    cfg = ok.adam_cfg(lr=1e-2)
    for step in range(1, 4):
        g = 0.1 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
        ok.ok_adam_step(d_p, ok.to_device_complex(g, dtype="float32"), d_m, d_v, 2 * n, cfg, step)
        p, m, v = N.adam_step(p, g.astype(np.complex64).astype(complex), m, v, step, 1e-2)
    torch.cuda.synchronize()
    got = ok.to_host_complex(d_p)
    assert np.max(np.abs(got - p)) < 1e-5


def test_train_step_decreases_loss_and_matches_oracle_step(nl):
    """One fused training step equals the oracle's gradient followed by its Adam step, and ten
    steps follow the oracle's trajectory on pairs (xi, psi = N0 xi) of a fixed target network N0."""
    ok = nl.ok
    torch = nl.torch
    nf = 4
    target = I.net_init_params(2, 0.5, 106, noise=0.2)
    params = I.net_init_params(2, 0.5, 107, noise=0.05)
    xi = I.gaussian_sources(nl.dims, nf, 108)
    psi = N.forward(nl.P, target, xi)[-1]
    d_p = nl.params(params)
    d_m = torch.zeros_like(d_p)
    d_v = torch.zeros_like(d_p)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    grad = torch.empty_like(d_p)
    work = ok.empty_bytes(ok.ok_net_workspace_bytes(nl.dims, 2, nf, 1))
    cfg = ok.adam_cfg(lr=3e-3)
    d_xi, d_psi = nl.up(xi), nl.up(psi)
    ok.ok_net_train_step(nl.dims, 2, d_p, d_m, d_v, nl.T, d_xi, d_psi, nf, 0, cfg, 1, loss, grad, work)
    nl.sync()
    L0, G = N.loss_and_grad(nl.P, params, xi, psi)
    p1, _, _ = N.adam_step(params, G, np.zeros_like(G), np.zeros_like(G), 1, 3e-3)
    assert abs(loss.item() - L0) / L0 < TOL_RED
    # first Adam step moves every coordinate by ~lr sign(g): compare away from tiny gradients
    got = ok.to_host_complex(d_p, params.shape)
    big = (np.abs(G.real) > 1e-3 * np.abs(G).max())
    assert np.max(np.abs(got.real - p1.real)[big]) < 1e-5
    # nine more steps follow the oracle's Adam trajectory (the loss of step t is taken before its update)
    p, m, v = p1, (1 - 0.9) * 2 * G, (1 - 0.999) * ((2 * G.real) ** 2 + 1j * (2 * G.imag) ** 2)
    for step in range(2, 11):
        ok.ok_net_train_step(nl.dims, 2, d_p, d_m, d_v, nl.T, d_xi, d_psi, nf, 0, cfg, step, loss, grad, work)
        Lt, Gt = N.loss_and_grad(nl.P, p, xi, psi)
        p, m, v = N.adam_step(p, Gt, m, v, step, 3e-3)
    nl.sync()
    assert Lt < L0
    assert abs(loss.item() - Lt) / Lt < 1e-3


def test_full_size_layer_sampled():
    """One layer on the 24^3 x 64 lattice (12 fields, right-hand side fastest) against the oracle
    at sampled sites, in the launch configuration of the preconditioned batched solve."""
    ok = lib()
    import torch
    dims = (24, 24, 24, 64)
    V = int(np.prod(dims))
    U = I.random_su3_links(dims, 0.3, 110)
    links = ok.to_device_complex(U)
    T = ok.empty_bytes(ok.ok_net_transports_bytes(dims))
    ok.ok_net_transports(dims, links, T)
    del links
    nf = 12
    phi = (np.random.default_rng(111).standard_normal((V, 12, nf, 2)).astype(np.float32))
    d_in = torch.from_numpy(phi).cuda()
    out = torch.empty_like(d_in)
    A = rand_A((27, 4, 4), 112)
    ok.ok_net_layer(dims, ok.to_device_complex(A, dtype="float32"), T, d_in, out, nf, ok.OK_SPINOR_RHS_INNER)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    rng = np.random.default_rng(113)
    sites = np.concatenate([[0, V - 1, 24 * 24 * 24 * 63 + 23], rng.integers(0, V, 20)])
    shape = I.lattice_shape(dims)
    Lx, Ly, Lz, Lt = dims
    field = phi[..., 0].astype(float) + 1j * phi[..., 1]   # (V, 12, nf)
    for s in sites:
        x, y, z, t = s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz, s // (Lx * Ly * Lz)
        # a 5^4 window around the site holds every hop and every transport path
        idx = np.ix_(*[(np.arange(-2, 3) + c) % L for c, L in zip((t, z, y, x), (Lt, Lz, Ly, Lx))])
        Uw = U[idx]
        fw = field.reshape(shape + (12, nf))[idx]
        fw = np.moveaxis(fw, -1, 0).reshape((nf, 5, 5, 5, 5, 4, 3))
        # a periodic 5^4 window reproduces every hop of the centre: all paths stay within +-2
        Pw = N.all_transports(Uw)
        want = N.layer(Pw, A, fw)[:, 2, 2, 2, 2]
        g = got[s, :, :, 0] + 1j * got[s, :, :, 1]      # (12, nf)
        assert rel(np.moveaxis(g, -1, 0).reshape(nf, 4, 3), want) < TOL_MAP, s


@pytest.mark.parametrize("dims", [(3, 3, 3, 3), (4, 3, 5, 4), (5, 4, 3, 6)], ids=["3^4", "4x3x5x4", "5x4x3x6"])
def test_small_lattices_coinciding_hops(dims):
    """At L = 3 the hops +2 and -1 (and -2 and +1) reach the same site and at L = 4 the hops +2 and -2
    do; the layer must still be the plain sum over the 27 hops (both layouts, and the adjoint)."""
    L = NetLattice(dims, eps=0.5, seed=120)
    ok = L.ok
    A = rand_A((27, 4, 4), 121)
    for nf, inner in ((2, False), (5, True)):
        phi = I.gaussian_sources(L.dims, nf, 122)
        d_in = L.up(phi, inner)
        out = L.torch.empty_like(d_in)
        fl = ok.OK_SPINOR_RHS_INNER if inner else 0
        ok.ok_net_layer(L.dims, L.params(A), L.T, d_in, out, nf, fl)
        L.sync()
        assert rel(L.down(out, nf, inner), N.layer(L.P, A, phi)) < TOL_MAP
        ok.ok_net_layer(L.dims, L.params(A), L.T, d_in, out, nf, fl | ok.OK_NET_ADJOINT)
        L.sync()
        assert rel(L.down(out, nf, inner), N.layer_adjoint(L.P, A, phi)) < TOL_MAP


@pytest.mark.parametrize("n_layers", [1, 2, 3, 16])
def test_network_depths(nl, n_layers):
    """One layer (no work buffer), two (one ping-pong field), three and sixteen (both alternate)."""
    ok = nl.ok
    params = I.net_init_params(n_layers, 0.7, 130 + n_layers, noise=0.05)
    net = ok.Net(n_layers, nl.params(params), nl.T)
    phi = I.gaussian_sources(nl.dims, 2, 131)
    d_in = nl.up(phi)
    out = nl.torch.empty_like(d_in)
    nb = ok.ok_net_workspace_bytes(nl.dims, n_layers, 2, 0)
    work = ok.empty_bytes(nb)
    ok.ok_net_apply(nl.dims, net, d_in, out, 2, 0, work)
    nl.sync()
    assert rel(nl.down(out, 2), N.forward(nl.P, params, phi)[-1]) < 4 * TOL_MAP


def test_gauge_covariance_on_gpu():
    """The GPU network on gauge-transformed links and fields equals the transformed output."""
    dims = (4, 5, 4, 6)
    U = I.random_su3_links(dims, 0.4, 140)
    g = I.random_su3_field(dims, 141)
    ok = lib()
    import torch
    params = I.net_init_params(2, 0.6, 142, noise=0.1)
    phi = I.gaussian_sources(dims, 1, 143)
    from oracle.lattice import cmul
    outs = []
    for links, f in ((U, phi), (I.gauge_transform_links(U, g), cmul(g, phi))):
        T = ok.empty_bytes(ok.ok_net_transports_bytes(dims))
        ok.ok_net_transports(dims, ok.to_device_complex(links), T)
        net = ok.Net(2, ok.to_device_complex(params, dtype="float32"), T)
        d_in = ok.to_device_complex(f, dtype="float32")
        out = torch.empty_like(d_in)
        ok.ok_net_apply(dims, net, d_in, out, 1, 0, ok.empty_bytes(ok.ok_net_workspace_bytes(dims, 2, 1, 0)))
        torch.cuda.synchronize()
        outs.append(ok.to_host_complex(out, f.shape))
    assert rel(outs[1], cmul(g, outs[0])) < 1e-5


def test_training_checkpoint_resume_is_bit_identical(nl, tmp_path):
    """Training interrupted after 7 of 16 steps, checkpointed and resumed from the file gives the
    same parameters, Adam moments and loss history as the uninterrupted run, bit for bit (the
    step fixes the mini-batch and the learning rate; the reductions have a fixed order)."""
    from paper_1311_5029_amd import train as TR
    ok = nl.ok
    nf = 8
    target = I.net_init_params(2, 0.5, 116, noise=0.2)
    xi = I.gaussian_sources(nl.dims, nf, 117)
    psi = N.forward(nl.P, target, xi)[-1]
    d_xi, d_psi = nl.up(xi), nl.up(psi)
    kw = dict(n_layers=2, steps=16, batch=4, lr=3e-3, log_every=1)
    full_ck = str(tmp_path / "full.npz")
    net_a, hist_a = TR.train(nl.dims, nl.T, d_xi, d_psi, nf, 0.5, checkpoint=full_ck, **kw)
    part_ck = str(tmp_path / "part.npz")
    TR.train(nl.dims, nl.T, d_xi, d_psi, nf, 0.5, checkpoint=part_ck, stop_after=7, **kw)
    st = TR.load_checkpoint(part_ck)
    assert st["step"] == 7 and len(st["history"]) == 7
    net_b, hist_b = TR.train(nl.dims, nl.T, d_xi, d_psi, nf, 0.5, checkpoint=part_ck, resume=part_ck, **kw)
    nl.sync()
    assert hist_a == hist_b
    assert np.array_equal(net_a.params.cpu().numpy(), net_b.params.cpu().numpy())
    a, b = TR.load_checkpoint(full_ck), TR.load_checkpoint(part_ck)
    assert a["step"] == b["step"] == 16
    for k in ("params", "adam_m", "adam_v"):
        assert np.array_equal(a[k], b[k]), k
    with pytest.raises(ValueError):
        TR.train(nl.dims, nl.T, d_xi, d_psi, nf, 0.5, resume=part_ck, **dict(kw, lr=1e-3))
