"""Host logic of the force-matching autograd wrappers (no GPU): each call's backward uses the
coefficients, saved forward state and cotangent of that call, even when other forward passes
ran in between, and the loss's upstream gradient scales the result.  The device calls are replaced by a stand-in batch whose forces are a known function
of the coefficients."""
import torch

from paper_2511_22951_amd import fm, md


class _Batch:
    """forces: f = A (c * c) as [3, n]; saved = the first 3 n coefficients (so the backward
    can tell which forward pass it belongs to); backward: d(sum f . G)/dc = 2 c (A^T G)."""

    def __init__(self, n, n_coef, seed=0):
        g = torch.Generator().manual_seed(seed)
        self.n = n
        self.A = torch.randn(3 * n, n_coef, generator=g, dtype=torch.float64)
        self.saved = torch.zeros(3, n, dtype=torch.float64)

    def forces(self, pot, saved=True):
        c = torch.cat(pot.coef)
        if saved:
            self.saved.copy_(c[:3 * self.n].reshape(3, self.n))
        return (self.A @ (c * c)).reshape(3, self.n)

    def loss(self, pot, f_ref, saved, grad_force):
        f = self.forces(pot, saved=False)
        saved.copy_(torch.cat(pot.coef)[:3 * self.n].reshape(3, self.n))
        grad_force.copy_(2.0 * (f - f_ref) / self.n)
        return ((f - f_ref) ** 2).sum() / self.n

    def backward(self, pot, grad_force, saved=None):
        c = torch.cat(pot.coef)
        s = self.saved if saved is None else saved
        assert torch.equal(s.reshape(-1), c[:3 * self.n]), "saved state of another forward"
        return 2.0 * c * (self.A.t() @ grad_force.reshape(-1))


def _pot(n_each=8):
    z = [torch.zeros(n_each, dtype=torch.float64) for _ in range(3)]
    return md.EAMPotential(*z, 1.0, 0.1, 1.0, 0.1, 1.5, device="cpu")


def test_backward_after_a_second_forward_uses_its_own_call():
    pot = _pot()
    batch = _Batch(n=4, n_coef=24)
    g = torch.Generator().manual_seed(1)
    c1 = torch.randn(24, generator=g, dtype=torch.float64, requires_grad=True)
    c2 = torch.randn(24, generator=g, dtype=torch.float64, requires_grad=True)
    w = torch.randn(3, 4, generator=g, dtype=torch.float64)
    f1 = fm.EAMForces.apply(c1, batch, pot)
    f2 = fm.EAMForces.apply(c2, batch, pot)
    v2 = pot.version
    (f1 * w).sum().backward()
    assert torch.allclose(c1.grad, 2.0 * c1.detach() * (batch.A.t() @ w.reshape(-1)))
    # the later coefficients, their version and their own backward are untouched
    assert torch.equal(torch.cat(pot.coef), c2.detach()) and pot.version == v2
    (f2 * w).sum().backward()
    assert torch.allclose(c2.grad, 2.0 * c2.detach() * (batch.A.t() @ w.reshape(-1)))


def test_backward_right_after_forward():
    pot = _pot()
    batch = _Batch(n=4, n_coef=24, seed=3)
    c = torch.linspace(-1, 1, 24, dtype=torch.float64, requires_grad=True)
    f_ref = torch.zeros(3, 4, dtype=torch.float64)
    loss = fm.force_matching_loss(c, batch, pot, f_ref)
    loss.backward()
    f = batch.A @ (c.detach() ** 2)
    want = 2.0 * c.detach() * (batch.A.t() @ (2.0 * f / batch.n))
    assert torch.allclose(c.grad, want)


def test_fused_loss_backward_after_a_second_loss_uses_its_own_call():
    pot = _pot()
    batch = _Batch(n=4, n_coef=24, seed=5)
    g = torch.Generator().manual_seed(6)
    c1 = torch.randn(24, generator=g, dtype=torch.float64, requires_grad=True)
    c2 = torch.randn(24, generator=g, dtype=torch.float64, requires_grad=True)
    f_ref = torch.randn(3, 4, generator=g, dtype=torch.float64)
    l1 = fm.force_matching_loss(c1, batch, pot, f_ref)
    l2 = fm.force_matching_loss(c2, batch, pot, f_ref)
    v2 = pot.version
    (3.0 * l1).backward()  # upstream gradient 3
    f1 = batch.A @ (c1.detach() ** 2)
    want1 = 3.0 * 2.0 * c1.detach() * (batch.A.t() @ (2.0 * (f1 - f_ref.reshape(-1)) / batch.n))
    assert torch.allclose(c1.grad, want1)
    assert torch.equal(torch.cat(pot.coef), c2.detach()) and pot.version == v2
    l2.backward()
    f2 = batch.A @ (c2.detach() ** 2)
    want2 = 2.0 * c2.detach() * (batch.A.t() @ (2.0 * (f2 - f_ref.reshape(-1)) / batch.n))
    assert torch.allclose(c2.grad, want2)
    assert torch.allclose(l1.detach(), ((f1 - f_ref.reshape(-1)) ** 2).sum() / batch.n)
