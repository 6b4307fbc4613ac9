"""The complex-gradient convention the autograd binding relies on (CPU).

For a real loss of a complex output a, torch hands backward 2 dL/d conj(a);
the adjoint entry point takes gbar = dL/d conj(a), so the binding halves
what torch passes.  A custom Function written that way must reproduce
torch's own gradient of the same map."""
import torch


def test_torch_passes_twice_the_conjugate_derivative():
    c = torch.tensor([0.3 + 0.7j, -1.1 + 0.2j, 0.4 - 0.9j], dtype=torch.complex128)
    tau = torch.tensor([0.1 - 0.2j, 0.5 + 0.1j, -0.3j], dtype=torch.complex128)
    seen = {}

    class Lin(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x):
            return c * x

        @staticmethod
        def backward(ctx, g):
            seen["g"] = g.clone()
            gbar = g / 2
            return (2 * (gbar.conj() * c).real).sum()

    x = torch.tensor(0.8, dtype=torch.float64, requires_grad=True)
    ((c * x - tau).abs() ** 2).sum().backward()
    native = x.grad.clone()
    x2 = torch.tensor(0.8, dtype=torch.float64, requires_grad=True)
    ((Lin.apply(x2) - tau).abs() ** 2).sum().backward()
    assert torch.allclose(x2.grad, native, rtol=1e-15, atol=0)
    # dL/d conj(a) = a - tau for L = sum |a - tau|^2
    assert torch.allclose(seen["g"], 2 * (c * 0.8 - tau), rtol=1e-15, atol=0)
