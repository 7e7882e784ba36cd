"""Seeded synthetic SU(3) link fields in the canonical boundary layout.

This module is shared input tooling: it draws random numbers and builds
link matrices, and holds none of the flow's arithmetic (no staples, forces,
integrator or observables).  Both the GPU library and the CPU oracle are fed
from the arrays it returns.

Canonical layout (the C-ABI's): complex128, C-contiguous, shape
``[d3, d2, d1, d0, 4, 3, 3]`` -- site index ``n0 + d0*(n1 + d1*(n2 + d2*n3))``
with ``n0`` fastest, then the direction ``mu = 0..3``, then a row-major 3x3
matrix.  ``dims = (d0, d1, d2, d3)``; the twisted short-short plane is (0, 1)
(the paper's (1, 2) plane of an L x L x 3L x 3L box, section 3.1).

Generators (all seeded, all return SU(3) to rounding):

* ``identity``      -- the free vacuum (every link = 1).
* ``near_identity`` -- U = exp(i * eps * H), H = sum_a h_a lambda_a / 2 with
  Gell-Mann matrices lambda_a and h_a ~ N(0, 1) i.i.d. per link.
* ``haar``          -- Haar-distributed SU(3) (hot start): Gram-Schmidt on two
  complex Gaussian rows (Haar on the first two rows of U(3)), third row the
  conjugated cross product, which fixes det = 1 and keeps right invariance.

SU(N) fields (layout ``[d3, d2, d1, d0, 4, N, N]``, 2 <= N):

* ``identity_n``      -- every link = 1.
* ``near_identity_n`` -- U = exp(i * eps * H), H = (A + A^+)/2 made traceless,
  A with i.i.d. complex Gaussian entries (each of re, im ~ N(0, 1/2)).
* ``haar_n``          -- QR of a complex Gaussian matrix with the phases of
  R's diagonal moved into Q (Haar on U(N)), times det^(-1/N) (Haar on SU(N)).

Random numbers come from ``torch.Generator(device).manual_seed(seed)`` so the
same (seed, device) pair always reproduces the same field.
"""

from __future__ import annotations

import math

import torch

__all__ = ["lattice_shape", "identity", "near_identity", "haar", "su3_haar",
           "gell_mann", "identity_n", "near_identity_n", "haar_n"]


def lattice_shape(dims):
    d0, d1, d2, d3 = (int(x) for x in dims)
    if min(d0, d1, d2, d3) < 1:
        raise ValueError(f"bad lattice dims {dims}")
    return (d3, d2, d1, d0)


def gell_mann(device="cpu"):
    """The eight Gell-Mann matrices, shape [8, 3, 3] complex128."""
    lam = torch.zeros(8, 3, 3, dtype=torch.complex128)
    lam[0, 0, 1] = lam[0, 1, 0] = 1
    lam[1, 0, 1] = -1j
    lam[1, 1, 0] = 1j
    lam[2, 0, 0] = 1
    lam[2, 1, 1] = -1
    lam[3, 0, 2] = lam[3, 2, 0] = 1
    lam[4, 0, 2] = -1j
    lam[4, 2, 0] = 1j
    lam[5, 1, 2] = lam[5, 2, 1] = 1
    lam[6, 1, 2] = -1j
    lam[6, 2, 1] = 1j
    lam[7, 0, 0] = lam[7, 1, 1] = 1 / math.sqrt(3)
    lam[7, 2, 2] = -2 / math.sqrt(3)
    return lam.to(device)


def _gen(seed, device):
    g = torch.Generator(device=torch.device(device))
    g.manual_seed(int(seed))
    return g


def identity(dims, device="cpu"):
    shape = lattice_shape(dims) + (4,)
    eye = torch.eye(3, dtype=torch.complex128, device=device)
    return eye.expand(shape + (3, 3)).contiguous()


def near_identity(dims, eps, seed, device="cpu", chunk=1 << 21):
    """U = exp(i*eps*H) per link, H a Gaussian traceless Hermitian matrix."""
    shape = lattice_shape(dims) + (4,)
    n = math.prod(shape)
    g = _gen(seed, device)
    h = torch.randn(n, 8, dtype=torch.float64, device=device, generator=g)
    lam = gell_mann(device)
    out = torch.empty(n, 3, 3, dtype=torch.complex128, device=device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        H = torch.einsum("na,aij->nij", h[s:e].to(torch.complex128), lam) * 0.5
        out[s:e] = torch.linalg.matrix_exp(1j * float(eps) * H)
    return out.reshape(shape + (3, 3))


def su3_haar(n, seed, device="cpu", generator=None):
    """n Haar-random SU(3) matrices, shape [n, 3, 3] complex128."""
    g = generator if generator is not None else _gen(seed, device)
    z = torch.randn(n, 2, 3, 2, dtype=torch.float64, device=device, generator=g)
    z = torch.view_as_complex(z)
    r0 = z[:, 0]
    r0 = r0 / torch.linalg.vector_norm(r0, dim=-1, keepdim=True)
    r1 = z[:, 1]
    r1 = r1 - (r0.conj() * r1).sum(-1, keepdim=True) * r0
    r1 = r1 / torch.linalg.vector_norm(r1, dim=-1, keepdim=True)
    r2 = torch.stack([r0[:, 1] * r1[:, 2] - r0[:, 2] * r1[:, 1],
                      r0[:, 2] * r1[:, 0] - r0[:, 0] * r1[:, 2],
                      r0[:, 0] * r1[:, 1] - r0[:, 1] * r1[:, 0]], dim=-1).conj()
    return torch.stack([r0, r1, r2], dim=1)


def haar(dims, seed, device="cpu", chunk=1 << 22):
    """Haar-random SU(3) hot start.  Each chunk of `chunk` links draws its own
    normals, so the links depend on (seed, chunk, device)."""
    shape = lattice_shape(dims) + (4,)
    n = math.prod(shape)
    g = _gen(seed, device)
    out = torch.empty(n, 3, 3, dtype=torch.complex128, device=device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        out[s:e] = su3_haar(e - s, None, device, generator=g)
    return out.reshape(shape + (3, 3))


def identity_n(dims, N, device="cpu"):
    shape = lattice_shape(dims) + (4,)
    eye = torch.eye(int(N), dtype=torch.complex128, device=device)
    return eye.expand(shape + (int(N), int(N))).contiguous()


def near_identity_n(dims, N, eps, seed, device="cpu", chunk=1 << 20):
    """SU(N): U = exp(i*eps*H) per link, H a Gaussian traceless Hermitian matrix."""
    N = int(N)
    shape = lattice_shape(dims) + (4,)
    n = math.prod(shape)
    g = _gen(seed, device)
    out = torch.empty(n, N, N, dtype=torch.complex128, device=device)
    eye = torch.eye(N, dtype=torch.complex128, device=device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        a = torch.randn(e - s, N, N, 2, dtype=torch.float64, device=device, generator=g)
        A = torch.view_as_complex(a) * math.sqrt(0.5)
        H = 0.5 * (A + A.conj().transpose(-1, -2))
        H = H - (torch.diagonal(H, dim1=-2, dim2=-1).sum(-1) / N)[:, None, None] * eye
        out[s:e] = torch.linalg.matrix_exp(1j * float(eps) * H)
    return out.reshape(shape + (N, N))


def haar_n(dims, N, seed, device="cpu", chunk=1 << 20):
    """Haar-random SU(N) hot start."""
    N = int(N)
    shape = lattice_shape(dims) + (4,)
    n = math.prod(shape)
    g = _gen(seed, device)
    out = torch.empty(n, N, N, dtype=torch.complex128, device=device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        z = torch.randn(e - s, N, N, 2, dtype=torch.float64, device=device, generator=g)
        Z = torch.view_as_complex(z)
        Q, R = torch.linalg.qr(Z)
        d = torch.diagonal(R, dim1=-2, dim2=-1)
        Q = Q * (d / d.abs())[:, None, :]
        det = torch.linalg.det(Q)
        out[s:e] = Q * (det ** (-1.0 / N))[:, None, None]
    return out.reshape(shape + (N, N))
