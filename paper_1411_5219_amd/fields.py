"""Device buffers for the library's fields (torch allocations + ABI pack calls).

Only allocation and host <-> device transfer happen here; layout changes
run in the library's pack / unpack kernels.
"""

from __future__ import annotations

import math

import numpy as np
import torch

from . import lqcd as L


class Lattice:
    def __init__(self, extents, theta=(0.0, 0.0, 0.0, math.pi), device="cuda:0"):
        self.L = tuple(int(v) for v in extents)
        self.theta = tuple(float(t) for t in theta)
        self.g = L.geom(self.L, self.theta)
        self.V = int(np.prod(self.L))
        self.device = torch.device(device)

    def nbytes(self, kind, prec, recon=18):
        return L.lqcd_field_bytes(self.g, kind, prec, recon)

    def empty(self, kind, prec, recon=18, nrhs=1):
        n = self.nbytes(kind, prec, recon) * nrhs
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def zeros(self, kind, prec, recon=18, nrhs=1):
        return self.empty(kind, prec, recon, nrhs).zero_()

    def gauge(self, U, prec=64, recon=18, stream=None):
        """Canonical complex128 (4, V, 3, 3) numpy or torch -> internal field."""
        Ut = torch.as_tensor(np.ascontiguousarray(U)) if isinstance(U, np.ndarray) else U
        Ud = Ut.to(self.device, dtype=torch.complex128).contiguous()
        out = self.empty(L.FIELD_GAUGE, prec, recon)
        L.lqcd_pack_gauge(self.g, prec, recon, Ud, out, stream)
        return out

    def spinor(self, psi, prec=64, stream=None):
        """Canonical complex128 (V,4,3) or (nrhs,V,4,3) -> internal full-lattice fields."""
        pt = torch.as_tensor(np.ascontiguousarray(psi)) if isinstance(psi, np.ndarray) else psi
        pd = pt.to(self.device, dtype=torch.complex128).contiguous()
        nrhs = 1 if pd.dim() == 3 else pd.shape[0]
        out = self.empty(L.FIELD_SPINOR_FULL, prec, nrhs=nrhs)
        L.lqcd_pack_spinor(self.g, prec, nrhs, pd, out, stream)
        return out

    def unpack(self, field, prec=64, nrhs=1, stream=None, numpy=True):
        shape = (self.V, 4, 3) if nrhs == 1 else (nrhs, self.V, 4, 3)
        out = torch.empty(shape, dtype=torch.complex128, device=self.device)
        L.lqcd_unpack_spinor(self.g, prec, nrhs, field, out, stream)
        if numpy:
            torch.cuda.synchronize(self.device)
            return out.cpu().numpy()
        return out

    def parity_view(self, full, parity, prec=64, nrhs=1):
        """The parity half of full-lattice fields, as separate tensors per rhs
        stacked into one contiguous parity field buffer (a copy)."""
        pb = self.nbytes(L.FIELD_SPINOR_PARITY, prec)
        f = full.view(nrhs, 2, pb)[:, parity, :]
        return f.contiguous().view(-1)

    def workspace(self, op, params=None):
        n = L.lqcd_workspace_bytes(self.g, op, params)
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def colour(self, chi, prec=64, stream=None):
        """Canonical complex128 (V,3) or (nrhs,V,3) -> internal full-lattice colour fields."""
        pt = torch.as_tensor(np.ascontiguousarray(chi)) if isinstance(chi, np.ndarray) else chi
        pd = pt.to(self.device, dtype=torch.complex128).contiguous()
        nrhs = 1 if pd.dim() == 2 else pd.shape[0]
        out = self.empty(L.FIELD_COLOUR_FULL, prec, nrhs=nrhs)
        L.lqcd_pack_colour(self.g, prec, nrhs, pd, out, stream)
        return out

    def unpack_colour(self, field, prec=64, nrhs=1, stream=None, numpy=True):
        shape = (self.V, 3) if nrhs == 1 else (nrhs, self.V, 3)
        out = torch.empty(shape, dtype=torch.complex128, device=self.device)
        L.lqcd_unpack_colour(self.g, prec, nrhs, field, out, stream)
        if numpy:
            torch.cuda.synchronize(self.device)
            return out.cpu().numpy()
        return out

    def colour_parity(self, full, parity, prec=64, nrhs=1):
        """The parity half of full-lattice colour fields, stacked per rhs (a copy)."""
        pb = self.nbytes(L.FIELD_COLOUR_PARITY, prec)
        return full.view(nrhs, 2, pb)[:, parity, :].contiguous().view(-1)

    def stag_workspace(self, op, nshift=0):
        n = L.lqcd_workspace_bytes_stag(self.g, op, nshift)
        return torch.empty(n, dtype=torch.uint8, device=self.device)
