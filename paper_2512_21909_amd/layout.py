"""Layout queries and host-side marshalling between per-block arrays and the
library's flat storage (offsets come from ``cdcc_irrep_layout``)."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib


class Layout:
    """Result of ``cdcc_irrep_layout`` for one symmetry shape."""

    def __init__(self, sym: dict):
        lib = _lib.load()
        s = _lib.Sym()
        h = int(sym["h"])
        s.nirrep = h
        for g in range(h):
            s.nocc[g], s.nvir[g], s.ncd[g] = int(sym["nocc"][g]), int(sym["nvir"][g]), int(sym["ncd"][g])
        self.c = _lib.LayoutC()
        _lib.check(lib.cdcc_irrep_layout(ctypes.byref(s), ctypes.byref(self.c)), "cdcc_irrep_layout")
        self.sym = {"h": h, "nocc": list(sym["nocc"]), "nvir": list(sym["nvir"]), "ncd": list(sym["ncd"])}
        self.h = h
        c = self.c
        r8 = lambda a: [int(a[g]) for g in range(h)]
        r88 = lambda a: [[int(a[i][j]) for j in range(h)] for i in range(h)]
        self.n_oo, self.n_vv = r8(c.n_oo), r8(c.n_vv)
        self.n_oo_pk, self.n_vv_pk = r8(c.n_oo_pk), r8(c.n_vv_pk)
        self.amp_off = r8(c.amp_off)
        self.oo_off, self.vv_off = r88(c.oo_off), r88(c.vv_off)
        self.b_off, self.bvo_off = r88(c.b_off), r88(c.bvo_off)
        self.t1_off, self.occ_off, self.vir_off, self.cd_off = r8(c.t1_off), r8(c.occ_off), r8(c.vir_off), r8(c.cd_off)
        self.amp_size, self.b_size, self.bvo_size, self.t1_size = c.amp_size, c.b_size, c.bvo_size, c.t1_size
        self.nocc_tot, self.nvir_tot, self.ncd_tot = c.nocc_tot, c.nvir_tot, c.ncd_tot
        v = self.vo = _lib.VoLayoutC()
        _lib.check(lib.cdcc_vo_layout(ctypes.byref(self.c), ctypes.byref(v)), "cdcc_vo_layout")
        self.n_vo, self.vo_off = r8(v.n_vo), r88(v.vo_off)
        self.lvo_off, self.mvo_off = r8(v.lam_off), r8(v.m_off)
        self.lvo_size, self.mvo_size = int(v.lam_size), int(v.m_size)

    # -- marshalling of inputs --------------------------------------------------
    def pack_amp(self, blocks: dict, out: np.ndarray | None = None) -> np.ndarray:
        no, nv, h = self.sym["nocc"], self.sym["nvir"], self.h
        flat = np.zeros(self.amp_size) if out is None else out
        for G in range(h):
            nr, nc = self.n_oo[G], self.n_vv[G]
            mat = flat[self.amp_off[G]:self.amp_off[G] + nr * nc].reshape(nr, nc)
            for gi in range(h):
                r0, rr = self.oo_off[G][gi], no[gi] * no[gi ^ G]
                for ga in range(h):
                    c0, cc = self.vv_off[G][ga], nv[ga] * nv[ga ^ G]
                    if rr and cc:
                        mat[r0:r0 + rr, c0:c0 + cc] = blocks[(G, gi, ga)].reshape(rr, cc)
        return flat

    def unpack_amp(self, flat) -> dict:
        flat = np.asarray(flat)
        no, nv, h = self.sym["nocc"], self.sym["nvir"], self.h
        out = {}
        for G in range(h):
            nr, nc = self.n_oo[G], self.n_vv[G]
            mat = flat[self.amp_off[G]:self.amp_off[G] + nr * nc].reshape(nr, nc)
            for gi in range(h):
                gj = gi ^ G
                r0, rr = self.oo_off[G][gi], no[gi] * no[gj]
                for ga in range(h):
                    gb = ga ^ G
                    c0, cc = self.vv_off[G][ga], nv[ga] * nv[gb]
                    out[(G, gi, ga)] = mat[r0:r0 + rr, c0:c0 + cc].reshape(no[gi], no[gj], nv[ga], nv[gb]).copy()
        return out

    def _vo_geom(self, right: str):
        no, nv = self.sym["nocc"], self.sym["nvir"]
        if right == "oo":
            return self.n_oo, self.oo_off, self.lvo_off, self.lvo_size, no
        return self.n_vv, self.vv_off, self.mvo_off, self.mvo_size, nv

    def pack_vo(self, blocks: dict, right: str) -> np.ndarray:
        """lambda_bi^mn (right = "oo") or M_bi^dc (right = "vv") blocks keyed
        (G, gb, gx) with shape (v_gb, o_gi, x_gx, x_gy) -> flat vo layout."""
        no, nv, h = self.sym["nocc"], self.sym["nvir"], self.h
        ncols, coff, base, size, cdim = self._vo_geom(right)
        flat = np.zeros(size)
        for G in range(h):
            mat = flat[base[G]:base[G] + self.n_vo[G] * ncols[G]].reshape(self.n_vo[G], ncols[G])
            for gb in range(h):
                r0, rr = self.vo_off[G][gb], nv[gb] * no[gb ^ G]
                for gx in range(h):
                    c0, cc = coff[G][gx], cdim[gx] * cdim[gx ^ G]
                    if rr and cc:
                        mat[r0:r0 + rr, c0:c0 + cc] = blocks[(G, gb, gx)].reshape(rr, cc)
        return flat

    def unpack_vo(self, flat, right: str) -> dict:
        flat = np.asarray(flat)
        no, nv, h = self.sym["nocc"], self.sym["nvir"], self.h
        ncols, coff, base, size, cdim = self._vo_geom(right)
        out = {}
        for G in range(h):
            mat = flat[base[G]:base[G] + self.n_vo[G] * ncols[G]].reshape(self.n_vo[G], ncols[G])
            for gb in range(h):
                gi = gb ^ G
                r0, rr = self.vo_off[G][gb], nv[gb] * no[gi]
                for gx in range(h):
                    c0, cc = coff[G][gx], cdim[gx] * cdim[gx ^ G]
                    out[(G, gb, gx)] = mat[r0:r0 + rr, c0:c0 + cc].reshape(nv[gb], no[gi], cdim[gx],
                                                                           cdim[gx ^ G]).copy()
        return out

    def partial_flops(self):
        """(S, A) algorithmic flops of the partial symmetric-antisymmetric
        contraction (cdcc_partial_flops)."""
        out = (ctypes.c_double * 2)()
        _lib.check(_lib.load().cdcc_partial_flops(ctypes.byref(self.c), out), "cdcc_partial_flops")
        return float(out[0]), float(out[1])

    def pack_B(self, blocks: dict) -> np.ndarray:
        flat = np.zeros(self.b_size)
        for (gP, ga), blk in blocks.items():
            if gP < self.h and ga < self.h and blk.size:
                flat[self.b_off[gP][ga]:self.b_off[gP][ga] + blk.size] = blk.ravel()
        return flat

    def pack_Bvo(self, blocks: dict) -> np.ndarray:
        flat = np.zeros(self.bvo_size)
        for (gP, ga), blk in blocks.items():
            if blk.size:
                flat[self.bvo_off[gP][ga]:self.bvo_off[gP][ga] + blk.size] = blk.ravel()
        return flat

    def pack_t1(self, t1: list) -> np.ndarray:
        flat = np.zeros(self.t1_size)
        for g in range(self.h):
            x = np.asarray(t1[g])
            if x.size:
                flat[self.t1_off[g]:self.t1_off[g] + x.size] = x.ravel()
        return flat

    def pack_eps(self, per_irrep: list) -> np.ndarray:
        return np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in per_irrep]) \
            if per_irrep else np.zeros(0)

    def density_flops(self):
        """((ab|cd) products, contraction with L) algorithmic flops of the vvvv
        density contraction (cdcc_density_flops)."""
        out = (ctypes.c_double * 2)()
        _lib.check(_lib.load().cdcc_density_flops(ctypes.byref(self.c), out), "cdcc_density_flops")
        return float(out[0]), float(out[1])

    def flops(self, kind: int = 0):
        """(assembly, contraction, dressing) algorithmic flops (cdcc_ladder_flops)."""
        out = (ctypes.c_double * 3)()
        _lib.check(_lib.load().cdcc_ladder_flops(ctypes.byref(self.c), int(kind), out), "cdcc_ladder_flops")
        return float(out[0]), float(out[1]), float(out[2])
