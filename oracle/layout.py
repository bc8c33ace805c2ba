"""Direct-product-decomposition storage written out in Python (oracle side).

Follows the selection rule of the paper's symmetry section (a tensor element is
stored only when the product of its index irreps is totally symmetric), for the
flat layout the C ABI documents: amplitude blocks per pair irrep G, rows (i,j)
ordered by irrep of i then i then j, columns (a,b) likewise; Cholesky blocks per
(irrep of P, irrep of a) as [a][c][P]; tensors with one virtual and one
occupied index in their first pair (lambda_bi^mn, M_bi^dc) as one block per
pair irrep G with rows (b,i) ordered by irrep of b then b then i and the
columns of the amplitude layout ((m,n) rows or (d,c) columns). Independent
re-statement used to pin the library's layout function.
"""
from __future__ import annotations

import numpy as np


class OracleLayout:
    def __init__(self, sym: dict):
        self.sym = sym
        h = self.h = sym["h"]
        no, nv, nc = sym["nocc"], sym["nvir"], sym["ncd"]
        self.n_oo = [sum(no[g] * no[g ^ G] for g in range(h)) for G in range(h)]
        self.n_vv = [sum(nv[g] * nv[g ^ G] for g in range(h)) for G in range(h)]
        self.oo_off = [[0] * h for _ in range(h)]
        self.vv_off = [[0] * h for _ in range(h)]
        for G in range(h):
            ro = rv = 0
            for g in range(h):
                self.oo_off[G][g] = ro
                self.vv_off[G][g] = rv
                ro += no[g] * no[g ^ G]
                rv += nv[g] * nv[g ^ G]
        self.amp_off = []
        off = 0
        for G in range(h):
            self.amp_off.append(off)
            off += self.n_oo[G] * self.n_vv[G]
        self.amp_size = off
        self.b_off = [[0] * h for _ in range(h)]
        self.bvo_off = [[0] * h for _ in range(h)]
        ob = ov = 0
        for gP in range(h):
            for ga in range(h):
                self.b_off[gP][ga] = ob
                self.bvo_off[gP][ga] = ov
                ob += nv[ga] * nv[ga ^ gP] * nc[gP]
                ov += nv[ga] * no[ga ^ gP] * nc[gP]
        self.b_size, self.bvo_size = ob, ov
        self.t1_off = []
        ot = 0
        for g in range(h):
            self.t1_off.append(ot)
            ot += no[g] * nv[g]
        self.t1_size = ot
        self.occ_off = list(np.concatenate([[0], np.cumsum(no)[:-1]]).astype(int))
        self.vir_off = list(np.concatenate([[0], np.cumsum(nv)[:-1]]).astype(int))
        self.cd_off = list(np.concatenate([[0], np.cumsum(nc)[:-1]]).astype(int))
        self.nocc_tot, self.nvir_tot, self.ncd_tot = sum(no), sum(nv), sum(nc)
        # (b,i) rows: irrep of b, then b, then i
        self.n_vo = [sum(nv[g] * no[g ^ G] for g in range(h)) for G in range(h)]
        self.vo_off = [[0] * h for _ in range(h)]
        for G in range(h):
            r = 0
            for g in range(h):
                self.vo_off[G][g] = r
                r += nv[g] * no[g ^ G]
        self.lvo_off, self.mvo_off = [], []
        ol = om = 0
        for G in range(h):
            self.lvo_off.append(ol)
            self.mvo_off.append(om)
            ol += self.n_vo[G] * self.n_oo[G]
            om += self.n_vo[G] * self.n_vv[G]
        self.lvo_size, self.mvo_size = ol, om

    # ---- flat <-> blocks -------------------------------------------------
    def pack_amp(self, blocks: dict) -> np.ndarray:
        h, no, nv = self.h, self.sym["nocc"], self.sym["nvir"]
        flat = np.zeros(self.amp_size)
        for G in range(h):
            mat = flat[self.amp_off[G]:self.amp_off[G] + self.n_oo[G] * self.n_vv[G]].reshape(
                self.n_oo[G], self.n_vv[G])
            for gi in range(h):
                r0, nr = self.oo_off[G][gi], no[gi] * no[gi ^ G]
                for ga in range(h):
                    c0, ncol = self.vv_off[G][ga], nv[ga] * nv[ga ^ G]
                    mat[r0:r0 + nr, c0:c0 + ncol] = blocks[(G, gi, ga)].reshape(nr, ncol)
        return flat

    def unpack_amp(self, flat: np.ndarray) -> dict:
        h, no, nv = self.h, self.sym["nocc"], self.sym["nvir"]
        out = {}
        for G in range(h):
            mat = np.asarray(flat[self.amp_off[G]:self.amp_off[G] + self.n_oo[G] * self.n_vv[G]]).reshape(
                self.n_oo[G], self.n_vv[G])
            for gi in range(h):
                gj = gi ^ G
                r0, nr = self.oo_off[G][gi], no[gi] * no[gj]
                for ga in range(h):
                    gb = ga ^ G
                    c0, ncol = self.vv_off[G][ga], nv[ga] * nv[gb]
                    out[(G, gi, ga)] = mat[r0:r0 + nr, c0:c0 + ncol].reshape(no[gi], no[gj], nv[ga], nv[gb]).copy()
        return out

    def pack_vo(self, blocks: dict, right: str) -> np.ndarray:
        """lambda_bi^mn (right = "oo") or M_bi^dc (right = "vv") blocks keyed
        (G, gb, gm or gd) -> flat."""
        h, no, nv = self.h, self.sym["nocc"], self.sym["nvir"]
        ncols = self.n_oo if right == "oo" else self.n_vv
        coff = self.oo_off if right == "oo" else self.vv_off
        base = self.lvo_off if right == "oo" else self.mvo_off
        cdim = no if right == "oo" else nv
        flat = np.zeros(self.lvo_size if right == "oo" else self.mvo_size)
        for G in range(h):
            mat = flat[base[G]:base[G] + self.n_vo[G] * ncols[G]].reshape(self.n_vo[G], ncols[G])
            for gb in range(h):
                r0, nr = self.vo_off[G][gb], nv[gb] * no[gb ^ G]
                for gx in range(h):
                    c0, nc_ = coff[G][gx], cdim[gx] * cdim[gx ^ G]
                    mat[r0:r0 + nr, c0:c0 + nc_] = blocks[(G, gb, gx)].reshape(nr, nc_)
        return flat

    def unpack_vo(self, flat: np.ndarray, right: str) -> dict:
        h, no, nv = self.h, self.sym["nocc"], self.sym["nvir"]
        ncols = self.n_oo if right == "oo" else self.n_vv
        coff = self.oo_off if right == "oo" else self.vv_off
        base = self.lvo_off if right == "oo" else self.mvo_off
        cdim = no if right == "oo" else nv
        out = {}
        for G in range(h):
            mat = np.asarray(flat[base[G]:base[G] + self.n_vo[G] * ncols[G]]).reshape(self.n_vo[G], ncols[G])
            for gb in range(h):
                gi = gb ^ G
                r0, nr = self.vo_off[G][gb], nv[gb] * no[gi]
                for gx in range(h):
                    c0, nc_ = coff[G][gx], cdim[gx] * cdim[gx ^ G]
                    out[(G, gb, gx)] = mat[r0:r0 + nr, c0:c0 + nc_].reshape(
                        nv[gb], no[gi], cdim[gx], cdim[gx ^ G]).copy()
        return out

    def full_vo(self, blocks: dict, right: str) -> np.ndarray:
        """Scatter vo blocks into a full (v, o, x, x) tensor (x = o or v)."""
        h, no, nv = self.h, self.sym["nocc"], self.sym["nvir"]
        xd = self.nocc_tot if right == "oo" else self.nvir_tot
        xoff = self.occ_off if right == "oo" else self.vir_off
        cdim = no if right == "oo" else nv
        out = np.zeros((self.nvir_tot, self.nocc_tot, xd, xd))
        for (G, gb, gx), blk in blocks.items():
            gi, gy = gb ^ G, gx ^ G
            b0, i0, x0, y0 = self.vir_off[gb], self.occ_off[gi], xoff[gx], xoff[gy]
            out[b0:b0 + nv[gb], i0:i0 + no[gi], x0:x0 + cdim[gx], y0:y0 + cdim[gy]] = blk
        return out

    def pack_B(self, blocks: dict, vo: bool = False) -> np.ndarray:
        h = self.h
        flat = np.zeros(self.bvo_size if vo else self.b_size)
        offs = self.bvo_off if vo else self.b_off
        for gP in range(h):
            for ga in range(h):
                blk = blocks[(gP, ga)]
                flat[offs[gP][ga]:offs[gP][ga] + blk.size] = blk.ravel()
        return flat

    def pack_t1(self, t1: list) -> np.ndarray:
        return np.concatenate([np.asarray(x).ravel() for x in t1]) if self.t1_size else np.zeros(0)

    # ---- blocks -> full (symmetry-free) tensors ------------------------------
    def full_B(self, blocks: dict) -> np.ndarray:
        h, nv, nc = self.h, self.sym["nvir"], self.sym["ncd"]
        out = np.zeros((self.ncd_tot, self.nvir_tot, self.nvir_tot))
        for gP in range(h):
            p0 = self.cd_off[gP]
            for ga in range(h):
                gc = ga ^ gP
                a0, c0 = self.vir_off[ga], self.vir_off[gc]
                blk = blocks[(gP, ga)]  # (a, c, P)
                out[p0:p0 + nc[gP], a0:a0 + nv[ga], c0:c0 + nv[gc]] = blk.transpose(2, 0, 1)
        return out

    def full_Bvo(self, blocks: dict) -> np.ndarray:
        """L^P_am for a virtual, m occupied: shape (P, v, o)."""
        h, nv, no, nc = self.h, self.sym["nvir"], self.sym["nocc"], self.sym["ncd"]
        out = np.zeros((self.ncd_tot, self.nvir_tot, self.nocc_tot))
        for gP in range(h):
            p0 = self.cd_off[gP]
            for ga in range(h):
                gm = ga ^ gP
                a0, m0 = self.vir_off[ga], self.occ_off[gm]
                out[p0:p0 + nc[gP], a0:a0 + nv[ga], m0:m0 + no[gm]] = blocks[(gP, ga)].transpose(2, 0, 1)
        return out

    def full_t1(self, t1: list) -> np.ndarray:
        out = np.zeros((self.nocc_tot, self.nvir_tot))
        for g in range(self.h):
            o0, v0 = self.occ_off[g], self.vir_off[g]
            out[o0:o0 + t1[g].shape[0], v0:v0 + t1[g].shape[1]] = t1[g]
        return out

    def full_amp(self, blocks: dict) -> np.ndarray:
        h, no, nv = self.h, self.sym["nocc"], self.sym["nvir"]
        out = np.zeros((self.nocc_tot,) * 2 + (self.nvir_tot,) * 2)
        for (G, gi, ga), blk in blocks.items():
            gj, gb = gi ^ G, ga ^ G
            i0, j0, a0, b0 = self.occ_off[gi], self.occ_off[gj], self.vir_off[ga], self.vir_off[gb]
            out[i0:i0 + no[gi], j0:j0 + no[gj], a0:a0 + nv[ga], b0:b0 + nv[gb]] = blk
        return out

    def blocks_from_full(self, full: np.ndarray) -> dict:
        h, no, nv = self.h, self.sym["nocc"], self.sym["nvir"]
        out = {}
        for G in range(h):
            for gi in range(h):
                gj = gi ^ G
                for ga in range(h):
                    gb = ga ^ G
                    i0, j0, a0, b0 = self.occ_off[gi], self.occ_off[gj], self.vir_off[ga], self.vir_off[gb]
                    out[(G, gi, ga)] = full[i0:i0 + no[gi], j0:j0 + no[gj], a0:a0 + nv[ga], b0:b0 + nv[gb]].copy()
        return out

    def allowed_mask(self) -> np.ndarray:
        """Boolean (o,o,v,v) mask of symmetry-allowed amplitude entries."""
        io = np.concatenate([[g] * n for g, n in enumerate(self.sym["nocc"])]).astype(int) if self.nocc_tot else np.zeros(0, int)
        iv = np.concatenate([[g] * n for g, n in enumerate(self.sym["nvir"])]).astype(int) if self.nvir_tot else np.zeros(0, int)
        x = io[:, None, None, None] ^ io[None, :, None, None] ^ iv[None, None, :, None] ^ iv[None, None, None, :]
        return x == 0
