"""CPU emulation of the fused kernel's register/LDS algorithm, driven by the planner's own
device image (qp_plan_image).  complex128, one point at a time, every thread of the point's
thread group emulated explicitly: registers [thread][8]; the opening rotation stage folded into
the product state; exchanges through the kernel's own LDS byte addresses (per-lane words and
per-exchange register offsets) and sign bits; readout with the plan's parity masks; the adjoint
sweep with uncompute and per-gate M accumulation, the folded stage taking its statistics at its
output.

This checks the planner (fusion, GF(2) entangler maps, sign forms, round mappings, readout
folding, gradient map) and the algorithm independently of the GPU; the oracle is the
reference it is compared with.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

HDR = np.dtype([("n", "<i4"), ("n_params", "<i4"), ("n_out", "<i4"), ("n_fused", "<i4"), ("n_rounds", "<i4"),
                ("enc_kind", "<i4"), ("enc_gate", "<i4"), ("enc_scale", "<i4"), ("n_feat", "<i4"),
                ("coord", "<i4", 16), ("zmask", "<u4", 8), ("off_rounds", "<i4"), ("off_xf", "<i4"),
                ("off_xb", "<i4"), ("off_fused", "<i4"), ("off_csr_ptr", "<i4"), ("off_csr_idx", "<i4"),
                ("off_rff_B", "<i4"), ("off_rff_W", "<i4"), ("bytes", "<i4"), ("n_dgroups", "<i4"),
                ("off_dgroups", "<i4"), ("off_dgates", "<i4"), ("n_docc", "<i4"), ("off_docc", "<i4"),
                ("off_dcsr_ptr", "<i4"), ("off_dcsr_idx", "<i4"), ("zplain", "<u4", 8), ("n_head", "<i4"),
                ("head_gate", "<i4", 16), ("off_lanes", "<i4")])
ROUND = np.dtype([("gate", "<i4", 3), ("pad0", "<i4"), ("sgate", "<i4", 2), ("pad1", "<i4", 2),
                  ("tpos", "<i4", 16), ("tpost", "<i4", 16)])
XCHG = np.dtype([("acol", "<u4", 16), ("src_r", "<u4", 8), ("qu", "<u4", 32), ("qv", "<u4", 32), ("ue", "<u4", 3),
                 ("ve", "<u4", 3), ("nterms", "<u4"), ("sign_at_src", "<u4"), ("qsign_r", "<u4"), ("identity", "<u4"),
                 ("pad1", "<u4", 2), ("roff", "<u4", 8), ("woff", "<u4", 8), ("mcol", "<u4", 16)])
FUSED = np.dtype([("qubit", "<i4"), ("ncomp", "<i4"), ("kind", "<i4", 3), ("param", "<i4", 3), ("stat_out", "<i4"),
                  ("pad", "<i4", 3)])
LANE = np.dtype([("wb", "<u4"), ("rb", "<u4"), ("sgn", "<u4"), ("pad", "<u4")])
assert ROUND.itemsize == 160 and XCHG.itemsize == 528 and FUSED.itemsize == 48


def plan_image(circ):
    from paper_2506_23246_amd import _lib as L
    from paper_2506_23246_amd.api import make_desc
    d, keep = make_desc(circ)
    nb = C.c_size_t(0)
    st = L.qp_plan_image(C.byref(d), None, 0, C.byref(nb))
    buf = (C.c_ubyte * nb.value)()
    st = L.qp_plan_image(C.byref(d), buf, nb.value, C.byref(nb))
    assert st == 0, st
    raw = bytes(buf)
    h = np.frombuffer(raw, HDR, 1)[0]
    R = int(h["n_rounds"])
    plan = {
        "h": h,
        "rounds": np.frombuffer(raw, ROUND, R, int(h["off_rounds"])),
        "xf": np.frombuffer(raw, XCHG, R, int(h["off_xf"])),
        "xb": np.frombuffer(raw, XCHG, R, int(h["off_xb"])),
        "fused": np.frombuffer(raw, FUSED, int(h["n_fused"]), int(h["off_fused"])),
        # per-lane exchange words [direction][round][thread of the point]
        "lanes": np.frombuffer(raw, LANE, 2 * R * (1 << (int(h["n"]) - 3)),
                               int(h["off_lanes"])).reshape(2, R, 1 << (int(h["n"]) - 3)) if R else None,
        "csr_ptr": np.frombuffer(raw, "<i4", int(h["n_params"]) + 1, int(h["off_csr_ptr"])),
    }
    nnz = int(plan["csr_ptr"][-1])
    plan["csr_idx"] = np.frombuffer(raw, "<i4", nnz, int(h["off_csr_idx"])) if nnz else np.zeros(0, np.int32)
    return plan


def _par(x):
    return bin(int(x)).count("1") & 1


def _deposit(u, tpos, n):
    j = 0
    for k in range(3, n):
        j |= ((u >> (k - 3)) & 1) << int(tpos[k])
    return j


def _regoff(r, tpos):
    return ((r & 1) << int(tpos[0])) | (((r >> 1) & 1) << int(tpos[1])) | (((r >> 2) & 1) << int(tpos[2]))


def _rot(kind, th):
    c, s = math.cos(th / 2), math.sin(th / 2)
    if kind == 0:
        return np.array([[c, -1j * s], [-1j * s, c]])
    if kind == 1:
        return np.array([[c, -s], [s, c]], dtype=complex)
    return np.array([[c - 1j * s, 0], [0, c + 1j * s]])


def _fused_matrix(f, params):
    U = np.eye(2, dtype=complex)
    for c in range(int(f["ncomp"])):
        U = _rot(int(f["kind"][c]), float(params[int(f["param"][c])])) @ U
    return U


def _swap_slots(n):
    return 2 if n == 10 else (1 if n in (8, 12) else 0)


def _swap(regs, i):
    """Swap slot i: register bit i trades places with thread bit 4 + i (a relabelling)."""
    out = np.empty_like(regs)
    TP = regs.shape[1]
    for u in range(TP):
        for r in range(8):
            rb, ub = (r >> i) & 1, (u >> (4 + i)) & 1
            u2 = (u & ~(1 << (4 + i))) | (rb << (4 + i))
            r2 = (r & ~(1 << i)) | (ub << i)
            out[:, u2, r2] = regs[:, u, r]
    return out


def _swz(i):
    """The LDS index swizzle (an involution, linear over GF(2))."""
    return i ^ (((i >> 4) ^ (i >> 8) ^ (i >> 12) ^ (i >> 16)) & 15)


def descriptor_words(X, n, rpos, u):
    """Reader side of an exchange for thread u from the descriptor alone (index map columns and the
    bilinear split of the sign form): thread part of the source index sb, the eight uniform source
    offsets and the eight sign bits."""
    jn = _deposit(u, rpos, n)
    if X["identity"]:
        return jn, [_regoff(r, rpos) for r in range(8)], [0] * 8
    sb = 0
    for k in range(n):
        if (jn >> k) & 1:
            sb ^= int(X["acol"][k])
    srcr = [int(v) for v in X["src_r"]]
    sg = [0] * 8
    nt = int(X["nterms"])
    if nt:
        xb = sb if X["sign_at_src"] else jn
        pu = sum(_par(int(X["qu"][t]) & xb) << t for t in range(nt))
        pv = sum(_par(int(X["qv"][t]) & xb) << t for t in range(nt))
        q0 = _par(pu & pv)
        bs = [_par((pu & int(X["ve"][i])) ^ (int(X["ue"][i]) & pv)) for i in range(3)]
        for r in range(8):
            s = q0 ^ ((int(X["qsign_r"]) >> r) & 1)
            for i in range(3):
                if (r >> i) & 1:
                    s ^= bs[i]
            sg[r] = s
    return sb, srcr, sg


def _exchange(regs, wpos, rpos, X, L, n, TP):
    """regs: [S][TP][8] complex -> new regs (the kernel's exchange, for one point at pbase = 0);
    wpos/rpos are the writer's and reader's physical-to-logical bit maps (unused: the emulation
    goes through the kernel's own address tables), L the plan's lane words of this exchange
    ([TP]: writer and reader LDS byte bases, sign bits).  Every thread writes register r at byte
    wb ^ woff[r] and reads register r from rb ^ roff[r], negated where its sign bit is set."""
    S = regs.shape[0]
    buf = {}
    for u in range(TP):
        for r in range(8):
            addr = int(L[u]["wb"]) ^ int(X["woff"][r])
            assert addr not in buf, "two writes to one LDS entry"
            buf[addr] = regs[:, u, r]
    assert len(buf) == 8 * TP
    out = np.zeros_like(regs)
    for u in range(TP):
        sg = int(L[u]["sgn"])
        for r in range(8):
            v = buf[int(L[u]["rb"]) ^ int(X["roff"][r])]
            out[:, u, r] = -v if (sg >> r) & 1 else v
    return out


def _apply(regs, svs, bit, U):
    for r in range(8):
        if r & (1 << bit):
            continue
        r1 = r | (1 << bit)
        x, y = regs[svs, :, r].copy(), regs[svs, :, r1].copy()
        regs[svs, :, r] = U[0, 0] * x + U[0, 1] * y
        regs[svs, :, r1] = U[1, 0] * x + U[1, 1] * y


def _stats(regs, b, s):
    """s += (S_x, S_y, S_z) of the pairs on register bit b (lambda-family 4..7, psi-family 0..3)."""
    for r in range(8):
        if r & (1 << b):
            continue
        r1 = r | (1 << b)
        for sv in range(4):
            x0, x1 = regs[4 + sv, :, r], regs[4 + sv, :, r1]
            y0, y1 = regs[sv, :, r], regs[sv, :, r1]
            s[0] += np.sum(np.imag(np.conj(x0) * y1 + np.conj(x1) * y0))
            s[1] += np.sum(np.real(np.conj(x1) * y0 - np.conj(x0) * y1))
            s[2] += np.sum(np.imag(np.conj(x0) * y0 - np.conj(x1) * y1))


def emulate_point(plan, params, theta, J, gate_rx, seeds_f=None, seeds_g=None, stats_at_round_input=False):
    """One point: returns f [m], g [m,3] and (if seeds given) the per-gate adjoint products:
    M [F,2,2] (lambda after the gate, psi before it) and S [F,3] = Im <lambda|sigma_k|psi> with
    both taken before the gate (k = x, y, z), the statistic the kernel accumulates.  With
    stats_at_round_input, S of every gate of a round is taken after all of the round's gates are
    pulled back (valid because they act on different qubits and commute), as the pipelined
    kernel does."""
    h = plan["h"]
    n, m, R = int(h["n"]), int(h["n_out"]), int(h["n_rounds"])
    TP = 1 << (n - 3)
    rounds, xf, xb, fused = plan["rounds"], plan["xf"], plan["xb"], plan["fused"]
    Us = [_fused_matrix(f, params) for f in fused]
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    e0, e1 = c.astype(complex), (-1j * s if gate_rx else s.astype(complex))
    d0, d1 = -0.5 * s + 0j, (-0.5j * c if gate_rx else 0.5 * c + 0j)
    # leading rotation stage (rounds 0 .. H-1): applied to each qubit's factor, product state
    # formed in round H-1's output mapping
    H = int(h["n_head"])
    for q in range(n):
        g = int(h["head_gate"][q])
        if g >= 0:
            U = Us[g]
            e0[q], e1[q] = U[0, 0] * e0[q] + U[0, 1] * e1[q], U[1, 0] * e0[q] + U[1, 1] * e1[q]
            d0[q], d1[q] = U[0, 0] * d0[q] + U[0, 1] * d1[q], U[1, 0] * d0[q] + U[1, 1] * d1[q]
    regs = np.zeros((8, TP, 8), complex)
    t0 = rounds[H - 1]["tpost"] if H > 0 else rounds[0]["tpos"]
    for u in range(TP):
        for r in range(8):
            j = _deposit(u, t0, n) | _regoff(r, t0)
            amp = 1 + 0j
            der = np.zeros(3, complex)
            for q in range(n):
                b = (j >> (n - 1 - q)) & 1
                e = e1[q] if b else e0[q]
                d = d1[q] if b else d0[q]
                der = der * e + amp * J[q] * d
                amp = amp * e
            regs[0, u, r] = amp
            regs[1:4, u, r] = der
    nsw = _swap_slots(n)
    for k in range(H, R):
        if k > 0:
            regs[:4] = _exchange(regs[:4], rounds[k - 1]["tpost"], rounds[k]["tpos"], xf[k], plan["lanes"][0, k], n, TP)
        for b in range(3):
            g = int(rounds[k]["gate"][b])
            if g >= 0:
                _apply(regs, slice(0, 4), b, Us[g])
        for i in range(nsw):
            regs[:4] = _swap(regs[:4], i)
            g = int(rounds[k]["sgate"][i])
            if g >= 0:
                _apply(regs, slice(0, 4), i, Us[g])
    tl = rounds[R - 1]["tpost"]
    f = np.zeros(m)
    gg = np.zeros((m, 3))
    z = np.zeros((m, TP, 8))
    for u in range(TP):
        for r in range(8):
            j = _deposit(u, tl, n) ^ _regoff(r, tl)
            for i in range(m):
                z[i, u, r] = -1.0 if _par(int(h["zmask"][i]) & j) else 1.0
    psi = regs[0]
    for i in range(m):
        f[i] = np.sum(z[i] * np.abs(psi) ** 2)
        for cc in range(3):
            gg[i, cc] = 2 * np.sum(z[i] * np.real(np.conj(psi) * regs[1 + cc]))
    if seeds_g is None:
        return f, gg, None, None
    Df = sum(seeds_f[i] * z[i] for i in range(m)) if seeds_f is not None else 0.0
    D = [sum(seeds_g[i, cc] * z[i] for i in range(m)) for cc in range(3)]
    regs[4] = Df * regs[0] + D[0] * regs[1] + D[1] * regs[2] + D[2] * regs[3]
    for cc in range(3):
        regs[5 + cc] = D[cc] * regs[0]
    M = np.zeros((len(fused), 2, 2), complex)
    S = np.zeros((len(fused), 3))
    def head_m(g, b):
        """M of a leading-stage gate: lambda at the stage output, psi pulled back through this gate
        only (the stage's other gates act on other qubits and leave the pair sums unchanged)."""
        tmp = regs.copy()
        _apply(tmp, slice(0, 4), b, Us[g].conj().T)
        for r in range(8):
            if r & (1 << b):
                continue
            r1 = r | (1 << b)
            for sv in range(4):
                x0, x1 = tmp[4 + sv, :, r], tmp[4 + sv, :, r1]
                y0, y1 = tmp[sv, :, r], tmp[sv, :, r1]
                M[g, 0, 0] += np.sum(np.conj(x0) * y0)
                M[g, 0, 1] += np.sum(np.conj(x0) * y1)
                M[g, 1, 0] += np.sum(np.conj(x1) * y0)
                M[g, 1, 1] += np.sum(np.conj(x1) * y1)

    for k in range(R - 1, -1, -1):
        if k < H:   # leading stage: statistics at the stage output, nothing pulled back
            for i in reversed(range(nsw)):
                g = int(rounds[k]["sgate"][i])
                if g >= 0:
                    head_m(g, i)
                    _stats(regs, i, S[g])
                regs = _swap(regs, i)
            for b in range(3):
                g = int(rounds[k]["gate"][b])
                if g >= 0:
                    head_m(g, b)
                    _stats(regs, b, S[g])
            if k > 0:
                regs = _exchange(regs, rounds[k]["tpos"], rounds[k - 1]["tpost"], xb[k], plan["lanes"][1, k], n, TP)
            continue
        for i in reversed(range(nsw)):   # swap-slot gates, then undo the swaps
            g = int(rounds[k]["sgate"][i])
            if g >= 0:
                Ud = Us[g].conj().T
                _apply(regs, slice(0, 4), i, Ud)
                for r in range(8):
                    if r & (1 << i):
                        continue
                    r1 = r | (1 << i)
                    for sv in range(4):
                        x0, x1 = regs[4 + sv, :, r], regs[4 + sv, :, r1]
                        y0, y1 = regs[sv, :, r], regs[sv, :, r1]
                        M[g, 0, 0] += np.sum(np.conj(x0) * y0)
                        M[g, 0, 1] += np.sum(np.conj(x0) * y1)
                        M[g, 1, 0] += np.sum(np.conj(x1) * y0)
                        M[g, 1, 1] += np.sum(np.conj(x1) * y1)
                _apply(regs, slice(4, 8), i, Ud)
                _stats(regs, i, S[g])
            regs = _swap(regs, i)
        for b in (2, 1, 0):
            g = int(rounds[k]["gate"][b])
            if g < 0:
                continue
            Ud = Us[g].conj().T
            _apply(regs, slice(0, 4), b, Ud)
            for r in range(8):
                if r & (1 << b):
                    continue
                r1 = r | (1 << b)
                for sv in range(4):
                    x0, x1 = regs[4 + sv, :, r], regs[4 + sv, :, r1]
                    y0, y1 = regs[sv, :, r], regs[sv, :, r1]
                    M[g, 0, 0] += np.sum(np.conj(x0) * y0)
                    M[g, 0, 1] += np.sum(np.conj(x0) * y1)
                    M[g, 1, 0] += np.sum(np.conj(x1) * y0)
                    M[g, 1, 1] += np.sum(np.conj(x1) * y1)
            _apply(regs, slice(4, 8), b, Ud)
            if not stats_at_round_input:
                _stats(regs, b, S[g])
        if stats_at_round_input:
            for b in range(3):
                g = int(rounds[k]["gate"][b])
                if g >= 0:
                    _stats(regs, b, S[g])
        if k > 0:
            regs = _exchange(regs, rounds[k]["tpos"], rounds[k - 1]["tpost"], xb[k], plan["lanes"][1, k], n, TP)
    return f, gg, M, S


def grads_from_m(plan, params, M):
    """d L / d theta_k = sum over components driven by theta_k of 2 Re sum_ab dU_ab M_ab."""
    K = int(plan["h"]["n_params"])
    out = np.zeros(K)
    P = {0: np.array([[0, 1], [1, 0]]), 1: np.array([[0, -1j], [1j, 0]]), 2: np.diag([1, -1])}
    for k in range(K):
        for e in range(int(plan["csr_ptr"][k]), int(plan["csr_ptr"][k + 1])):
            fi, ci = int(plan["csr_idx"][e]) >> 2, int(plan["csr_idx"][e]) & 3
            f = plan["fused"][fi]
            U = np.eye(2, dtype=complex)
            for c in range(int(f["ncomp"])):
                Rm = _rot(int(f["kind"][c]), float(params[int(f["param"][c])]))
                if c == ci:
                    Rm = -0.5j * P[int(f["kind"][c])] @ Rm
                U = Rm @ U
            out[k] += 2 * np.real(np.sum(U * M[fi]))
    return out


def grads_from_s(plan, params, S):
    """d L / d theta_k = sum over components c driven by theta_k of n(c) . S_gate, where
    n(c) is the axis of G_c = W^H P_c W, W the product of the gate's components before c; for a
    gate of the leading stage (statistic at the gate output) the axis of U G_c U^H."""
    K = int(plan["h"]["n_params"])
    out = np.zeros(K)
    P = {0: np.array([[0, 1], [1, 0]]), 1: np.array([[0, -1j], [1j, 0]]), 2: np.diag([1, -1])}
    paulis = [P[0], P[1], P[2]]
    for k in range(K):
        for e in range(int(plan["csr_ptr"][k]), int(plan["csr_ptr"][k + 1])):
            fi, ci = int(plan["csr_idx"][e]) >> 2, int(plan["csr_idx"][e]) & 3
            f = plan["fused"][fi]
            Wm = np.eye(2, dtype=complex)
            for c in range(ci):
                Wm = _rot(int(f["kind"][c]), float(params[int(f["param"][c])])) @ Wm
            G = Wm.conj().T @ P[int(f["kind"][ci])] @ Wm
            if int(f["stat_out"]):
                U = _fused_matrix(f, params)
                G = U @ G @ U.conj().T
            nvec = [0.5 * np.real(np.trace(sk @ G)) for sk in paulis]
            out[k] += float(np.dot(nvec, S[fi]))
    return out
