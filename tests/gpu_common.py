"""Helpers shared by the GPU parity tests: state transfer from the oracle to the
library (the oracle's state is the reference input; nothing flows back)."""
import numpy as np

import oracle as O
import paper_1712_07028_amd as fsl


def transfer(o, s, w):
    """Import the oracle's current state into the library."""
    s.set(fsl.FIELD_FLAGS, o.get(O.FLAGS))
    s.set(fsl.FIELD_F, o.get(O.F))
    s.set(fsl.FIELD_MASS, o.get(O.MASS))
    s.set(fsl.FIELD_PHI, o.get(O.PHI))
    s.set(fsl.FIELD_BUBBLE_ID, o.get(O.BUBBLE_ID))
    s.set(fsl.FIELD_PID, o.get(O.PID))
    if w.particles is not None and w.particles.n:
        st = o.particles_get(w.particles.n)
        p = w.particles
        cur = type(p)(x=st["x"], u=st["u"], omega=st["omega"], R=p.R, rho_p=p.rho_p)
        # both sides restart the particle update from this table (no previous-step
        # force in the two-step average); coverage is already consistent
        o.particles_set(cur)
        s.particles_set(cur)
    b = o.bubbles()
    s.bubbles_set([x["M"] for x in b], list(range(len(b))), [x["alive"] for x in b])


def near_threshold(phi_o, eps, tol=1e-9):
    return (np.abs(phi_o - (1 - eps)) < tol) | (np.abs(phi_o - eps) < tol)


def compare_step(o, s, w, f_rtol=1e-6, m_tol=1e-6, ft_rtol=1e-5, allow_flag_mismatch=0, x_tol=1e-9):
    """Compare the states after one step; returns a dict of the measured errors."""
    fo, fg = o.get(O.FLAGS), s.get(fsl.FIELD_FLAGS)
    mism = fo != fg
    out = {"flag_mismatch": int(mism.sum())}
    assert mism.sum() <= allow_flag_mismatch, f"{mism.sum()} flag mismatches at {np.argwhere(mism)[:10]}"
    act = ((fo == O.LIQ) | (fo == O.IFC)) & ~mism
    Fo, Fg = o.get(O.F), s.get(fsl.FIELD_F)
    err = np.abs(Fg[:, act] - Fo[:, act]) / np.abs(Fo[:, act])
    out["f_rel"] = float(err.max()) if err.size else 0.0
    assert out["f_rel"] < f_rtol, out
    ifc = (fo == O.IFC) & ~mism
    if ifc.any():
        mo, mg = o.get(O.MASS)[ifc], s.get(fsl.FIELD_MASS)[ifc]
        po, pg = o.get(O.PHI)[ifc], s.get(fsl.FIELD_PHI)[ifc]
        out["m_abs"] = float(np.abs(mo - mg).max())
        out["phi_abs"] = float(np.abs(po - pg).max())
        assert out["m_abs"] < m_tol and out["phi_abs"] < m_tol, out
    if w.particles is not None and w.particles.n:
        n = w.particles.n
        a, b = o.particles_get(n), s.particles_get(n)
        # per particle and component: each force component against the particle's
        # force, each torque component against the larger of the particle's torque and
        # its force at one lever arm R + 1 (the farthest boundary node of Eq. torque; a
        # torque that vanishes by symmetry leaves only the rounding of the force's
        # link terms at that arm)
        Fn = np.linalg.norm(a["F"], axis=1)
        Tn = np.linalg.norm(a["T"], axis=1)
        arm = w.particles.R + 1.0
        dF = np.abs(a["F"] - b["F"]).max(axis=1)
        dT = np.abs(a["T"] - b["T"]).max(axis=1)
        out["F_rel"] = float((dF / np.maximum(Fn, 1e-300)).max())
        out["T_rel"] = float((dT / np.maximum(np.maximum(Tn, arm * Fn), 1e-300)).max())
        out["x_abs"] = float(np.abs(a["x"] - b["x"]).max())
        assert out["F_rel"] < ft_rtol and out["T_rel"] < ft_rtol, out
        assert out["x_abs"] < x_tol, out
        assert (o.get(O.PID) == s.get(fsl.FIELD_PID)).all()
    # face forces (momentum exchange of the bounce-back links): each component within
    # 1e-5 of its own size plus 1e-9 per face cell (rounding of the FP32 populations)
    Wo, Wg = o.walls(), s.walls()
    area = np.array([w.n[1] * w.n[2], w.n[0] * w.n[2], w.n[0] * w.n[1]], dtype=np.float64)[:, None, None]
    out["wall_err"] = float((np.abs(Wo - Wg) / (1e-5 * np.abs(Wo) + 1e-9 * area)).max())
    assert out["wall_err"] <= 1.0, (out, Wo, Wg)
    bo, bg = o.bubbles(), s.bubbles()
    for x, y in zip(bo, bg):
        if not x["alive"]:
            continue
        assert y["alive"]
        out.setdefault("V_rel", 0.0)
        out["V_rel"] = max(out["V_rel"], abs(x["V"] - y["V"]) / x["V"])
        assert abs(x["rho_g"] - y["rho_g"]) < 1e-7, (x, y)
    assert out.get("V_rel", 0.0) < 1e-6, out
    return out
