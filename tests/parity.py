"""Element-by-element comparison of the GPU path's outputs with the FP64 oracle.

Bars (FP32 GPU vs FP64 oracle, same seeded inputs, same Philox seed):
  * hit triangle and instance label: bit-exact, except rays the oracle marks
    ambiguous (second hit within 1e-6 m, edge graze, near miss, at the trace
    limit), which are counted and excluded;
  * detection flag: equal, except rays within 1e-5 relative of an eq.5 or
    range threshold (oracle's ``marginal``) or ambiguous;
  * depth (t, range, point coordinates): 1e-5 relative;
  * intensity / R_lambda: 1e-4 relative (to max(I, R_lambda));
  * depth and intensity tolerances skip grazing hits (cos < 0.01), where an
    FP32 ray direction moves the hit by tan(theta) x 1e-7.
"""
import numpy as np

NO = 0xFFFFFFFF


def u32(t):
    a = t.detach().cpu().numpy() if hasattr(t, "detach") else np.asarray(t)
    return a.view(np.uint32) if a.dtype == np.int32 else a.astype(np.uint32)


def to_np(out: dict, beams=None) -> dict:
    r = {}
    for k, t in out.items():
        a = t.detach().cpu().numpy()
        if k in ("tri", "label"):
            a = a.view(np.uint32)
        if k == "material":
            a = a.view(np.uint16)
        if beams is not None:
            a = a[..., beams]
        r[k] = a
    return r


def compare(g: dict, o: dict, check_debug: bool = True) -> dict:
    """g: GPU outputs (numpy, already restricted to o['beams']); o: oracle dict."""
    amb = o["ambiguous"]
    n = len(amb)
    rep = {"n": n, "ambiguous": int(amb.sum()), "grazing": int(o["grazing"].sum()),
           "marginal": int((o["marginal"] & ~amb).sum())}
    # the ambiguous rays by class (a ray can be in several): second hit within 1e-6 m, edge graze, near
    # miss in front, hit at the trace limit
    for cls in ("amb_tie", "amb_edge", "amb_near", "amb_limit"):
        if cls in o:
            rep[cls] = int(np.asarray(o[cls]).sum())
    ok = ~amb
    if check_debug:
        bad = ok & (g["tri"] != o["tri"])
        rep["tri_mismatch"] = int(bad.sum())
        assert not bad.any(), f"hit triangle differs on {bad.sum()} unambiguous rays, e.g. beams {o['beams'][bad][:8]}"
        hit = ok & (o["tri"] != NO)
        m_bad = hit & (g["material"] != o["material"])
        assert not m_bad.any(), "material differs"
    vcmp = ok & ~o["marginal"]
    bad = vcmp & (g["valid"] != o["valid"])
    rep["valid_mismatch"] = int(bad.sum())
    assert not bad.any(), f"valid differs on {bad.sum()} rays, e.g. beams {o['beams'][bad][:8]}"
    both = vcmp & (o["valid"] == 1)
    assert np.array_equal(g["label"][both], o["label"][both]), "label differs"
    nv = vcmp & (o["valid"] == 0)
    assert np.all(g["label"][nv] == NO) and np.all(g["intensity"][nv] == 0) and np.all(g["range"][nv] == 0)
    assert np.all(g["x"][nv] == 0) and np.all(g["y"][nv] == 0) and np.all(g["z"][nv] == 0)
    fine = both & ~o["grazing"]
    rng = o["range"][fine]
    e_r = np.abs(g["range"][fine] - rng) / rng
    rep["range_max_rel"] = float(e_r.max()) if e_r.size else 0.0
    assert np.all(e_r <= 1e-5), f"range rel error {e_r.max():.3g}"
    for k in ("x", "y", "z"):
        e = np.abs(g[k][fine] - o[k][fine]) / rng
        assert np.all(e <= 1e-5), f"{k} rel error {e.max():.3g}"
    scale = np.maximum(np.abs(o["intensity"][fine]), o["r_lambda"][fine])
    e_i = np.abs(g["intensity"][fine] - o["intensity"][fine]) / scale
    rep["intensity_max_rel"] = float(e_i.max()) if e_i.size else 0.0
    assert np.all(e_i <= 1e-4), f"intensity rel error {e_i.max():.3g}"
    if check_debug:
        h = ok & (o["tri"] != NO) & ~o["grazing"]
        e_t = np.abs(g["t_hit"][h] - o["t_hit"][h]) / o["t_hit"][h]
        rep["t_max_rel"] = float(e_t.max()) if e_t.size else 0.0
        assert np.all(e_t <= 1e-5), f"t_hit rel error {e_t.max():.3g}"
        e_l = np.abs(g["r_lambda"][h] - o["r_lambda"][h]) / o["r_lambda"][h]
        assert np.all(e_l <= 1e-4), f"r_lambda rel error {e_l.max():.3g}"
        e_n = np.abs(g["normal"][:, h] - o["normal"][h].T)
        assert np.all(e_n <= 1e-5), f"normal error {e_n.max():.3g}"
        miss = ok & (o["tri"] == NO)
        assert np.all(g["t_hit"][miss] == 0) and np.all(g["material"][miss] == 0xFFFF)
    rep["hits"] = int((o["tri"] != NO).sum())
    rep["valid"] = int((o["valid"] == 1).sum())
    return rep


def compare_echoes(g: dict, o: dict) -> dict:
    """g: GPU echo outputs as numpy [E, n] (restricted to o['beams']); o: oracle simulate_echoes dict.

    Beams the oracle marks ambiguous (a sub-ray ambiguous as in compare(), or a
    gap within 1e-5 relative of the separation) are excluded; per echo, the
    detection flag skips marginal echoes, triangle / material (and the label,
    when it differs between them) skip echoes whose two strongest sub-rays are
    within 1e-5, and the range / intensity tolerances skip echoes with a
    grazing sub-ray.  Tolerances as in compare().
    """
    E, n = o["valid"].shape
    ok = ~o["ambiguous"]
    rep = {"n": n, "ambiguous": int((~ok).sum()), "echoes_formed": [int((o["tri"][e] != NO).sum()) for e in range(E)],
           "detected": [int(o["valid"][e].sum()) for e in range(E)], "range_max_rel": 0.0, "intensity_max_rel": 0.0}
    for e in range(E):
        formed = ok & (o["tri"][e] != NO)
        assert np.all(g["tri"][e][ok & ~formed] == NO) and np.all(g["valid"][e][ok & ~formed] == 0), e
        dom = o["amb_dom"][e]
        sel = formed & ~dom
        bad = sel & ((g["tri"][e] != o["tri"][e]) | (g["material"][e] != o["material"][e]))
        assert not bad.any(), f"echo {e}: strongest sub-ray differs on {bad.sum()} beams"
        vcmp = ok & ~o["marginal"][e]
        bad = vcmp & (g["valid"][e] != o["valid"][e])
        assert not bad.any(), f"echo {e}: valid differs on {bad.sum()} beams, e.g. {o['beams'][bad][:8]}"
        both = vcmp & (o["valid"][e] == 1)
        bad = both & ~dom & (g["label"][e] != o["label"][e])
        assert not bad.any(), f"echo {e}: label differs on {bad.sum()} beams"
        fine = both & ~o["grazing"][e]
        rng = o["range"][e][fine]
        e_r = np.abs(g["range"][e][fine] - rng) / rng
        assert np.all(e_r <= 1e-5), f"echo {e}: range rel error {e_r.max():.3g}"
        for k in ("x", "y", "z"):
            assert np.all(np.abs(g[k][e][fine] - o[k][e][fine]) / rng <= 1e-5), (e, k)
        scale = np.maximum(np.abs(o["intensity"][e][fine]), o["r_lambda"][e][fine])
        e_i = np.abs(g["intensity"][e][fine] - o["intensity"][e][fine]) / scale
        assert np.all(e_i <= 1e-4), f"echo {e}: intensity rel error {e_i.max():.3g}"
        fz = formed & ~o["grazing"][e]
        e_t = np.abs(g["t_hit"][e][fz] - o["t_hit"][e][fz]) / o["t_hit"][e][fz]
        assert np.all(e_t <= 1e-5), f"echo {e}: echo range rel error {e_t.max():.3g}"
        e_p = np.abs(g["r_lambda"][e][fz] - o["r_lambda"][e][fz]) / np.maximum(o["r_lambda"][e][fz], 1e-30)
        assert np.all(e_p <= 1e-4), f"echo {e}: strength rel error {e_p.max():.3g}"
        if e_r.size:
            rep["range_max_rel"] = max(rep["range_max_rel"], float(e_r.max()))
        if e_i.size:
            rep["intensity_max_rel"] = max(rep["intensity_max_rel"], float(e_i.max()))
    return rep
