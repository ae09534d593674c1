"""Per-step parity of the HIP path against the oracle, matched by particle id.

The GPU state (int32 cell + float32 offset, float32 momenta, float64 E) is read
back, promoted exactly to float64 and loaded into the oracle, both advance one
step, and the results are compared particle by particle through their ids.

Bars (FP32 state against the FP64 oracle):
  * the sets of live ids are equal and every cell index equals the oracle's
    floor(x), except for particles whose oracle position lies within BAND of a
    cell edge or a wall (float32 rounding can put them on either side);
  * positions agree within XTOL cells, momenta within UTOL relative to the
    larger of the old and new |u| (plus UFLOOR absolute, for u = 0 exactly);
    a momentum that the method sets from an energy (the recoil gamma - eps of a
    scattering event, the pair members at gamma = eps/2) is compared through
    that energy, within GTOL relative;
  * scattering-event decisions agree except where |U - p| < PTOL (U the Philox
    draw, p = min(Ndot h, 1)), photon-conversion decisions except where
    eps is within PTOL of 2 or the conversion point within BAND of an edge;
  * E after Ampere agrees within what the float32 positions allow: 4 pi Q times
    the per-cell particle count times XTOL.
Particles excused by these rules are counted and reported.
"""
import math

import numpy as np

from oracle import drag as odrag
from oracle import philox, pic, rics

BAND = 2e-6
XTOL = 1e-6
UTOL = 1e-5
UFLOOR = 1e-12
PTOL = 2e-6
GTOL = 1e-6


def oracle_config(cfg):
    keys = {k: v for k, v in cfg.items() if k in pic.DEFAULTS}
    return pic.make_config(**keys)


def snapshot(sim):
    lines = []
    for li in range(sim.n_lines):
        sp = [sim.get_particles(li, s) for s in range(4)]
        lines.append(dict(parts=sp, E=sim.get_field(li)))
    m = sim.moments(0)
    return dict(lines=lines, step=m["step"])


def oracle_from_snapshot(ocfg, snap):
    st = pic.State(ocfg)
    st.step = snap["step"]
    for li, L in enumerate(snap["lines"]):
        for s in range(4):
            p = L["parts"][s]
            pic.load_particles(st, li, s, p["cell"], p["off"], p["u"], p["id"])
        st.E[li] = L["E"].astype(np.float64).copy()
    return st


def _marginal_parents(ocfg, st_before, li):
    """(ids of leptons whose event, conversion or drag-branch decision sits within the
    tolerance of its threshold, ids of leptons that scatter)."""
    ln = st_before.lines[li]
    k0, k1 = philox.seed_key(ocfg["seed"])
    out = set()
    scattered = set()
    if ocfg["rics"] == "off":
        return out, scattered
    counts = pic.cell_counts(ln, st_before.parts[li])
    for s in (0, 1, 2):
        P = st_before.parts[li][s]
        if P["x"].size == 0:
            continue
        x0 = P["x"]
        b, mu, xr, rc = ln.geometry_at(x0)
        stoch = b >= ocfg["b_thr"]
        # b on either side of the threshold within float32 resolution also counts
        near_b = np.abs(b - ocfg["b_thr"]) < 1e-6 * ocfg["b_thr"]
        qm = pic.SPECIES_SIGN[s]
        Ep = pic.gather_E(st_before.E[li], x0)
        us = P["u"] + qm * Ep / ln.C
        _, _, rate = ln.rics_funcs(x0, b, mu, xr)
        lam = rate(us) * ln.h
        p = np.minimum(lam, 1.0)
        lo, hi = philox.split_id(P["id"])
        w = philox.philox4x32_10(st_before.step, lo, hi, philox.STREAM_RICS, k0, k1)
        U = philox.uniform24(w[0])
        if ocfg["emission"] == "perpendicular":
            eps = rics.photon_energy(us, b)
            dirn = np.where(us >= 0, 1.0, -1.0)
            turn = np.zeros(us.shape, dtype=bool)
        else:
            mu_r = rics.emission_cosine(w[1], w[2], w[3], ocfg["emission"])
            eps, _, dirn = rics.emission(us, b, mu_r)
            # the photon's direction is the sign of mu_r + beta_e
            ge = np.sqrt(1.0 + us * us) / np.sqrt(1.0 + 2.0 * b)
            be = np.sqrt(np.maximum(1.0 - 1.0 / (ge * ge), 0.0))
            turn = np.abs(mu_r + be) < 1e-5
        marg = near_b | (stoch & (np.abs(U - p) < PTOL + 1e-5 * p))
        marg |= stoch & (U < p) & turn
        # drag limiter switch |F(p0)| tau_min = |p0| in either half step of the continuous regime
        cont = ~stoch
        if cont.any():
            xc = x0[cont]
            force, dforce, _ = ln.rics_funcs(xc, b[cont], mu[cont], xr[cont])
            u0 = P["u"][cont]
            def switch(v):
                a, c = np.abs(force(v)) * ln.tau_hat, np.abs(v)
                return (a > 0) & (np.abs(a - c) <= 1e-4 * c)
            sw1 = switch(u0)
            u1 = odrag.half_step(u0, force, dforce, ln.h, ln.tau_hat, mu[cont]) + qm * Ep[cont] / ln.C
            sw2 = switch(u1)
            m2 = np.zeros_like(marg)
            m2[np.nonzero(cont)[0]] = sw1 | sw2
            marg |= m2
        marg |= stoch & (U < p) & (np.abs(eps - 2.0) < PTOL * eps)
        if ocfg["pairs"]:
            ev = stoch & (U < p) & (eps >= 2.0)
            if ocfg["conversion"] == "curvature":
                sp = x0 + dirn * (rc / ln.ds) * np.arcsin(np.minimum(2.0 / np.maximum(eps, 2.0), 1.0))
                tolx = 1e-5 * np.abs(sp - x0) + BAND
            else:
                sp = x0.copy()
                tolx = np.full_like(x0, BAND)
            frac = sp - np.round(sp)
            edge = (np.abs(frac) < tolx) | (np.abs(sp) < tolx) | (np.abs(sp - ln.n) < tolx)
            inside = (sp >= 0) & (sp < ln.n)
            cidx = np.clip(np.floor(np.where(inside, sp, 0)).astype(int), 0, ln.n - 1)
            cap = np.abs(counts[cidx] - ln.n_max) < 1.0
            marg |= ev & (edge | cap)
        out.update(int(i) for i in P["id"][marg])
        scattered.update(int(i) for i in P["id"][stoch & (U < p)])
    return out, scattered


def _child_ids(ocfg, step, parent_ids):
    k0, k1 = philox.seed_key(ocfg["seed"])
    ids = set()
    for pid in parent_ids:
        lo, hi = philox.split_id(np.uint64(pid))
        w = philox.philox4x32_10(step, lo, hi, philox.STREAM_CHILD, k0, k1)
        ids.add(int(philox.id_from_words(w[0], w[1])))
        ids.add(int(philox.id_from_words(w[2], w[3])))
    return ids


def _child_parent_x(ocfg, step, parts_before):
    """Position before the step of the parent of every pair member that a lepton of
    parts_before could create this step (child id -> parent x)."""
    k0, k1 = philox.seed_key(ocfg["seed"])
    out = {}
    for s in (0, 1):
        P = parts_before[s]
        if P["id"].size == 0:
            continue
        lo, hi = philox.split_id(P["id"].astype(np.uint64))
        w = philox.philox4x32_10(step, lo, hi, philox.STREAM_CHILD, k0, k1)
        x = P["cell"].astype(np.float64) + P["off"].astype(np.float64)
        for a, b in ((0, 1), (2, 3)):
            for cid, xp in zip(philox.id_from_words(w[a], w[b]), x):
                out[int(cid)] = float(xp)
    return out


def restrict(snap, keep):
    """The snapshot with only the particles whose id is in keep (a uint64 array);
    fields are kept whole."""
    lines = []
    for L in snap["lines"]:
        parts = []
        for P in L["parts"]:
            m = np.isin(P["id"], keep)
            parts.append({k: v[m] for k, v in P.items()})
        lines.append(dict(parts=parts, E=L["E"]))
    return dict(lines=lines, step=snap["step"])


def compare_step(ocfg, snap_before, snap_after, xtol=XTOL, utol=UTOL, xtol_new=None, check_field=True,
                 drop=None):
    """Advance the oracle from snap_before and compare with the GPU's snap_after.

    With check_field False the field after Ampere is not compared (for a
    sample of the particles, whose current is not the whole line's).  drop(li, s,
    side, ids, cells, new) -> bool mask names particles to leave out of the
    comparison; an id dropped on either side is dropped on both.

    Returns a report dict; raises AssertionError on an unexcused mismatch.
    """
    st = oracle_from_snapshot(ocfg, snap_before)
    before = oracle_from_snapshot(ocfg, snap_before)
    pic.step(st)
    rep = dict(compared=0, excused=0, max_dx=0.0, max_du_rel=0.0, max_dE=0.0, new=0)
    ambiguous = {}

    def refill_ambiguous(li, excused_ids):
        """Per cell, how many atmosphere (e-, ion) counts before the refill may differ
        between the float32 and float64 paths: an atmosphere particle within BAND of a
        face (its cell and the neighbour across that face), or at a wall (absorbed or
        not), or an excused one.  A refill differs from the oracle's by at most that
        many particles per species in a cell."""
        pre = oracle_from_snapshot(dict(ocfg, atmosphere=False, annihilation=False), snap_before)
        pic.step(pre)
        amb = {}
        for s in (2, 3):
            x = pre.parts[li][s]["x"]
            ids = pre.parts[li][s]["id"]
            near = np.abs(x - np.round(x)) < BAND
            for b in np.round(x[near]).astype(np.int64):
                for c in (int(b) - 1, int(b)):
                    amb[c] = amb.get(c, 0) + 1
            for i, xx in zip(ids, x):
                if int(i) in excused_ids:
                    c = int(math.floor(xx))
                    amb[c] = amb.get(c, 0) + 1
            # absorbed on one side only: the particle kept by the other path lies
            # within BAND of a wall
            B = snap_before["lines"][li]["parts"][s]
            xb = B["cell"].astype(np.float64) + B["off"].astype(np.float64)
            walls = (xb < 1.0) | (xb > pre.lines[li].n - 1.0)
            for c in np.floor(np.clip(xb[walls], 0, pre.lines[li].n - 1)).astype(np.int64):
                amb[int(c)] = amb.get(int(c), 0) + 1
        return amb

    def annihilation_ambiguous(li, excused_ids):
        """Cells whose end-of-step count (before annihilation) may differ between the
        float32 and float64 paths: a particle within BAND of one of their faces, or
        an excused particle inside.  Only there may the annihilation differ."""
        if li not in ambiguous:
            pre = oracle_from_snapshot(dict(ocfg, annihilation=False), snap_before)
            pic.step(pre)
            cells = set()
            for s in range(4):
                P = pre.parts[li][s]
                x = P["x"]
                near = np.abs(x - np.round(x)) < BAND
                for b in np.round(x[near]).astype(np.int64):
                    cells.update((int(b) - 1, int(b)))
                for i, xx in zip(P["id"], x):
                    if int(i) in excused_ids:
                        cells.add(int(math.floor(xx)))
            ambiguous[li] = cells
        return ambiguous[li]
    for li, Lg in enumerate(snap_after["lines"]):
        ln = st.lines[li]
        n = ln.n
        marg, scattered = _marginal_parents(ocfg, before, li)
        excused_new = _child_ids(ocfg, before.step, marg)
        atm_cells_excused = {}  # cell -> one-sided injected atmosphere particles excused
        atm_amb = None
        ann_excused = {}        # cell -> one-sided e-/e+ excused by an ambiguous annihilation
        parent_x = None
        maxcount = 1
        for s in range(4):
            G = Lg["parts"][s]
            O = st.parts[li][s]
            B = snap_before["lines"][li]["parts"][s]
            if drop is not None:
                bid = B["id"].astype(np.uint64)
                gd = drop(li, s, "gpu", G["id"], G["cell"].astype(np.int64), ~np.isin(G["id"].astype(np.uint64), bid))
                od = drop(li, s, "oracle", O["id"], np.floor(O["x"]).astype(np.int64),
                          ~np.isin(O["id"].astype(np.uint64), bid))
                gone = np.union1d(G["id"][gd].astype(np.uint64), O["id"][od].astype(np.uint64))
                kg = ~np.isin(G["id"].astype(np.uint64), gone)
                ko = ~np.isin(O["id"].astype(np.uint64), gone)
                rep["dropped"] = rep.get("dropped", 0) + int((~kg).sum())
                G = {k: v[kg] for k, v in G.items()}
                O = {k: v[ko] for k, v in O.items()}
            before_ids = set(int(i) for i in B["id"])
            u_before = dict(zip((int(i) for i in B["id"]), B["u"].astype(np.float64)))
            gid = G["id"].astype(np.uint64)
            oid = O["id"].astype(np.uint64)
            go = np.argsort(gid)
            oo = np.argsort(oid)
            gs, os_ = gid[go], oid[oo]
            common, gi, oi = np.intersect1d(gs, os_, assume_unique=True, return_indices=True)
            only_g = np.setdiff1d(gs, os_, assume_unique=True)
            only_o = np.setdiff1d(os_, gs, assume_unique=True)
            xg = G["cell"][go][gi].astype(np.float64) + G["off"][go][gi].astype(np.float64)
            xo = O["x"][oo][oi]
            cg = G["cell"][go][gi]
            co = np.floor(xo).astype(np.int64)
            ug = G["u"][go][gi].astype(np.float64)
            uo = O["u"][oo][oi]
            ub = np.array([u_before.get(int(i), 0.0) for i in common])
            is_new = np.array([int(i) not in before_ids for i in common], dtype=bool)
            exc = np.array([int(i) in marg or int(i) in excused_new for i in common], dtype=bool)
            near_edge = np.abs(xo - np.round(xo)) < BAND
            raw_cell = cg != co
            bad_cell = raw_cell & ~near_edge & ~exc
            tolx = np.where(is_new, xtol_new if xtol_new is not None else xtol, xtol)
            if ocfg["conversion"] == "curvature" and is_new.any():
                # a pair member sits at the parent's position plus the distance
                # d = (R_curv / ds) arcsin(2/eps), computed from the parent's float32
                # state: a relative error e of eps moves it by d e tan(t)/t, t = d ds / R_curv
                # the angle (arcsin's slope), with e within the momentum tolerance
                if parent_x is None:
                    parent_x = _child_parent_x(ocfg, snap_before["step"], snap_before["lines"][li]["parts"])
                xp = np.array([parent_x.get(int(i), x) for i, x in zip(common, xo)])
                dist = np.abs(xo - xp)
                _, _, _, rcur = ln.geometry_at(np.clip(xp, 0.0, n))
                theta = np.minimum(dist * ln.ds / rcur, 0.5 * math.pi * (1.0 - 1e-9))
                slope = np.where(theta > 1e-8, np.tan(theta) / np.maximum(theta, 1e-8), 1.0)
                tolx = np.where(is_new, np.maximum(tolx, utol * dist * slope + xtol), tolx)
            dx = np.abs(xg - xo)
            raw_x = dx > tolx
            bad_x = raw_x & ~exc
            scale = np.maximum(np.abs(uo), np.abs(ub))
            if s >= 2:
                scale = np.maximum(scale, np.where(is_new, math.sqrt(ocfg["atm_T"]) * 1e-3, 0.0))
            du = np.abs(ug - uo)
            # a momentum set from an energy (event recoil gamma - eps, pair members at eps/2)
            # is conditioned by gamma^2/|u|: allow GTOL relative error in gamma there
            from_energy = is_new | np.array([int(i) in scattered for i in common], dtype=bool)
            if s >= 2:
                from_energy &= ~is_new
            gam = np.sqrt(1.0 + uo * uo)
            cond = np.where(from_energy, GTOL * gam * gam / np.maximum(np.abs(uo), 1e-4), 0.0)
            raw_u = du > utol * scale + cond + UFLOOR
            bad_u = raw_u & ~exc
            nbad = int(bad_cell.sum() + bad_x.sum() + bad_u.sum())
            if nbad:
                i = np.nonzero(bad_cell | bad_x | bad_u)[0][:5]
                raise AssertionError(
                    f"line {li} species {s}: {nbad} mismatches; e.g. ids {common[i]} "
                    f"x_gpu {xg[i]} x_orc {xo[i]} u_gpu {ug[i]} u_orc {uo[i]} u_before {ub[i]}")
            rep["compared"] += int(common.size)
            rep["new"] += int(is_new.sum())
            rep["excused"] += int(((raw_cell | raw_x | raw_u) & (exc | near_edge)).sum())
            if common.size:
                rep["max_dx"] = max(rep["max_dx"], float(dx[~exc].max()) if (~exc).any() else 0.0)
                rel = du / np.maximum(scale, 1e-30)
                rep["max_du_rel"] = max(rep["max_du_rel"], float(rel[~exc].max()) if (~exc).any() else 0.0)
            # ids on one side only
            for side, ids, X in (("gpu", only_g, G), ("oracle", only_o, O)):
                for pid in ids:
                    pid = int(pid)
                    if pid in excused_new or pid in marg:
                        rep["excused"] += 1
                        continue
                    if s < 2 and ocfg.get("annihilation"):
                        # kept by one side only: annihilated by the other in a cell whose count
                        # the two paths may see differently
                        if side == "gpu":
                            k = int(np.nonzero(G["id"] == np.uint64(pid))[0][0])
                            cell = int(G["cell"][k])
                        else:
                            k = int(np.nonzero(O["id"] == np.uint64(pid))[0][0])
                            cell = int(math.floor(O["x"][k]))
                        if cell in annihilation_ambiguous(li, marg | excused_new):
                            ann_excused[cell] = ann_excused.get(cell, 0) + 1
                            rep["excused"] += 1
                            continue
                    if pid in before_ids:
                        # absorption decision: the kept position must lie within BAND of a wall
                        if side == "gpu":
                            k = int(np.nonzero(G["id"] == np.uint64(pid))[0][0])
                            xx = float(G["cell"][k]) + float(G["off"][k])
                        else:
                            k = int(np.nonzero(O["id"] == np.uint64(pid))[0][0])
                            xx = float(O["x"][k])
                        if min(abs(xx), abs(n - xx)) < BAND:
                            rep["excused"] += 1
                            continue
                        raise AssertionError(f"line {li} species {s}: particle {pid} kept only by the {side} "
                                             f"at x = {xx}")
                    if s >= 2:
                        if side == "gpu":
                            k = int(np.nonzero(G["id"] == np.uint64(pid))[0][0])
                            cell = int(G["cell"][k])
                        else:
                            k = int(np.nonzero(O["id"] == np.uint64(pid))[0][0])
                            cell = int(math.floor(O["x"][k]))
                        if atm_amb is None:
                            atm_amb = refill_ambiguous(li, marg | excused_new)
                        key = (cell, s)
                        atm_cells_excused[key] = atm_cells_excused.get(key, 0) + 1
                        if atm_cells_excused[key] > atm_amb.get(cell, 0):
                            raise AssertionError(f"line {li} species {s}: new atmosphere particle {pid} only on the "
                                                 f"{side} in cell {cell}, beyond what ambiguous counts there allow")
                        rep["excused"] += 1
                        continue
                    raise AssertionError(f"line {li} species {s}: new particle {pid} only on the {side}")
            cnt = np.bincount(np.floor(O["x"]).astype(np.int64), minlength=n) if O["x"].size else np.zeros(n)
            maxcount = max(maxcount, int(cnt.max()) if cnt.size else 1)
        # an atmosphere cell may differ by the refill of one excused particle only
        if atm_cells_excused:
            rep["atm_cells_excused"] = sorted(c for c, _ in atm_cells_excused)
            for c, _ in atm_cells_excused:
                assert min(c, n - 1 - c) < ln.atm_depth + 2, f"atmosphere mismatch outside the layer, cell {c}"
        if not check_field:
            continue
        # field after Ampere
        Eg = Lg["E"]
        Eo = st.E[li]
        dE = np.abs(Eg - Eo)
        tolE = 4.0 * math.pi * ln.Q * (2.0 * maxcount * xtol + 1e-6) + 1e-12 * np.abs(Eo)
        for c, m in ann_excused.items():
            # each particle annihilated on one side only moves up to a cell's worth of charge
            tolE[c] += 4.0 * math.pi * ln.Q * m
        if ann_excused:
            rep["annihilation_cells_excused"] = sorted(ann_excused)
        if (dE > tolE).any():
            k = int(np.argmax(dE - tolE))
            raise AssertionError(f"line {li}: E mismatch at cell {k}: gpu {Eg[k]} oracle {Eo[k]} tol {tolE[k]}")
        rep["max_dE"] = max(rep["max_dE"], float((dE / (4 * math.pi * ln.Q)).max()))
    return rep, st


def sampled_compare(ocfg, snap_before, snap_after, n_sample, rng, n_max=None):
    """compare_step on a sample of a full-size line (one line).

    Given the field, a particle's push, drag, event and conversion do not depend on
    the other particles, and the atmosphere refill depends only on the end-of-step
    counts of the atmosphere species.  The sample is therefore every atmosphere
    particle, n_sample seeded e-/e+ per lepton species, the pair members the sampled
    leptons can create this step (ids from the child stream) and the atmosphere
    particles injected this step.  The field after Ampere is not compared.

    With n_max given (a line at its density limit) the two couplings through cell
    counts are taken from the whole line: the sample's pair members are compared
    only in cells where the whole line's count at the step's start is below n_max
    (elsewhere no pair is made; the GPU must have made none), and e-/e+ only in
    cells that certainly annihilated nothing -- an end count of at most n_max - 2
    with both e- and e+ left (annihilation stops at n_max - 1 or n_max, or where
    one of them runs out).  The oracle steps the sample without annihilation."""
    L0, L1 = snap_before["lines"][0], snap_after["lines"][0]
    keep = []
    for s in range(4):
        ids = L0["parts"][s]["id"]
        keep.append(ids if s >= 2 or ids.size <= n_sample else rng.choice(ids, size=n_sample, replace=False))
    parents = np.concatenate(keep[:3]).astype(np.uint64)
    k0, k1 = philox.seed_key(ocfg["seed"])
    lo, hi = philox.split_id(parents)
    w = philox.philox4x32_10(snap_before["step"], lo, hi, philox.STREAM_CHILD, k0, k1)
    children = [philox.id_from_words(w[0], w[1]), philox.id_from_words(w[2], w[3])]
    injected = [np.setdiff1d(L1["parts"][s]["id"], L0["parts"][s]["id"]) for s in (2, 3)]
    keep_before = np.unique(np.concatenate(keep).astype(np.uint64))
    keep_after = np.unique(np.concatenate(keep + children + injected).astype(np.uint64))
    drop = None
    if n_max is not None:
        n = int(L0["E"].shape[0])

        def counts(L, species):
            return sum(np.bincount(L["parts"][s]["cell"].astype(np.int64), minlength=n) for s in species)
        blocked = counts(L0, range(4)) >= n_max
        e1, p1 = counts(L1, (0,)), counts(L1, (1,))
        unsafe = ~((counts(L1, range(4)) <= n_max - 2) & (e1 > 0) & (p1 > 0))
        before_all = np.concatenate([L0["parts"][s]["id"] for s in (0, 1)]).astype(np.uint64)
        for s in (0, 1):
            made = ~np.isin(L1["parts"][s]["id"].astype(np.uint64), before_all)
            cells = L1["parts"][s]["cell"][made].astype(np.int64)
            assert not blocked[cells].any(), "a pair made in a cell at n_max"
        ocfg = dict(ocfg, annihilation=False)

        def drop(li, s, side, ids, cells, new):
            if s >= 2:
                return np.zeros(ids.shape, dtype=bool)
            return unsafe[cells] | (new & blocked[cells])
    rep, st = compare_step(ocfg, restrict(snap_before, keep_before), restrict(snap_after, keep_after),
                           check_field=False, drop=drop)
    rep["sampled"] = [int(k.size) for k in keep]
    return rep, st
