"""Rovibronic line list of diatomic band systems (Sec. 2.2.2), plain FP64.

TEST INFRASTRUCTURE ONLY (part of the oracle; see oracle/__init__.py): the
product path never imports it, and it shares no code with the GPU library.

For one electronic band system (upper state u, lower state l) the paper
builds each line from:
  - the vibrational term (Dunham-like, three constants):
        E_V = w_e (V + 1/2) - w_e x_e (V + 1/2)^2 + w_e y_e (V + 1/2)^3;
  - the rotational constants of level V:
        B_v = B_e - alpha_e (V + 1/2),  D_v = D_e + beta_e (V + 1/2);
  - the rotational term of the coupling case:
        Hund (a): E_J = B_v J (J + 1) - D_v J^2 (J + 1)^2,
        Hund (b): E = B_v N (N + 1) - D_v N^2 (N + 1)^2 + S gamma (N + 1/2 - S),
                  N = J - S (doublets: spin component S = +1/2 or -1/2);
  - the line centre from the state energies, nu = E_u - E_l with
        E = T_e + E_V + E_rot;
  - the Hoenl-London factor S_JJ of the branch (P: dJ = J_u - J_l = -1,
    Q: 0, R: +1) from the paper's tables for Hund's case (a) (in J_u, per
    Lambda_u, Lambda_l) and Hund's case (b) (in J_l);
  - the molecular Einstein coefficient with the rotationless transition
    moment Re' (Re'^2 = Re^2 F_vv, per band):
        A = 64 pi^4 nu^3 (e a0 Re')^2 S_JJ / (3 h (2 J_u + 1))
    (wavenumber form; the printed 1e-7 is the factor between h in J s and in
    erg s, the reading used here with every constant in CGS).

Readings (the paper names the terms but not how a band system is
enumerated):
  - Hund (a): J_u = 0..J_max, each J_u with its P, Q and R line; a level
    exists when J >= Lambda of its state; a line exists when both levels do
    and S_JJ > 0 (so the Q branch of a Sigma-Sigma system is absent).
  - Hund (b) (a doublet Sigma-Sigma system, as the case (b) table implies):
    lower levels (N_l, S_l) with N_l = 0..J_max, S_l = +-1/2, J_l = N_l + S_l
    >= 1/2; from each, P (J_u = J_l - 1) and R (J_u = J_l + 1) keep the spin
    component (N_u = N_l -+ 1) and Q (J_u = J_l) flips it (N_u = N_l + 2 S_l);
    an upper level exists when N_u >= 0 and J_u >= 1/2.
  - Level degeneracies g = g_e (2J + 1); the energies are returned split into
    an electronic-vibrational part (T_e + E_V, populated at T_v) and a
    rotational part (populated at T_tr).
  - Lines whose centre lies outside [nu_min, nu_max] are dropped.
  - Order: system, then V_u, then V_l, then the rotational index (J_u, or
    N_l then S_l = +1/2, -1/2), then the branch P, Q, R.
"""
from __future__ import annotations

import math

import numpy as np

# CGS constants: h and c exact (SI definitions), the elementary charge in
# statcoulomb from its exact SI value, the Bohr radius as the paper prints it.
H_CGS = 6.62607015e-27
C_CGS = 2.99792458e10
E_ESU = 1.602176634e-19 * C_CGS / 10.0
A0_CM = 5.291772083e-9

HUND_A, HUND_B = 0, 1
P_BRANCH, Q_BRANCH, R_BRANCH = 0, 1, 2


def vib_term(we: float, wexe: float, weye: float, v):
    """E_V of vibrational level v (cm^-1)."""
    x = np.asarray(v, np.float64) + 0.5
    return we * x - wexe * x ** 2 + weye * x ** 3


def rot_constants(Be: float, ae: float, De: float, be: float, v):
    """(B_v, D_v) of vibrational level v (cm^-1)."""
    x = np.asarray(v, np.float64) + 0.5
    return Be - ae * x, De + be * x


def rot_term_a(B: float, D: float, J):
    """Hund's case (a) rotational energy of level J (cm^-1)."""
    J = np.asarray(J, np.float64)
    return B * J * (J + 1.0) - D * J ** 2 * (J + 1.0) ** 2


def rot_term_b(B: float, D: float, gamma: float, J, S):
    """Hund's case (b) rotational energy of level J of spin component S."""
    J = np.asarray(J, np.float64)
    S = np.asarray(S, np.float64)
    N = J - S
    return B * N * (N + 1.0) - D * N ** 2 * (N + 1.0) ** 2 + S * gamma * (N + 0.5 - S)


def honl_london_a(branch: int, Ju, lam_u: int, lam_l: int):
    """Hoenl-London factor of Hund's case (a) (the paper's table, by J_u)."""
    J = np.asarray(Ju, np.float64)
    L = float(lam_u)
    if lam_u == 0 and lam_l == 0:
        return {P_BRANCH: J + 1.0, Q_BRANCH: 0.0 * J, R_BRANCH: J}[branch]
    if lam_u == lam_l:
        if branch == P_BRANCH:
            return (J + 1.0 + L) * (J + 1.0 - L) / (J + 1.0)
        if branch == Q_BRANCH:
            return (2.0 * J + 1.0) * L * L / (J * (J + 1.0))
        return (J + L) * (J - L) / J
    if abs(lam_u - lam_l) != 1:
        raise ValueError("Hund's case (a) table covers dLambda = 0, +-1")
    sg = 1.0 if lam_u - lam_l == 1 else -1.0   # upper sign for dLambda = +1
    if branch == P_BRANCH:
        return (J + 1.0 - sg * L) * (J + 2.0 - sg * L) / (2.0 * (J + 1.0))
    if branch == Q_BRANCH:
        return (J + sg * L) * (J + 1.0 - sg * L) * (2.0 * J + 1.0) / (2.0 * J * (J + 1.0))
    return (J + sg * L) * (J - 1.0 + sg * L) / (2.0 * J)


def honl_london_b(branch: int, Jl):
    """Hoenl-London factor of Hund's case (b) (the paper's table, by J_l)."""
    J = np.asarray(Jl, np.float64)
    if branch == P_BRANCH:
        return (J * J - 0.25) / J
    if branch == Q_BRANCH:
        return (2.0 * J + 1.0) / (4.0 * J * (J + 1.0))
    return ((J + 1.0) ** 2 - 0.25) / (J + 1.0)


def einstein_A(nu, Re2: float, S, Ju):
    """Molecular Einstein coefficient (s^-1) of a line at nu (cm^-1)."""
    nu = np.asarray(nu, np.float64)
    return (64.0 * math.pi ** 4 * nu ** 3 * (E_ESU * A0_CM) ** 2 * Re2 * np.asarray(S, np.float64)
            / (3.0 * H_CGS * (2.0 * np.asarray(Ju, np.float64) + 1.0)))


def _band_lines_a(s, vu: int, vl: int):
    """Candidate lines of one (V_u, V_l) band of a Hund (a) system, in order
    J_u, branch: dict of arrays (a line is kept when 'ok')."""
    Ju = np.repeat(np.arange(s.J_max + 1, dtype=np.float64), 3)
    br = np.tile(np.array([P_BRANCH, Q_BRANCH, R_BRANCH]), s.J_max + 1)
    Jl = Ju - np.where(br == P_BRANCH, -1.0, np.where(br == Q_BRANCH, 0.0, 1.0))
    ok = (Ju >= s.Lambda_u) & (Jl >= s.Lambda_l) & (Jl >= 0)
    S = np.zeros_like(Ju)
    for b in (P_BRANCH, Q_BRANCH, R_BRANCH):
        m = ok & (br == b)
        if np.any(m):
            S[m] = honl_london_a(b, Ju[m], s.Lambda_u, s.Lambda_l)
    ok &= S > 0.0
    Bu, Du = rot_constants(s.Be_u, s.ae_u, s.De_u, s.be_u, vu)
    Bl, Dl = rot_constants(s.Be_l, s.ae_l, s.De_l, s.be_l, vl)
    return dict(Ju=Ju, Jl=Jl, S=S, ok=ok,
                Eu_rot=rot_term_a(float(Bu), float(Du), Ju), El_rot=rot_term_a(float(Bl), float(Dl), Jl))


def _band_lines_b(s, vu: int, vl: int):
    """Candidate lines of one band of a Hund (b) doublet system, in order
    N_l, S_l (+1/2, -1/2), branch."""
    Nl = np.repeat(np.arange(s.J_max + 1, dtype=np.float64), 6)
    Sl = np.tile(np.repeat(np.array([0.5, -0.5]), 3), s.J_max + 1)
    br = np.tile(np.array([P_BRANCH, Q_BRANCH, R_BRANCH]), 2 * (s.J_max + 1))
    Jl = Nl + Sl
    Ju = Jl + np.where(br == P_BRANCH, -1.0, np.where(br == Q_BRANCH, 0.0, 1.0))
    Su = np.where(br == Q_BRANCH, -Sl, Sl)
    Nu = Ju - Su
    ok = (Jl >= 0.5) & (Nu >= 0.0) & (Ju >= 0.5)
    S = np.zeros_like(Jl)
    for b in (P_BRANCH, Q_BRANCH, R_BRANCH):
        m = ok & (br == b)
        if np.any(m):
            S[m] = honl_london_b(b, Jl[m])
    ok &= S > 0.0
    Bu, Du = rot_constants(s.Be_u, s.ae_u, s.De_u, s.be_u, vu)
    Bl, Dl = rot_constants(s.Be_l, s.ae_l, s.De_l, s.be_l, vl)
    return dict(Ju=Ju, Jl=Jl, S=S, ok=ok,
                Eu_rot=rot_term_b(float(Bu), float(Du), s.gamma_u, Ju, Su),
                El_rot=rot_term_b(float(Bl), float(Dl), s.gamma_l, Jl, Sl))


def rovib_lines(systems, nu_min: float, nu_max: float):
    """Every line of the band systems with nu in [nu_min, nu_max]: dict of
    arrays nu0, A, Eu_ev, Eu_rot, El_ev, El_rot, gu, gl, species, in the
    order stated in the module docstring."""
    out = {k: [] for k in ("nu0", "A", "Eu_ev", "Eu_rot", "El_ev", "El_rot", "gu", "gl", "species")}
    for s in systems:
        Re2 = np.asarray(s.Re2, np.float64).reshape(s.nv_u, s.nv_l)
        for vu in range(s.nv_u):
            Eu_ev = s.Te_u + float(vib_term(s.we_u, s.wexe_u, s.weye_u, vu))
            for vl in range(s.nv_l):
                El_ev = s.Te_l + float(vib_term(s.we_l, s.wexe_l, s.weye_l, vl))
                c = _band_lines_a(s, vu, vl) if s.hund == HUND_A else _band_lines_b(s, vu, vl)
                nu = (Eu_ev + c["Eu_rot"]) - (El_ev + c["El_rot"])
                keep = c["ok"] & (nu >= nu_min) & (nu <= nu_max)
                if not np.any(keep):
                    continue
                m = int(keep.sum())
                out["nu0"].append(nu[keep])
                out["A"].append(einstein_A(nu[keep], float(Re2[vu, vl]), c["S"][keep], c["Ju"][keep]))
                out["Eu_ev"].append(np.full(m, Eu_ev))
                out["Eu_rot"].append(c["Eu_rot"][keep])
                out["El_ev"].append(np.full(m, El_ev))
                out["El_rot"].append(c["El_rot"][keep])
                out["gu"].append(s.g_u * (2.0 * c["Ju"][keep] + 1.0))
                out["gl"].append(s.g_l * (2.0 * c["Jl"][keep] + 1.0))
                out["species"].append(np.full(m, s.species, np.int32))
    return {k: (np.concatenate(v) if v else np.zeros(0, np.int32 if k == "species" else np.float64))
            for k, v in out.items()}
