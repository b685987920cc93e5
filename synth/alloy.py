"""Material properties of the solidification workload (inputs only).

The paper's die-casting runs (section 4) fill the mould with an Al-10 % Si
alloy at 1000 K and hold the walls at 500 K.  Its freezing and solidus
temperatures are 660 C and 577 C; the liquidus follows from a straight
liquidus line, and the partition coefficient is the ratio of the liquidus
to the solidus slope.  The two phase-diagram points those lines need, the
eutectic composition (12.6 wt % Si) and the largest solubility of Si in
solid Al (1.65 wt % at the eutectic temperature), are standard Al-Si data
that the paper does not print.  The thermophysical values are typical of
liquid Al-Si alloys and are chosen here (the paper uses temperature-dependent
tables it does not list); the smear width T_eps = 2 K is the paper's.
"""
from __future__ import annotations

T_FREEZE = 933.15      # K, pure Al (660 C)
T_EUTECTIC = 850.15    # K, solidus of hypoeutectic Al-Si (577 C)
C_EUTECTIC = 12.6      # wt % Si
C_SOLID_MAX = 1.65     # wt % Si in solid Al at the eutectic temperature


def al_si_alloy(si_wt=10.0, T_wall=500.0, T_ref=1000.0, gravity=(0.0, 0.0, -9.81)):
    """Property set of an Al-Si alloy with `si_wt` % Si.  T_wall None means
    thermally insulated walls."""
    m_liq = (T_FREEZE - T_EUTECTIC) / C_EUTECTIC      # K per wt %
    m_sol = (T_FREEZE - T_EUTECTIC) / C_SOLID_MAX
    return dict(
        rho=2400.0,            # kg/m^3
        cp=1100.0,             # J/(kg K)
        k=100.0,               # W/(m K)
        mu=1.3e-3,             # Pa s
        beta=1.2e-4,           # 1/K
        lam=20e-6,             # m, dendrite arm spacing (Eq. 3)
        Lf=430e3,              # J/kg
        T_f=T_FREEZE,
        T_liq=T_FREEZE - m_liq * si_wt,
        T_sol=T_EUTECTIC,
        T_eps=2.0,
        k_p=m_liq / m_sol,
        T_ref=float(T_ref),
        g=tuple(float(v) for v in gravity),
        T_wall=None if T_wall is None else float(T_wall),
    )


def al_alloy(T_liq=913.0, T_sol=833.0, k=150.0, cp=900.0, Lf=3.9e5, T_wall=600.0, T_ref=950.0,
             gravity=(0.0, 0.0, -9.81)):
    """Property set of an aluminium alloy given by its liquidus and solidus:
    rho 2400 kg/m^3, k 150 W/(m K), c_p 900 J/(kg K), latent heat 3.9e5 J/kg,
    liquidus 913 K, solidus 833 K by default.  The Scheil partition
    coefficient follows from straight liquidus and solidus lines through the
    melting point of pure Al: k_p = (T_f - T_liq) / (T_f - T_sol).  The
    viscosity, expansion coefficient and dendrite arm spacing are those of
    al_si_alloy."""
    base = al_si_alloy(T_wall=T_wall, T_ref=T_ref, gravity=gravity)
    base.update(k=float(k), cp=float(cp), Lf=float(Lf), T_liq=float(T_liq), T_sol=float(T_sol),
                k_p=(T_FREEZE - T_liq) / (T_FREEZE - T_sol))
    return base
