"""Physical constants and scheme parameters of the oracle (test infrastructure).

The paper defers the discretisation to ICON's published one and prints no
constants; these are the documented ICON values for a dry atmosphere
(Earth radius 6.371e6 m as the workloads state) and the scheme constants of
the readings, each commented below.
"""

RD = 287.04          # gas constant of dry air [J/kg/K]
CPD = 1004.64        # specific heat at constant pressure [J/kg/K]
CVD = CPD - RD       # specific heat at constant volume [J/kg/K]
GRAV = 9.80665       # [m/s^2]
P0 = 1.0e5           # reference pressure [Pa]
OMEGA = 7.29212e-5   # Earth angular velocity [1/s]


def default_params():
    """Scheme parameters (same names and defaults as the library's dc_params)."""
    return {
        "eta": 0.65,            # implicit weight of the vertical solver (off-centering)
        "adv_w0": 0.25,         # corrector weight of the predictor-time advective tendency
        "adv_w1": 0.75,         # corrector weight of the predicted-state advective tendency
        "divdamp_c4": 0.0025,   # 4th-order divergence damping, coefficient c4 * mean_area^2
        "rayleigh_tau0": 0.05,  # sponge damping rate [1/s]
        "rayleigh_zfrac": 2.0 / 3.0,  # sponge starts at this fraction of the model top
        "smag_cs": 0.015,       # Smagorinsky constant
        "smag_cap": 16.0,       # nu <= A_e / (smag_cap * dt)
        "hdiff_k4": 1.0 / 128.0,  # 4th-order background diffusion, k4 * A_e^2
        "diffuse_w": 1,         # apply 2nd-order Smagorinsky diffusion to w
        "diffuse_theta": 0,     # optional 2nd-order Smagorinsky diffusion of theta_v, exner updated
        "theta_enh_nlev": 0,    # with diffuse_theta: lowest levels whose theta_v coefficient is raised
        "theta_enh_thresh": 5.0,  # ... in cells colder than their neighbours' mean by more than this [K]
        "miura": 0,             # 1: rho and theta_v at edges by second-order upwind (Miura) reconstruction
        "vt_rbf": 0,            # 1: tangential wind by RBF vector reconstruction instead of Perot
        "rd": RD, "cpd": CPD, "cvd": CVD, "omega": OMEGA,
    }
