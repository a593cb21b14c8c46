"""Default tracking parameters (plain values; the C struct is filled from them).

Lengths are in quanta of 1/256 cm unless the name says otherwise.  The values
are readings chosen for the TPC geometry the paper's detector has (152 pad
rows between 85 and 247 cm, 20-degree sectors, 1 mm / 1.5 mm cluster
resolution); the paper itself gives no tracking parameters.
"""
import math

Q = 256  # quanta per cm

DEFAULT_PARAMS = dict(
    q_shift=8,
    tan_half_q16=int(round(math.tan(math.radians(10.0)) * 65536)),  # sector half opening 10 deg
    # hit grid: y bin width, target occupancy, shortest z bin
    bin_y_q=3 * Q,
    bin_occ=2,
    bin_zmin_q=Q,
    # neighbour windows (cm -> quanta) and residual weights (1/sigma^2, sigma_y:sigma_z = 2:3)
    win_y_q=int(1.5 * Q),
    win_z_q=int(2.5 * Q),
    w_y=9,
    w_z=4,
    # score cut: w sigma^2 = 5898.24 q^2, 1.5 for the line through two neighbours,
    # chi2 of 2 dof at 20 (tail 4.5e-5: a 150-row track keeps all its links with
    # probability 0.993)  ->  S_max(i) = 176947 (X_{i+1} - X_{i-1})^2
    smax_k=int(round(9 * (0.1 * Q) ** 2 * 1.5 * 20.0)),
    l_min=5,
    ext_win_y_q=1 * Q,
    ext_win_z_q=int(1.5 * Q),
    ext_edge_q=int(1.5 * Q),
    max_miss=5,
    n_min=10,
    f_min_q8=128,
    sinphi_max=0.95,
    sigma_y=0.1,
    sigma_z=0.15,
    cov0=(0.1 ** 2, 0.15 ** 2, 1e-2, 1e-2, 10.0),
)
