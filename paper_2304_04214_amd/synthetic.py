"""Seeded synthetic inputs for the STG channel workloads.

This module only draws random numbers and builds synthetic input profiles; it
holds none of the method's arithmetic (no equilibrium, collision, wall law,
Cholesky factor or mode sum).  Both the HIP path and the FP64 oracle receive
the arrays it returns.

What stands in for what (the paper's precursor RANS data and DNS statistics
are not available):

* Mode table: directions d uniform on the sphere, unit amplitude directions
  sigma perpendicular to d at a uniform angle, phases phi ~ U[0, 2 pi),
  temporal frequencies omega = omega~ / T_ref with omega~ ~ Normal(0, 2 pi)
  and T_ref = delta / U_c steps, wavenumbers in geometric progression between
  k_e / 2 and 1.5 k_cut, spectral weights q from a von Karman-Pao-type shape
  with a cut-off (the paper names a "modified von Karman spectrum" without
  constants; Sec. III.A).  sum(q) = 1.
* Reynolds stresses: smooth SPD profiles in units of u_tau^2 with
  eta = (y + 1/2)/delta - 1:  R11 = 1 + 3 eta^2, R22 = 0.5 + 0.5 eta^2,
  R33 = 0.7 + 0.8 eta^2, R21 = eta (linear total shear stress), R31 = R32 = 0.
* RANS k and omega (for the per-row spectrum): k = tr(R)/2 of the synthetic
  Reynolds stresses; omega = sqrt(k) / (0.09^(1/4) l_m) with the mixing
  length l_m = min(0.41 d_w, 0.09 delta), d_w = distance of the row centre
  to the nearer wall.  A textbook mixing-length closure standing in for the
  k-omega precursor.
* Initial perturbations: uniform noise for a velocity perturbation and a
  population perturbation (the mean profile itself is built by each side).
"""
import numpy as np

SEED_BASE = 230404214

# Channel workloads (x streamwise, y wall-normal, z spanwise).
# u_tau solves u_tau u+(Re_tau) = U_c with the Reichardt law (kappa 0.41,
# B 7.8); nu0 = u_tau delta / Re_tau; tau0 = 1/2 + 3 nu0; delta = ny/2.
# The numbers are literal workload constants; a CPU test recomputes them
# with the oracle's wall law.
WORKLOADS = {
    "c1": dict(nx=64, ny=32, nz=32, re_tau=None, u_tau=0.008369396673286735, tau0=0.52,
               n_modes=100, steps=50, ywall=1, storage="f64-oracle"),
    "c2": dict(nx=768, ny=64, nz=192, re_tau=1000.0, u_tau=0.004448498381757104,
               tau0=0.5004270558446486, n_modes=200, steps=1000, ywall=2, storage="f32"),
    "c3": dict(nx=1536, ny=128, nz=384, re_tau=5200.0, u_tau=0.0037741807439038936,
               tau0=0.5001393543659287, n_modes=300, steps=2000, ywall=2, storage="f16dev"),
    "c4": dict(nx=256, ny=64, nz=64, re_tau=1000.0, u_tau=0.004448498381757104,
               tau0=0.5004270558446486, n_modes=200, steps=400, ywall=2, storage="f32"),
    "c5": dict(nx=1536, ny=256, nz=384, re_tau=5200.0, u_tau=0.0037741807439038936,
               tau0=0.5002787087318575, n_modes=300, steps=5000, ywall=2, storage="f32"),
    # the large adjoint run: 512 x 64 x 128 with the Re_tau = 1000 lattice parameters of ny = 64
    "c5a": dict(nx=512, ny=64, nz=128, re_tau=1000.0, u_tau=0.004448498381757104,
                tau0=0.5004270558446486, n_modes=300, steps=2000, ywall=2, storage="f16dev"),
}
# u_tau of the centreline speed U_C at each friction Reynolds number (u_tau u+(Re_tau) = U_C, Reichardt law).
U_TAU_OF_RE = {1000.0: 0.004448498381757104, 2000.0: 0.004137851781451391, 5200.0: 0.0037741807439038936}
U_C = 0.1      # centreline speed, lattice units
CS_SMAG = 0.1  # C_s; C_smag = C_s^2 = 0.01 (Sec. IV.A)


def rng(seed_offset=0):
    return np.random.Generator(np.random.PCG64(SEED_BASE + seed_offset))


def mode_table(n_modes, delta, seed_offset=0, u_c=U_C, k_range=None):
    """Random STG mode parameters (raw draws, no method arithmetic).

    Returns dict with q[N], sigma[3,N], kmag[N], d[3,N], phi[N], omega[N].
    k_range = (k_lo, k_hi) replaces the wavenumber range (q keeps its shape).
    """
    g = rng(seed_offset)
    ct = g.uniform(-1.0, 1.0, n_modes)
    az = g.uniform(0.0, 2 * np.pi, n_modes)
    st = np.sqrt(1.0 - ct * ct)
    d = np.stack([st * np.cos(az), st * np.sin(az), ct])
    # two unit vectors perpendicular to d, sigma at a uniform angle between them
    ref = np.where(np.abs(d[0]) < 0.9, np.array([[1.0], [0.0], [0.0]]), np.array([[0.0], [1.0], [0.0]]))
    e1 = np.cross(d.T, ref.T).T
    e1 /= np.linalg.norm(e1, axis=0)
    e2 = np.cross(d.T, e1.T).T
    ang = g.uniform(0.0, 2 * np.pi, n_modes)
    sigma = np.cos(ang) * e1 + np.sin(ang) * e2
    phi = g.uniform(0.0, 2 * np.pi, n_modes)
    t_ref = delta / u_c
    omega = g.normal(0.0, 2 * np.pi, n_modes) / t_ref
    # wavenumbers: geometric progression from k_e/2 to 1.5 k_cut
    l_e = 0.5 * delta
    k_e = 2 * np.pi / l_e
    k_cut = np.pi
    k_eta = 4 * k_cut
    kmag = np.geomspace(0.5 * k_e, 1.5 * k_cut, n_modes) if k_range is None else np.geomspace(*k_range, n_modes)
    r = kmag / k_e
    E = r ** 4 / (1 + 2.4 * r * r) ** (17.0 / 6.0) * np.exp(-(12 * kmag / k_eta) ** 2) \
        * np.exp(-(4 * np.maximum(kmag - 0.9 * k_cut, 0.0) / k_cut) ** 3)
    dk = np.gradient(kmag)
    q = E * dk
    q /= q.sum()
    return dict(q=q, sigma=sigma, kmag=kmag, d=d, phi=phi, omega=omega)


def reynolds_stress(ny, u_tau):
    """Synthetic SPD Reynolds-stress profiles R[6, ny] = (R11, R21, R22, R31, R32, R33)."""
    delta = ny / 2.0
    eta = (np.arange(ny) + 0.5) / delta - 1.0
    R = np.zeros((6, ny))
    R[0] = 1.0 + 3.0 * eta ** 2
    R[1] = eta
    R[2] = 0.5 + 0.5 * eta ** 2
    R[5] = 0.7 + 0.8 * eta ** 2
    return R * u_tau ** 2


def spectrum_k_range(delta):
    """Wavenumbers for the per-row spectrum: from half the wavenumber of the
    largest eddy length any row can have (2 d_w <= 2 delta) to 1.5 times the
    unit lattice's cut-off pi."""
    return 0.5 * 2 * np.pi / (2 * delta), 1.5 * np.pi


def rans_k_omega(ny, u_tau):
    """Synthetic RANS k[ny], omega[ny] (see the module docstring)."""
    delta = ny / 2
    R = reynolds_stress(ny, u_tau)
    k = 0.5 * (R[0] + R[2] + R[5])
    d_w = np.minimum(np.arange(ny) + 0.5, ny - np.arange(ny) - 0.5)
    l_m = np.minimum(0.41 * d_w, 0.09 * delta)
    return k, np.sqrt(k) / (0.09 ** 0.25 * l_m)


def amp_bins(ny, n_bins=None):
    """Amplitude scalings s_b = 1 with y-rows split evenly over n_bins bins."""
    n_bins = ny if n_bins is None else n_bins
    bin_of_y = (np.arange(ny) * n_bins) // ny
    return np.ones(n_bins), bin_of_y.astype(np.int32)


def perturbations(nx, ny, nz, seed_offset=0, dtype=np.float64):
    """Uniform noise in [-1, 1): du[3, nx, ny, nz] and dpop[19, nx, ny, nz]."""
    g = rng(1000 + seed_offset)
    du = g.uniform(-1.0, 1.0, (3, nx, ny, nz)).astype(dtype)
    dp = g.uniform(-1.0, 1.0, (19, nx, ny, nz)).astype(dtype)
    return du, dp


def smooth_field(nx, ny, nz, seed_offset=0, n_waves=4):
    """A smooth random velocity field u[3, nx, ny, nz] (sums of a few lattice-periodic waves)."""
    g = rng(2000 + seed_offset)
    x = np.arange(nx)[:, None, None]
    y = np.arange(ny)[None, :, None]
    z = np.arange(nz)[None, None, :]
    u = np.zeros((3, nx, ny, nz))
    for a in range(3):
        for _ in range(n_waves):
            kx, ky, kz = g.integers(0, 3, 3)
            ph = g.uniform(0, 2 * np.pi)
            amp = g.uniform(-1, 1)
            u[a] += amp * np.cos(2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / nz) + ph)
    return u / n_waves
