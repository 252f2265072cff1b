"""One relativistic lattice Boltzmann time step, stage by stage (the oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).  Plain NumPy, FP64.

Units and conventions (the paper uses natural units, Sec. III A, and leaves the
lattice normalisation implicit; readings listed in the design notes):
  * lattice units: spacing 1, c = 1, time step dt = cfl (0 < cfl <= 1), T0 = 1;
  * populations F_q are the energy-weighted angular distribution
    F(v) = (1/alpha!) int dp p^alpha f(p v) with alpha = D (Sec. III B);
  * T^{mu nu} = sum_q w_q F_q v_q^mu v_q^nu with v^0 = 1, i.e. the moment
    integral of Sec. III A evaluated with the quadrature, overall constant 1;
  * metric g = diag(-1, +1, ..., +1), so T_eq = (eps + P) u u + P g has
    T^{00} = eps at rest (Sec. III A, ideal-fluid tensor) and the Landau
    condition reads T^{mu nu} u_nu = -eps u^mu;
  * arrays: populations (Q, ny, nx); fields (ny, nx); x is the fast axis.
Only the first D spatial components take part (D = 3 for the paper's
spherical stencil, D = 2 for the in-plane circle stencil).
"""
import numpy as np

from . import forcing as _forcing

# ---------------------------------------------------------------------------
# (b) streaming
# ---------------------------------------------------------------------------


def stream(F, st, cfl):
    """Pull-stream every population along its direction by linear interpolation.

    Sec. II (LB algorithm, streaming step) and Sec. III B: the spherical
    momentum set is off-lattice, so streaming interpolates linearly.  Reading:
    population q arriving at node x comes from the point x - cfl * v_q in the
    lattice plane (the out-of-plane component moves along the single periodic
    z layer and changes nothing); its value there is the bilinear interpolant
    of the four surrounding nodes; boundaries are periodic (Sec. V).
    """
    out = np.empty_like(F)
    for q in range(st.Q):
        sx = -cfl * st.v[q, 0]
        sy = -cfl * st.v[q, 1]
        ix, iy = int(np.floor(sx)), int(np.floor(sy))
        tx, ty = sx - ix, sy - iy

        def at(dx, dy, plane=F[q]):
            # value at node (x + ix + dx, y + iy + dy), periodic
            return np.roll(plane, shift=(-(iy + dy), -(ix + dx)), axis=(0, 1))

        out[q] = ((1 - tx) * (1 - ty) * at(0, 0) + tx * (1 - ty) * at(1, 0)
                  + (1 - tx) * ty * at(0, 1) + tx * ty * at(1, 1))
    return out


# ---------------------------------------------------------------------------
# (c) moments and the Landau frame
# ---------------------------------------------------------------------------


def moments(F, st):
    """Energy-momentum tensor and the third moment of the populations.

    Sec. III A (T^{alpha beta} as a momentum integral) evaluated with the
    quadrature of Sec. III B.  Returns
      T  (D+1, D+1, ny, nx): T^{mu nu} = sum_q w_q F_q v^mu v^nu, v^0 = 1
      R  (D, D, D, ny, nx):  R^{ijk}  = sum_q w_q F_q v^i v^j v^k
    (R is needed only by the force term of Sec. III C.)
    """
    d = st.D
    v4 = np.concatenate([np.ones((st.Q, 1)), st.v[:, :d]], axis=1)
    T = np.einsum("q,qa,qb,qyx->abyx", st.w, v4, v4, F)
    vs = st.v[:, :d]
    R = np.einsum("q,qi,qj,qk,qyx->ijkyx", st.w, vs, vs, vs, F)
    return T, R


def landau(T):
    """Energy density and fluid velocity from the Landau-Lifshitz condition.

    Sec. III A and III B: u is the timelike eigenvector of the mixed tensor and
    eps its eigenvalue.  With g = diag(-1, 1, ...), T g u = -eps u.  Solved per
    site with ``numpy.linalg.eig``; the eigenvector with u.g.u < 0 is taken,
    normalised to u.g.u = -1 with u^0 > 0.
    Returns eps (ny, nx) and u (D+1, ny, nx).
    """
    n = T.shape[0]
    g = np.diag([-1.0] + [1.0] * (n - 1))
    M = np.einsum("abyx,bc->yxac", T, g)
    lam, vec = np.linalg.eig(M)                    # (ny,nx,n), (ny,nx,n,n)
    lam = lam.real
    vec = vec.real
    norm = np.einsum("yxai,ab,yxbi->yxi", vec, g, vec)  # u.g.u per eigenvector
    pick = np.argmin(norm, axis=-1)
    if np.any(np.take_along_axis(norm, pick[..., None], -1) >= 0):
        raise FloatingPointError("no timelike eigenvector: state is not physical")
    eps = -np.take_along_axis(lam, pick[..., None], -1)[..., 0]
    u = np.take_along_axis(vec, pick[..., None, None], -1)[..., 0]   # (ny,nx,n)
    u = u / np.sqrt(-np.einsum("yxa,ab,yxb->yx", u, g, u))[..., None]
    u = u * np.sign(u[..., :1])
    return eps, np.moveaxis(u, -1, 0)


# ---------------------------------------------------------------------------
# (d) equilibrium
# ---------------------------------------------------------------------------


def equilibrium(eps, beta, st):
    """Truncated Juettner equilibrium populations F_eq,q.

    Sec. III A: T_eq = (eps + P) u u + P g with P = eps / D for massless
    particles (D = 3: the ideal-gas P = eps/3 of Sec. III A/B).  Sec. III B:
    the distribution is expanded in the angular polynomials of App. A up to
    second order, with coefficients fixed by the orthogonality relations
    (weights 1, 3, 15/2 for D = 3; in general 1, D, D(D+2)/2):
        a0 = T^{00},  a1_i = D T^{0i},  a2_ij = N2 (T^{ij} - delta_ij T^{00}/D)
        F_eq(v) = a0 P^(0) + a1_i P^(1)_i(v) + a2_ij P^(2)_ij(v)
    with P^(0) = 1, P^(1)_i = v_i, P^(2)_ij = v_i v_j - delta_ij / D.
    eps (ny, nx); beta (D, ny, nx) is the 3-velocity, u = gamma (1, beta).
    """
    d = st.D
    P = eps / d
    gamma = 1.0 / np.sqrt(1.0 - (beta ** 2).sum(axis=0))
    u = np.concatenate([gamma[None], gamma[None] * beta], axis=0)
    g = np.diag([-1.0] + [1.0] * d)
    Teq = (eps + P)[None, None] * u[:, None] * u[None, :] \
        + P[None, None] * g[:, :, None, None]
    N2 = d * (d + 2) / 2.0
    a0 = Teq[0, 0]
    a1 = d * Teq[0, 1:]
    a2 = N2 * (Teq[1:, 1:] - np.eye(d)[:, :, None, None] * Teq[0, 0] / d)
    vs = st.v[:, :d]
    P2 = vs[:, :, None] * vs[:, None, :] - np.eye(d)[None] / d     # (Q, d, d)
    return (a0[None]
            + np.einsum("qi,iyx->qyx", vs, a1)
            + np.einsum("qij,ijyx->qyx", P2, a2))


# ---------------------------------------------------------------------------
# (e) collision and the force term
# ---------------------------------------------------------------------------


def collide(Fs, Feq, beta, tau, st):
    """Anderson-Witting relaxation of the streamed populations.

    Sec. III A: the collision term is -(p^mu u_mu / tau_R)(f - f_eq).  For a
    massless particle p^mu = |p| (1, v); dividing by p^0 gives the relaxation
    rate gamma (1 - beta . v) / tau_R (sign read so that f relaxes towards
    f_eq).  Discretised as in Sec. II (f* = f + dt C) with tau = tau_R / dt.
    """
    d = st.D
    gamma = 1.0 / np.sqrt(1.0 - (beta ** 2).sum(axis=0))
    bv = np.einsum("qi,iyx->qyx", st.v[:, :d], beta)
    omega = gamma[None] * (1.0 - bv) / tau
    return Fs - omega * (Fs - Feq)


def relaxation_time(eps, tau, eta_s=False):
    """Relaxation time of each site, in time steps.

    Sec. III A: the viscosity is eta = tau_R (eps + P)/5 with
    tau_R = 5 (eta/s) / T.  With ``eta_s`` False, tau_R / dt = tau everywhere
    (constant relaxation time).  With ``eta_s`` True, eta/s is held constant
    instead, so tau_R scales as 1/T; for massless particles the energy density
    goes as T^4, and with the lattice normalisation T0 = 1 at eps = 1 the
    local temperature is T = eps^(1/4), giving tau(eps) = tau * eps^(-1/4)
    (``tau`` is the relaxation time at eps = 1, i.e. 5 (eta/s) / dt).
    """
    if not eta_s:
        return tau
    return tau * eps ** -0.25


def force_source(T, R, fx, fy, dt, st, T0=1.0):
    """Population increment of the projected stirring-force term.

    Sec. III C and App. B.  The force F^mu = (0, F^i) enters the kinetic
    equation through F_i d f / d p^i, projected on the polynomials of App. A up
    to second order: F_i d^i_p f ~ exp(-p) sum_n a^(n) P^(n).  For D = 3 the
    coefficients are those printed in App. B,
        a0    = -(F_i / (6 T0)) V[v^i f]
        a1_j  = -(1/2)(F_j / T0) V[f]
        a2_ij =  (5/4) F_k V[f v^k v^i v^j] / T0 - (5/2) F_i V[f v^j] / T0
                 + (5/12) delta_ij F_k V[f v^k] / T0
    where V[.] = int dp p^2 int dOmega/4pi (.) is the number-weighted moment.
    Readings (design notes):
      * closure: the moments are taken from the streamed, pre-collision
        populations with f = exp(-p) A(v), so V[X] = 2! * sum_q w_q F_q X_q
        (V weights p^2, the populations p^3 / 3!); for D = 2 the same
        derivation gives V[X] = 1! * sum_q w_q F_q X_q and the coefficients
        a0 = -F.V1/2, a1 = -F V0,
        a2 = 2 (F_k V3_kij - F_i V1_j - F_j V1_i + delta_ij F.V1 / 2);
      * update: f* = f + dt C - dt F_i d^i_p f, i.e. momentum is injected along
        F (the sign printed in Sec. III C puts the spatial derivative where the
        momentum derivative is meant);
      * the population of exp(-p) sum a P is sum a P (alpha = D weighting), so
        dF_q = -dt (a0 + a1 . v_q + a2 : P^(2)(v_q)).
    fx, fy (ny, nx) are the in-plane force components; F_z = 0.
    """
    d = st.D
    Fvec = np.zeros((d,) + fx.shape)
    Fvec[0], Fvec[1] = fx, fy
    if d == 3:
        closure = 2.0                 # (alpha - 1)! with alpha = 3
        V0 = closure * T[0, 0]
        V1 = closure * T[0, 1:]
        V3 = closure * R
        FV1 = (Fvec * V1).sum(axis=0)
        a0 = -FV1 / (6.0 * T0)
        a1 = -0.5 * Fvec * V0[None] / T0
        a2 = (1.25 * np.einsum("kyx,kijyx->ijyx", Fvec, V3)
              - 2.5 * Fvec[:, None] * V1[None, :]
              + (5.0 / 12.0) * np.eye(3)[:, :, None, None] * FV1[None, None]) / T0
    elif d == 2:
        # Same derivation as App. B with circle averages and alpha = 2:
        # a0 = -F.V1/2!, a1 = -F V0/1!, a2 = (D(D+2)/(2 D!)) [F_k V3_kij
        #      - F_i V1_j - F_j V1_i + delta_ij F.V1 / D] with D = 2.
        closure = 1.0                 # (alpha - 1)! with alpha = 2
        V0 = closure * T[0, 0]
        V1 = closure * T[0, 1:]
        V3 = closure * R
        FV1 = (Fvec * V1).sum(axis=0)
        a0 = -FV1 / (2.0 * T0)
        a1 = -Fvec * V0[None] / T0
        a2 = 2.0 * (np.einsum("kyx,kijyx->ijyx", Fvec, V3)
                    - Fvec[:, None] * V1[None, :] - Fvec[None, :] * V1[:, None]
                    + 0.5 * np.eye(2)[:, :, None, None] * FV1[None, None]) / T0
    else:
        raise ValueError("unsupported angular dimension")
    vs = st.v[:, :d]
    P2 = vs[:, :, None] * vs[:, None, :] - np.eye(d)[None] / d
    proj = (a0[None] + np.einsum("qi,iyx->qyx", vs, a1)
            + np.einsum("qij,ijyx->qyx", P2, a2))
    return -dt * proj


# ---------------------------------------------------------------------------
# the whole step
# ---------------------------------------------------------------------------


def set_state(eps, beta_x, beta_y, st):
    """Step (a) of Sec. II / III C: populations start at the equilibrium."""
    beta = np.zeros((st.D,) + eps.shape)
    beta[0], beta[1] = beta_x, beta_y
    return equilibrium(eps, beta, st)


def check_physical(eps, beta):
    b2 = (beta ** 2).sum(axis=0)
    if not (np.all(np.isfinite(eps)) and np.all(np.isfinite(b2))
            and np.all(eps > 0) and np.all(b2 < 1)):
        raise FloatingPointError("unphysical state (eps <= 0, |beta| >= 1 or non-finite)")


def step(F, st, tau, cfl=1.0, force=None, step_index=0, realization=0, eta_s=False):
    """One RLBM time step, in the order of Sec. III C: (b) stream, (c) moments
    and Landau frame, (d) equilibrium, (e) collide and add the force term.

    ``force`` is None (unforced) or a dict with keys amplitude, k_lo, k_hi,
    seed; the force of this step is drawn with ``step_index`` (Philox counter).
    ``eta_s`` selects the constant-eta/s relaxation time (``relaxation_time``).
    """
    Fs = stream(F, st, cfl)
    T, R = moments(Fs, st)
    eps, u = landau(T)
    beta = u[1:] / u[0]
    check_physical(eps, beta)
    Feq = equilibrium(eps, beta, st)
    Fn = collide(Fs, Feq, beta, relaxation_time(eps, tau, eta_s), st)
    if force is not None and force.get("amplitude", 0.0) != 0.0:
        ny, nx = F.shape[1:]
        fx, fy = _forcing.force_field(nx, ny, force["amplitude"], force["k_lo"],
                                      force["k_hi"], force["seed"], step_index,
                                      realization)
        Fn = Fn + force_source(T, R, fx, fy, cfl, st)
    return Fn


def run(F, st, tau, n, cfl=1.0, force=None, first_step=0, realization=0, eta_s=False):
    for s in range(n):
        F = step(F, st, tau, cfl, force, first_step + s, realization, eta_s)
    return F
