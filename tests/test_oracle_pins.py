"""Pins of the FP64 oracle against facts the mathematics fixes (CPU only).

Each test is chosen so that a plausible slip in the oracle (a dropped term,
a wrong sign or index, swapped assets, a wrong boundary time, a wrong slice
order) breaks at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from synthetic import plain_fp64, EXCHANGE, BASKET

C1 = dict(sigma1=0.3, sigma2=0.2, rho=0.5, r=0.05)


def prob(M, **kw):
    d = dict(C1)
    d.update(kw)
    return oracle.Problem(M=M, **d)


# --- P1: quadratic monomials are exact discrete eigenfunctions -------------------------
@pytest.mark.parametrize("rho", [0.5, -0.7])
@pytest.mark.parametrize("ab", [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1)])
def test_monomial_exact_discrete_solution(ab, rho):
    """Centred differences are exact on x^a y^b (a+b<=2), so explicit Euler
    with the exact ring gives (1 + dt*lambda_ab)^m x^a y^b at every node.
    (2,0)/(0,2) pin 1/2 s1^2 vs 1/2 s2^2, (1,1) the mixed term and its sign,
    (1,0)/(0,1) the drift-reaction balance, (0,0) the reaction term."""
    a, b = ab
    p = prob(65, rho=rho)
    x = oracle.coords(p)
    mono = np.outer(x ** a, x ** b)
    lam = cf.monomial_eigenvalue(a, b, p.sigma1, p.sigma2, p.rho, p.r)
    dt, m = 1.0 / 1024, 1024
    u = mono.copy()
    for q in range(m):
        v = oracle.euler_step(p, dt, u)
        fac = (1.0 + dt * lam) ** (q + 1)
        ring = mono * fac
        v[0, :], v[-1, :], v[:, 0], v[:, -1] = ring[0, :], ring[-1, :], ring[:, 0], ring[:, -1]
        u = v
    expect = mono * (1.0 + dt * lam) ** m
    scale = np.abs(expect).max()
    assert np.abs(u - expect).max() <= 1e-13 * scale
    # the discrete factor approximates the PDE's e^{lambda T} to first order in dt
    assert abs((1.0 + dt * lam) ** m - math.exp(lam)) <= 0.6 * lam * lam * dt * math.exp(abs(lam)) + 1e-15


def test_monomial_factors_c1():
    """The discrete factors at 1024 steps of dt = 1/1024 for the fixed 65^2 parameters."""
    for (a, b), want in {(0, 0): 0.9512282632949352, (1, 1): 1.0832836825843881,
                         (2, 0): 1.1502627914335684, (0, 2): 1.0941699564224536,
                         (1, 0): 1.0, (0, 1): 1.0}.items():
        lam = cf.monomial_eigenvalue(a, b, **C1)
        assert abs((1.0 + lam / 1024) ** 1024 - want) <= 2e-15


def test_operator_on_monomials_pointwise():
    """L_h x^a y^b = lambda_ab x^a y^b at each interior node (one application)."""
    p = prob(17, rho=-0.3)
    x = oracle.coords(p)
    for a, b in [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1)]:
        mono = np.outer(x ** a, x ** b)
        Lu = oracle.apply_operator(p, mono)
        lam = cf.monomial_eigenvalue(a, b, p.sigma1, p.sigma2, p.rho, p.r)
        assert np.allclose(Lu[1:-1, 1:-1], lam * mono[1:-1, 1:-1], rtol=0, atol=1e-13)


# --- closed forms pinned by their definition as risk-neutral expectations ------------
def test_bs_call_matches_expectation():
    from scipy import integrate
    S, K, r, s, tau = 1.3, 1.0, 0.05, 0.3, 0.7

    def integrand(z):
        ST = S * math.exp((r - 0.5 * s * s) * tau + s * math.sqrt(tau) * z)
        return max(ST - K, 0.0) * math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)
    zk = (math.log(K / S) - (r - 0.5 * s * s) * tau) / (s * math.sqrt(tau))   # payoff kink
    val = math.exp(-r * tau) * integrate.quad(integrand, zk, 14, epsabs=1e-14, epsrel=1e-13,
                                              limit=400)[0]
    assert abs(cf.bs_call(S, K, r, s, tau) - val) < 1e-12
    assert abs(cf.bs_call(1.0, 1.0, 0.05, 0.3, 1.0) - 0.1423125478598582) < 1e-13
    assert abs(cf.bs_call(2.0, 1.0, 0.05, 0.3, 1.0) - 1.049652216075794) < 1e-12


def test_margrabe_matches_expectation():
    """E[max(S1_T - S2_T, 0)] e^{-r tau} by 2-D Gauss-Hermite quadrature."""
    x, y, tau, s1, s2, rho, r = 1.0, 1.0, 1.0, 0.3, 0.2, 0.5, 0.05
    z, w = np.polynomial.hermite_e.hermegauss(160)
    w = w / math.sqrt(2 * math.pi)
    Z1, Z2 = np.meshgrid(z, z, indexing="ij")
    W = np.outer(w, w)
    e1 = Z1
    e2 = rho * Z1 + math.sqrt(1 - rho * rho) * Z2
    ST1 = x * np.exp((r - 0.5 * s1 * s1) * tau + s1 * math.sqrt(tau) * e1)
    ST2 = y * np.exp((r - 0.5 * s2 * s2) * tau + s2 * math.sqrt(tau) * e2)
    val = math.exp(-r * tau) * float((np.maximum(ST1 - ST2, 0.0) * W).sum())
    mg = cf.margrabe(x, y, tau, s1, s2, rho)
    assert abs(mg - val) < 2e-5      # kink limits Gauss-Hermite accuracy
    assert abs(mg - 0.10524315781125254) < 1e-14
    # the C oracle's boundary routine uses an independently written Margrabe
    assert abs(oracle.lib().orc_margrabe(x, y, tau, s1, s2, rho) - mg) < 1e-15


# --- P2: F against Margrabe for the exchange option -------------------------------------
def _exchange_err(M, mF, bc=oracle.BC_FORWARD_INTRINSIC):
    p = prob(M, payoff_kind=oracle.PAYOFF_EXCHANGE, bc_kind=bc)
    u = oracle.serial_fine(p, 8, 1.0, mF)
    k = (M - 1) // 4   # node (1, 1)
    return u[k, k] - cf.margrabe(1.0, 1.0, 1.0, p.sigma1, p.sigma2, p.rho), u, p


@pytest.mark.slow
def test_fine_second_order_against_margrabe():
    e65, _, _ = _exchange_err(65, 128)
    e129, _, _ = _exchange_err(129, 512)
    e257, _, _ = _exchange_err(257, 2048)
    assert abs(e65) <= 2e-4
    assert 3.5 <= e65 / e129 <= 4.6
    assert 3.5 <= e129 / e257 <= 4.6


def test_fine_window_against_margrabe_exact_bc():
    errs = []
    for M, mF in [(65, 128), (129, 512)]:
        _, u, p = _exchange_err(M, mF, bc=oracle.BC_EXACT)
        x = oracle.coords(p)
        sel = (x >= 0.25) & (x <= 2.5)
        ref = np.array([[cf.margrabe(a, b, 1.0, p.sigma1, p.sigma2, p.rho) for b in x[sel]]
                        for a in x[sel]])
        errs.append(np.abs(u[np.ix_(sel, sel)] - ref).max())
    assert errs[0] < 2e-3
    assert 3.2 <= errs[0] / errs[1] <= 4.8


# --- P3: the one-asset reduction ----------------------------------------------------------
def _bs_row(M, mF, **kw):
    p = prob(M, payoff_kind=oracle.PAYOFF_BASKET, w1=1.0, w2=0.0, strike=1.0,
             bc_kind=oracle.BC_EXACT, **kw)
    u = oracle.serial_fine(p, 8, 1.0, mF)
    x = oracle.coords(p)
    j = int(round(2.0 / p.h))
    ref = np.array([cf.bs_call(a, 1.0, p.r, p.sigma1, 1.0) for a in x])
    return u, j, ref


def test_one_asset_reduction():
    u65, j65, ref65 = _bs_row(65, 128)
    u129, j129, ref129 = _bs_row(129, 512)
    e65 = np.abs(u65[:, j65] - ref65).max()
    e129 = np.abs(u129[:, j129] - ref129).max()
    assert e65 <= 1e-3
    assert 3.5 <= e65 / e129 <= 4.6
    # sigma2 and rho act only through y-differences.  The exact ring differs from the
    # discrete interior by the discretisation error, so y-differences do not vanish near
    # the y-edges; two units away from them, at S2 = 2, the effect has decayed below 1e-5.
    for kw in (dict(sigma2=0.25, rho=-0.6), dict(sigma2=0.1, rho=0.8)):   # stable at dt=1/1024
        u_alt, _, _ = _bs_row(65, 128, **kw)
        assert np.abs(u_alt[:, j65] - u65[:, j65]).max() < 1e-5
    assert np.abs(u65[:, j65 - 4:j65 + 5] - u65[:, [j65]]).max() < 1e-5


# --- P4: Parareal algebra -------------------------------------------------------------
@pytest.mark.parametrize("fg", [(0.9, 0.7), (1.1, 0.95), (-0.5, 0.3)])
def test_scalar_parareal_binomial(fg):
    f, g = fg
    N = 6
    u0 = np.array([1.0, -2.0, 0.5])
    for k in range(1, N + 1):
        U, K, _ = oracle.parareal_generic(u0, N, lambda n, v: f * v, lambda n, v: g * v,
                                          max_iters=k, tol=0.0)
        assert K == k
        for n in range(N + 1):
            want = cf.scalar_parareal(f, g, 1.0, k, n) * u0
            assert np.allclose(U[n], want, rtol=1e-13, atol=1e-15), (k, n)


def test_parareal_slice_dependent_propagators():
    """Propagators that depend on the slice index pin which slice is used where:
    the result must be prod_{n} f_n at the last slice after N iterations."""
    N = 5
    fs = [1.1, 0.9, 1.3, 0.7, 1.05]
    gs = [1.0, 1.0, 1.2, 0.8, 1.0]
    U, K, _ = oracle.parareal_generic(np.array([1.0]), N, lambda n, v: fs[n] * v,
                                      lambda n, v: gs[n] * v, max_iters=N, tol=0.0)
    assert K == N
    assert abs(U[N][0] - np.prod(fs)) < 1e-14
    U1, _, _ = oracle.parareal_generic(np.array([1.0]), N, lambda n, v: fs[n] * v,
                                       lambda n, v: gs[n] * v, max_iters=1, tol=0.0)
    # after one iteration: U^1_n = g_{n-1} U^1_{n-1} + (f_{n-1} - g_{n-1}) U^0_{n-1}
    U0 = np.cumprod([1.0] + gs)
    want = [1.0]
    for n in range(N):
        want.append(gs[n] * want[-1] + (fs[n] - gs[n]) * U0[n])
    assert np.allclose(U1[:, 0], want, rtol=1e-14)


def _c1_problems(payoff=BASKET, M=65, Mc=33):
    inst = plain_fp64(payoff)
    kw = dict(sigma1=inst.sigma1, sigma2=inst.sigma2, rho=inst.rho, r=inst.r,
              payoff_kind=inst.payoff, w1=inst.w1, w2=inst.w2, strike=inst.strike)
    return oracle.Problem(M=M, **kw), oracle.Problem(M=Mc, **kw), inst


def test_finite_termination_bitwise():
    pf, pc, inst = _c1_problems()
    ser = oracle.serial_fine(pf, inst.n_slices, inst.T, inst.fine_steps_per_slice)
    U, K, inc = oracle.parareal_bs(pf, pc, inst.n_slices, inst.T, inst.fine_steps_per_slice,
                                   inst.coarse_steps_per_slice, max_iters=inst.n_slices, tol=0.0)
    assert K == inst.n_slices
    assert np.array_equal(U, ser)


def test_converged_prefix_exact():
    """U^k_n = F^n u0 bitwise for n <= k (generic driver with the PDE propagators)."""
    pf, pc, _ = _c1_problems(M=17, Mc=9)
    N, T, mF, mG = 4, 1.0, 64, 16
    dT = T / N
    Fn = lambda n, v: oracle.fine(pf, mF, dT / mF, n * dT, v)
    Gn = lambda n, v: oracle.coarse(pf, pc, mG, dT / mG, n * dT, v)
    u0 = oracle.payoff_grid(pf)
    serial = [u0.ravel()]
    for n in range(N):
        serial.append(Fn(n, serial[-1]).ravel())
    for k in range(1, N + 1):
        U, K, _ = oracle.parareal_generic(u0, N, Fn, Gn, max_iters=k, tol=0.0)
        for n in range(k + 1):
            assert np.array_equal(U[n], serial[n]), (k, n)
        if k < N:
            assert not np.array_equal(U[N], serial[N])


def test_G_equal_F_stops_after_one_iteration():
    pf, pc, inst = _c1_problems()
    ser = oracle.serial_fine(pf, inst.n_slices, inst.T, inst.fine_steps_per_slice)
    U, K, inc = oracle.parareal_bs(pf, pc, inst.n_slices, inst.T, inst.fine_steps_per_slice,
                                   inst.coarse_steps_per_slice, coarse_kind=oracle.G_FINE,
                                   tol=1e-8)
    assert K == 1 and inc[0] == 0.0
    assert np.array_equal(U, ser)


def test_c1_parareal_reaches_serial():
    """With the spatially coarsened G the increments shrink slowly (the payoff kink next
    to the degenerate edges S1 = 0, S2 = 0 is neither resolved by the coarse grid nor
    smoothed by F), so the 1e-8 tolerance is met by finite termination at K = N, where
    the result equals serial F bitwise."""
    for payoff in (BASKET, EXCHANGE):
        pf, pc, inst = _c1_problems(payoff)
        ser = oracle.serial_fine(pf, inst.n_slices, inst.T, inst.fine_steps_per_slice)
        U, K, inc = oracle.parareal_bs(pf, pc, inst.n_slices, inst.T, inst.fine_steps_per_slice,
                                       inst.coarse_steps_per_slice, tol=inst.tol)
        assert 1 <= K <= inst.n_slices
        if K == inst.n_slices:
            assert np.array_equal(U, ser)
        else:
            assert inc[-1] < inst.tol
        assert inc[-1] < inc[0]


def test_nonfinite_increment_detected():
    with pytest.raises(FloatingPointError):
        oracle.parareal_generic(np.array([1.0]), 3, lambda n, v: v * np.nan, lambda n, v: v,
                                max_iters=3, tol=0.0)


# --- P6: transfers ---------------------------------------------------------------------
@pytest.mark.parametrize("Mf,Mc", [(65, 33), (513, 129), (33, 9)])
def test_restrict_prolong_identity(Mf, Mc):
    rng = np.random.default_rng(Mf)
    c = rng.standard_normal((Mc, Mc))
    assert np.array_equal(oracle.restrict(Mf, Mc, oracle.prolong(Mc, Mf, c)), c)


def test_prolong_exact_on_bilinear():
    Mf, Mc = 65, 17
    X = np.linspace(0, 4, Mc)
    x = np.linspace(0, 4, Mf)
    f = lambda a, b: 0.3 + 1.7 * a - 0.4 * b + 0.25 * a * b
    P = oracle.prolong(Mc, Mf, f(X[:, None], X[None, :]))
    assert np.abs(P - f(x[:, None], x[None, :])).max() < 1e-13


def test_coarse_output_ring_is_exact_bc():
    pf, pc, _ = _c1_problems()
    u = oracle.payoff_grid(pf)
    tau0, m, dt = 0.25, 16, 0.125 / 16
    G = oracle.coarse(pf, pc, m, dt, tau0, u)
    x = oracle.coords(pf)
    t1 = tau0 + m * dt
    for k in (0, 7, 64):
        assert G[0, k] == oracle.bc(pf, 0.0, x[k], t1)
        assert G[k, -1] == oracle.bc(pf, x[k], x[-1], t1)


# --- time step planning -------------------------------------------------------------
def test_gershgorin_bound_guarantees_stability():
    """Assemble the explicit update matrix column by column from the oracle's
    own operator and check its spectral radius at the planned bound."""
    p = prob(17, rho=-0.6, r=0.09)
    M = p.M
    n_in = (M - 2) ** 2
    A = np.zeros((n_in, n_in))
    idx = [(i, j) for i in range(1, M - 1) for j in range(1, M - 1)]
    for c, (i, j) in enumerate(idx):
        e = np.zeros((M, M))
        e[i, j] = 1.0
        A[:, c] = oracle.apply_operator(p, e)[1:-1, 1:-1].ravel()
    dt = oracle.stable_dt(p)
    lam = np.linalg.eigvals(A)
    assert np.abs(1.0 + dt * lam).max() <= 1.0 + 1e-12
    # the bound is within a factor 2 of the true limit 2/|lambda|_max for the real spectrum
    assert dt * np.abs(lam).max() > 1.0


def test_stable_dt_c1_value():
    p = prob(65)
    worst = 63 * 63 * (2 * 0.09 + 2 * 0.04 + 0.5 * 0.3 * 0.2) + 0.05
    assert abs(oracle.stable_dt(p) - 2.0 / worst) < 1e-18
    assert oracle.steps_for(p, 1.0 / 8, 0.9) == math.ceil((1.0 / 8) / (0.9 * 2.0 / worst))
