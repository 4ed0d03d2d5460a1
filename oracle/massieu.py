"""Oracle (test infrastructure only): residual Massieu-potential derivatives
A^r_mn from the moment sums an NVT run accumulates (Sec. 3, Eq. 1), and the
thermodynamic properties that follow from the first five derivatives.

Plain FP64 numpy, written from the statistical mechanics below; nothing here
is shared with the library.

Definition (Sec. 3, Eq. 1): A_mn = beta^m rho^n d^(m+n)(F/(N k T)) / d beta^m
d rho^n with beta = 1/T (k = 1), rho = N/V.  With molecular scaling (scaled
centres s = R/L fixed, bodies rigid), the residual part is

    A^r(beta, V) = -phi / N,   phi = ln INT exp(-beta U(s; V)) ds,

so derivatives of phi are canonical averages over the sampled ensemble:

    phi_b   = -<U>                  phi_bb  = k2(U)
    phi_bbb = -k3(U)                phi_V   = -beta <U_V>
    phi_VV  = -beta <U_VV> + beta^2 k2(U_V)
    phi_bV  = -<U_V> + beta k(U, U_V)
    phi_bbV = 2 k(U, U_V) - beta k(U, U, U_V)
    phi_bVV = -<U_VV> + beta k(U, U_VV) + 2 beta k2(U_V) - beta^2 k(U_V, U_V, U)

(k = joint cumulants, from d<A>/d beta = -k(A, U) and d<A>/dV = <A_V> -
beta k(A, U_V) for an observable A(s; V)).  Density derivatives follow from
rho d/d rho = -V d/dV and rho^2 d^2/d rho^2 = 2V d/dV + V^2 d^2/dV^2.

The moment sums are those of X = U - u0, Y = U_V = dU/dV and Z = U_VV; all
cumulants of order >= 2 are shift-invariant, so only <U> = u0 + <X> needs the
shift.
"""
import numpy as np

# order of the moment sums: count, X, X^2, X^3, Y, XY, X^2Y, Y^2, XY^2, Z, XZ
M_N, M_X, M_XX, M_XXX, M_Y, M_XY, M_XXY, M_YY, M_XYY, M_Z, M_XZ = range(11)

# order of the eight residual derivatives
A_ORDER = ("10", "01", "20", "11", "02", "30", "21", "12")


def residual_derivatives(moments, u0, temperature, volume, n_mol):
    """The eight A^r_mn (dict keyed '10', '01', ...) from the moment sums."""
    m = np.asarray(moments, dtype=np.float64)
    count = m[M_N]
    if count <= 0:
        raise ValueError("no samples")
    beta, V, N = 1.0 / temperature, float(volume), float(n_mol)
    mean = m / count
    x, y, z = mean[M_X], mean[M_Y], mean[M_Z]
    # second- and third-order (joint) cumulants from raw moments
    k_xx = mean[M_XX] - x * x
    k_xxx = mean[M_XXX] - 3.0 * mean[M_XX] * x + 2.0 * x ** 3
    k_xy = mean[M_XY] - x * y
    k_yy = mean[M_YY] - y * y
    k_xz = mean[M_XZ] - x * z
    k_xxy = mean[M_XXY] - 2.0 * x * mean[M_XY] - mean[M_XX] * y + 2.0 * x * x * y
    k_xyy = mean[M_XYY] - x * mean[M_YY] - 2.0 * y * mean[M_XY] + 2.0 * x * y * y

    phi_b = -(u0 + x)
    phi_bb = k_xx
    phi_bbb = -k_xxx
    phi_V = -beta * y
    phi_VV = -beta * z + beta ** 2 * k_yy
    phi_bV = -y + beta * k_xy
    phi_bbV = 2.0 * k_xy - beta * k_xxy
    phi_bVV = -z + beta * k_xz + 2.0 * beta * k_yy - beta ** 2 * k_xyy

    # A^r = -phi / N; beta^m d^m/d beta^m and the density operators above
    a = {
        "10": -beta * phi_b / N,
        "20": -beta ** 2 * phi_bb / N,
        "30": -beta ** 3 * phi_bbb / N,
        "01": V * phi_V / N,                                  # -V d/dV of -phi/N
        "02": -(2.0 * V * phi_V + V * V * phi_VV) / N,
        "11": beta * V * phi_bV / N,
        "21": beta ** 2 * V * phi_bbV / N,
        "12": -beta * (2.0 * V * phi_bV + V * V * phi_bVV) / N,
    }
    return a


def ideal_parts(dof):
    """A^i_mn of classical rigid molecules with `dof` quadratic degrees of
    freedom (3 translational + rotational): the ideal Massieu function is
    (dof / 2) ln(beta) + ln(rho) + const per molecule."""
    f = float(dof)
    return {"10": f / 2.0, "20": -f / 2.0, "30": f, "01": 1.0, "02": -1.0, "11": 0.0, "21": 0.0, "12": 0.0}


def properties(a_res, dof):
    """Properties per molecule (k = 1) from A_mn = A^i_mn + A^r_mn.

    Helmholtz energy per N k T is a(beta, rho) = A; with p = rho^2 da/drho / beta
    and u = da/dbeta:
      Z = p / (rho k T)            = A_01 (= 1 + A^r_01)
      u / (k T)                    = A_10
      c_v / k                      = -A_20
      (dp/drho)_T / (k T)          = 2 A_01 + A_02  (= 1 + 2 A^r_01 + A^r_02)
      (dp/dT)_rho / (rho k)        = A_01 - A_11
      c_p / k                      = c_v / k + ((dp/dT)_rho / (rho k))^2 / ((dp/drho)_T / (k T))
      w^2 m / (k T)                = (dp/drho)_s m / (k T) = (c_p / c_v) (dp/drho)_T / (k T)
      rho k T kappa_T              = 1 / ((dp/drho)_T / (k T))
    """
    ai = ideal_parts(dof)
    A = {k: ai[k] + a_res[k] for k in A_ORDER}
    dpdrho = 2.0 * A["01"] + A["02"]           # ideal: 2 - 1 = 1
    dpdT = A["01"] - A["11"]
    cv = -A["20"]
    cp = cv + dpdT * dpdT / dpdrho
    return {"Z": A["01"], "u_kT": A["10"], "cv_k": cv, "cp_k": cp, "dpdrho_kT": dpdrho,
            "dpdT_rhok": dpdT, "w2_m_kT": cp / cv * dpdrho, "rho_kT_kappaT": 1.0 / dpdrho}
