"""Independent textbook references for pinning the oracle (test code only).

Dense matrices are built with numpy.kron from the 2x2 Pauli matrices, qubit 1
being the rightmost Kronecker factor so that its bit is the least significant
one (Sec. II.A, eq. (ztensor)).  Propagation uses scipy's matrix exponential.
"""
import numpy as np
import scipy.linalg

I2 = np.eye(2, dtype=np.complex128)
SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def dense_pauli(n, x, z):
    mats = []
    for q in range(n, 0, -1):            # qubit n leftmost, qubit 1 rightmost
        b = 1 << (q - 1)
        xb, zb = bool(int(x) & b), bool(int(z) & b)
        mats.append(SY if (xb and zb) else SX if xb else SZ if zb else I2)
    out = np.array([[1.0 + 0j]])
    for m in mats:
        out = np.kron(out, m)
    return out


def sched_value(sched, t, path):
    # a second, independent evaluation of the schedules for the references
    T = path["T"]
    s = t / T if path["kind"] == "linear" else np.sin(np.pi * t / (2 * T)) ** 2
    if sched["kind"] == "const":
        return 1.0
    if sched["kind"] == "trig_t":
        return sched["amp"] * np.cos(sched["omega"] * t + sched["phase"])
    if sched["kind"] == "pwl_s":
        xs, vs = zip(*sched["knots"])
        return float(np.interp(s, xs, vs))
    hi_ok = s <= sched["s_hi"] if sched.get("hi_closed") else s < sched["s_hi"]
    if not (s >= sched["s_lo"] and hi_ok):
        return 0.0
    return float(np.polyval(list(reversed(sched["coef"])), s))


def dense_h(inst, t):
    N = 1 << inst.n
    H = np.zeros((N, N), dtype=np.complex128)
    for l in range(len(inst.w)):
        c = inst.w[l] * sched_value(inst.scheds[inst.sid[l]], t, inst.path)
        if c != 0.0:
            H += c * dense_pauli(inst.n, inst.x[l], inst.z[l])
    return H


def magnus4_propagate(inst, psi0, t0, t1, K):
    """Fourth-order Magnus integrator with two Gauss-Legendre nodes per step."""
    h = (t1 - t0) / K
    c1, c2 = 0.5 - np.sqrt(3) / 6, 0.5 + np.sqrt(3) / 6
    psi = np.array(psi0, dtype=np.complex128)
    for k in range(K):
        t = t0 + k * h
        A1 = -1j * dense_h(inst, t + c1 * h)
        A2 = -1j * dense_h(inst, t + c2 * h)
        Om = 0.5 * h * (A1 + A2) + (np.sqrt(3) / 12) * h * h * (A2 @ A1 - A1 @ A2)
        psi = scipy.linalg.expm(Om) @ psi
    return psi
