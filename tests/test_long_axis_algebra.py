"""The algebra the long-axis kernels rely on, checked on the CPU against direct
computations (no GPU, no oracle): the four-step FFT split with the two real lines packed
as one complex line and untangled through the partner slot of N - k, the slot order of
the kept rows and the inverse rebuilt from conjugates; and the segmented Crank-Nicolson
sweep, whose segments are joined by carries computed from fixed products P, Q and fixed
summary weights w, u of the factor table (the increment form of the sweep: d_i = f_i
Delta_i + g_i d_(i-1), e_i = d_i + g_i e_(i+1), u = psi + e, g = f / 2)."""
import numpy as np
import pytest


def four_step_r2c(rho, A, B):
    """Rows kb <= B/2 of the kept spectrum slots (spec[j][kb A + ka] = X_j[B ka + kb]) of
    the lines of rho, two lines packed per complex line, following the kernels' steps."""
    n1, N = rho.shape
    Bh = B // 2 + 1
    w4 = np.exp(-2j * np.pi * np.arange(N) / N)
    spec = np.zeros((n1, Bh * A), complex)
    for jp in range((n1 + 1) // 2):
        j = 2 * jp
        z = rho[j] + 1j * (rho[j + 1] if j + 1 < n1 else 0.0)
        W = np.zeros((B, A), complex)
        for a in range(A):                        # B-point columns, twiddle W_N^(a kb)
            W[:, a] = np.fft.fft(z[a + A * np.arange(B)]) * w4[a * np.arange(B)]
        Z = np.fft.fft(W, axis=1)                 # A-point rows: Z[kb, ka] = X[B ka + kb]
        for kb in range(Bh):
            for ka in range(A):
                if kb == 0:
                    zm = Z[0, (A - ka) % A]
                elif 2 * kb == B:
                    zm = Z[kb, A - 1 - ka]
                else:
                    zm = Z[B - kb, A - 1 - ka]
                zk = Z[kb, ka]
                spec[j, kb * A + ka] = (zk + np.conj(zm)) / 2
                if j + 1 < n1:
                    spec[j + 1, kb * A + ka] = (zk - np.conj(zm)) / 2j
    return spec


def four_step_c2r(spec, N, A, B, n1):
    """The inverse: rows past B/2 from the conjugates of row B - kb (columns reversed),
    inverse A-point rows, conjugate twiddle, inverse B-point columns (unnormalised)."""
    Bh = B // 2 + 1
    w4 = np.exp(-2j * np.pi * np.arange(N) / N)
    out = np.zeros((n1, N))
    for jp in range((n1 + 1) // 2):
        j = 2 * jp
        W = np.zeros((B, A), complex)
        for kb in range(B):
            Z = np.zeros(A, complex)
            for ka in range(A):
                mirror = kb >= Bh
                src = (B - kb) * A + (A - 1 - ka) if mirror else kb * A + ka
                a_ = spec[j, src]
                b_ = spec[j + 1, src] if j + 1 < n1 else 0.0
                Z[ka] = np.conj(a_) + 1j * np.conj(b_) if mirror else a_ + 1j * b_
            W[kb] = np.fft.ifft(Z) * A * np.conj(w4[np.arange(A) * kb])
        for a in range(A):
            x = np.fft.ifft(W[:, a]) * B
            out[j, a + A * np.arange(B)] = x.real
            if j + 1 < n1:
                out[j + 1, a + A * np.arange(B)] = x.imag
    return out


@pytest.mark.parametrize("N,A,B,n1", [(24, 6, 4, 5), (35, 7, 5, 4), (36, 6, 6, 3),
                                      (30, 6, 5, 2), (21, 7, 3, 3)])
def test_four_step_slots_partners_and_inverse(N, A, B, n1):
    rng = np.random.default_rng(N * 100 + n1)
    rho = rng.standard_normal((n1, N))
    spec = four_step_r2c(rho, A, B)
    ref = np.fft.fft(rho, axis=1)
    for kb in range(B // 2 + 1):
        for ka in range(A):
            np.testing.assert_allclose(spec[:, kb * A + ka], ref[:, B * ka + kb], atol=1e-12)
    np.testing.assert_allclose(four_step_c2r(spec, N, A, B, n1) / N, rho, atol=1e-12)


def cn_factors(N, A):
    """Factor table f_i = 2 A m_i of (1 + 2A) u_i - A (u_(i-1) + u_(i+1)) (Thomas factors
    m; zero on the two boundary rows)."""
    a, b = -A, 1 + 2 * A
    f = np.zeros(N, complex)
    c = 0
    for i in range(1, N - 1):
        m = 1 / (b - a * c)
        c = a * m
        f[i] = 2 * A * m
    return f


def sweep(psi, f):
    N = len(psi)
    g = f / 2
    D = np.zeros(N, complex)
    D[1:-1] = psi[:-2] + psi[2:] - 2 * psi[1:-1]
    d = np.zeros(N, complex)
    prev = 0
    for i in range(N):
        prev = f[i] * D[i] + g[i] * prev
        d[i] = prev
    e = np.zeros(N, complex)
    nxt = 0
    for i in range(N - 1, -1, -1):
        nxt = d[i] + g[i] * nxt
        e[i] = nxt
    return psi + e


def segment_tables(f, sn):
    """P, Q per segment and the summary weights w, u per row, as the set-up kernel forms
    them (products taken within each segment)."""
    N = len(f)
    g = f / 2
    P, Q = [], []
    w, u = np.zeros(N, complex), np.zeros(N, complex)
    for s in range(N // sn):
        a, b = s * sn, s * sn + sn - 1
        G = np.zeros(N, complex)
        acc = 1
        for i in range(a, b + 1):
            G[i] = acc                              # g_a ... g_(i-1)
            acc *= g[i]
        S, R = 0, 1
        for i in range(b, a - 1, -1):
            S = G[i] + (g[i + 1] if i < b else 0) * S
            w[i], u[i] = f[i] * R, f[i] * S
            R *= g[i]
        P.append(acc)
        Q.append(g[a] * S)
    return np.array(P), np.array(Q), w, u


def segmented_sweep(psi, f, sn):
    """Summaries from the weights, carries along the line, then each segment's sweep from
    its carries and its neighbours' values before the sweep."""
    N = len(psi)
    ns = N // sn
    g = f / 2
    P, Q, w, u = segment_tables(f, sn)
    ext = np.concatenate([[0], psi, [0]])
    D = ext[:-2] + ext[2:] - 2 * ext[1:-1]          # the long line's second differences
    Bf = [np.sum(w[s * sn:(s + 1) * sn] * D[s * sn:(s + 1) * sn]) for s in range(ns)]
    Bb = [np.sum(u[s * sn:(s + 1) * sn] * D[s * sn:(s + 1) * sn]) for s in range(ns)]
    C = np.zeros(ns, complex)
    c = 0
    for s in range(ns):
        C[s] = c
        c = P[s] * c + Bf[s]
    E = np.zeros(ns + 1, complex)
    for s in range(ns - 1, -1, -1):
        E[s] = Bb[s] + Q[s] * C[s] + P[s] * E[s + 1]
    out = np.zeros(N, complex)
    for s in range(ns):
        a = s * sn
        prev = C[s]
        d = np.zeros(sn, complex)
        for i in range(sn):
            prev = f[a + i] * D[a + i] + g[a + i] * prev
            d[i] = prev
        nxt = E[s + 1]
        for i in range(sn - 1, -1, -1):
            nxt = d[i] + g[a + i] * nxt
            out[a + i] = psi[a + i] + nxt
    return out


@pytest.mark.parametrize("A", [0.3, 0.4j, 15.0, 60j])   # imaginary / real time, mild and stiff
@pytest.mark.parametrize("N,sn", [(48, 12), (60, 20), (64, 32)])
def test_segmented_sweep_equals_direct_solve(N, sn, A):
    rng = np.random.default_rng(N + sn)
    psi = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    psi[0] = psi[-1] = 0
    f = cn_factors(N, A)
    ref = sweep(psi, f)
    got = segmented_sweep(psi, f, sn)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # and the direct solve is the Crank-Nicolson system itself
    M = np.eye(N - 2) * (1 + 2 * A) - A * (np.eye(N - 2, k=1) + np.eye(N - 2, k=-1))
    rhs = A * psi[:-2] + (1 - 2 * A) * psi[1:-1] + A * psi[2:]
    np.testing.assert_allclose(ref[1:-1], np.linalg.solve(M, rhs), atol=1e-10)
