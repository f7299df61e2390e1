"""Mutation check of the oracle pins (CPU only).

Each mutant below plants one plausible mistake in an oracle module (a
dropped term, a wrong sign, factor or index, a transposed or swapped operand,
a wrong stopping rule or output). The mutated module replaces the real one
for the duration of the check, and the pin suites of the oracle run against
it in this process: at least one pin must fail for every mutant. A mutant
that every pin accepts means the pins leave that part of the oracle open.
"""
import importlib
import inspect
import os
import types

import pytest

import oracle
from tests import (test_oracle_approx_pins, test_oracle_cluster_pins, test_oracle_knn_pins,
                   test_oracle_kron_pins, test_oracle_pins)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (module, original text, mutated text, what the mistake is)
MUTANTS = [
    # FISTA (Algorithm 1) and its pieces (Section IV.B)
    ("frpcag", "return 2.0 * (gamma_c * (Lc @ Z.T).T + gamma_r * (Lr @ Z))",
     "return 1.0 * (gamma_c * (Lc @ Z.T).T + gamma_r * (Lr @ Z))", "gradient without its factor 2"),
    ("frpcag", "return 2.0 * (gamma_c * (Lc @ Z.T).T + gamma_r * (Lr @ Z))",
     "return 2.0 * (gamma_r * (Lc @ Z.T).T + gamma_c * (Lr @ Z))", "gradient with the gammas swapped"),
    ("frpcag", "return 2.0 * (gamma_c * (Lc @ Z.T).T + gamma_r * (Lr @ Z))",
     "return 2.0 * (gamma_c * (Lc @ Z.T).T)", "gradient without the row-graph term"),
    ("frpcag", "return Y + np.sign(D) * np.maximum(np.abs(D) - lam, 0.0)",
     "return Y - np.sign(D) * np.maximum(np.abs(D) - lam, 0.0)", "prox with the wrong sign"),
    ("frpcag", "return Y + np.sign(D) * np.maximum(np.abs(D) - lam, 0.0)",
     "return Y + np.sign(D) * np.maximum(np.abs(D) - 2.0 * lam, 0.0)", "prox threshold 2 lambda"),
    ("frpcag", "beta = 2.0 * gamma_c * lmax_c + 2.0 * gamma_r * lmax_r",
     "beta = gamma_c * lmax_c + gamma_r * lmax_r", "step 2 lambda instead of lambda"),
    ("frpcag", "beta = 2.0 * gamma_c * lmax_c + 2.0 * gamma_r * lmax_r",
     "beta = 2.0 * gamma_r * lmax_c + 2.0 * gamma_c * lmax_r", "step with the norms swapped"),
    ("frpcag", "Z_next = S + ((t - 1.0) / t_next) * (S - S_prev)",
     "Z_next = S + ((t - 1.0) / t_next) * (S - Z)", "momentum on Z instead of S"),
    ("frpcag", "Z_next = S + ((t - 1.0) / t_next) * (S - S_prev)",
     "Z_next = S + (t / t_next) * (S - S_prev)", "momentum coefficient t/t' instead of (t-1)/t'"),
    ("frpcag", "t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0",
     "t_next = (1.0 + np.sqrt(1.0 + 4.0 * t)) / 2.0", "t update with t instead of t^2"),
    ("frpcag", "if np.sum((Z_next - Z) ** 2) < eps * np.sum(Z ** 2):",
     "if np.sum((Z_next - Z) ** 2) < eps * np.sum(Z_next ** 2):", "stop test against ||Z_{j+1}||"),
    ("frpcag", "if np.sum((Z_next - Z) ** 2) < eps * np.sum(Z ** 2):",
     "if np.sum((Z_next - Z) ** 2) <= eps * np.sum(Z ** 2):", "stop test not strict"),
    ("frpcag", "                return S, j", "                return S_prev, j", "early stop returns S_{j-1}"),
    ("frpcag", "    return S, J", "    return Z, J", "output Z_J instead of S_J"),
    ("frpcag", "S = prox_l1_centered(Z - lam * grad_smooth(Z,",
     "S = prox_l1_centered(Y - lam * grad_smooth(Z,", "gradient step taken from Y"),
    ("frpcag", "return float(gamma_c * np.sum(Z * ZLc) + gamma_r * np.sum(Z * LrZ))",
     "return float(np.sum(Z * ZLc) + gamma_r * np.sum(Z * LrZ))", "smooth term without gamma_c"),
    ("frpcag", "t[j + 1] = (1.0 + np.sqrt(1.0 + 4.0 * t[j] * t[j])) / 2.0",
     "t[j + 1] = (1.0 + np.sqrt(4.0 * t[j] * t[j])) / 2.0", "momentum sequence without the 1"),
    # alternate decoder (Section V.B)
    ("decoder", "return (np.outer(m_r, m_c) * X) + gr * (Lr @ X) + gc * (Lc @ X.T).T",
     "return X + gr * (Lr @ X) + gc * (Lc @ X.T).T", "operator without the sampling mask"),
    ("decoder", "return (np.outer(m_r, m_c) * X) + gr * (Lr @ X) + gc * (Lc @ X.T).T",
     "return (np.outer(m_r, m_c) * X) + gc * (Lr @ X) + gr * (Lc @ X.T).T", "operator with the gammas swapped"),
    ("decoder", "D = sp.diags(np.outer(m_r, m_c).ravel(order=\"F\"))",
     "D = sp.diags(np.outer(m_r, m_c).ravel(order=\"C\"))", "Kronecker mask in the wrong vec order"),
    ("decoder", "m_c[np.asarray(omega_c)] = 1.0", "m_c[:] = 1.0", "column mask all ones"),
    ("decoder", "            beta = rr_new / rr", "            beta = rr / rr_new", "CG beta inverted"),
    ("decoder", "            R -= alpha * Q", "            R += alpha * Q", "CG residual update sign"),
    ("decoder", "dgr = -float(np.sum(Lam * (Lr @ X)))", "dgr = float(np.sum(Lam * (Lr @ X)))",
     "gamma_r gradient sign"),
    ("decoder", "dgc = -float(np.sum(Lam * (Lc @ X.T).T))", "dgc = -float(np.sum(Lam * X))",
     "gamma_c gradient without L_c"),
    ("decoder", "Lam = solver(G, m_r, m_c, Lr, Lc, gr, gc)", "Lam = G",
     "backward without the adjoint solve"),
    # Algorithm 2 (Section V.C)
    ("approx", "    rhs = -(Lab @ R)", "    rhs = (Lab @ R)", "upsampling with the wrong sign"),
    ("approx", "k = int(np.count_nonzero((s >= ratio * s[0]) & (s > 0.0)))",
     "k = int(np.count_nonzero((s > ratio * s[0]) & (s > 0.0)))", "rank test > instead of >="),
    ("approx", "return float(np.sqrt(n * p / (rho_r * rho_c * (1.0 - delta))))",
     "return float(n * p / (rho_r * rho_c * (1.0 - delta)))", "scale without its square root"),
    ("approx", "return float(np.sqrt(n * p / (rho_r * rho_c * (1.0 - delta))))",
     "return float(np.sqrt(n * p / (rho_r * rho_c * (1.0 + delta))))", "delta with the wrong sign"),
    ("approx", "U = U / np.linalg.norm(U, axis=0, keepdims=True) if k else U",
     "U = U if k else U", "left vectors not normalised"),
    ("approx", "    U = _unit_columns(upsample(Lr, omega_r, Ut[:, :k]))",
     "    U = upsample(Lr, omega_r, Ut[:, :k])", "decoder 2 without normalisation"),
    ("approx", "    V = _unit_columns(upsample(Lc, omega_c, Vt[:, :k]))",
     "    V = upsample(Lc, omega_c, Vt[:, :k])", "decoder 3 without normalisation"),
    ("approx", "    V = _unit_columns(upsample(Lc, omega_c, Vt[:, :k]))",
     "    V = _unit_columns(upsample(Lc, omega_c, Vt[:, :max(k - 1, 1)]))", "decoder 3 one vector short"),
    # Algorithm 3 (Section VI)
    ("cluster", "new = np.argmin(D, axis=1)", "new = np.argmax(D, axis=1)", "k-means to the farthest centroid"),
    ("cluster", "C[j] = P[members].mean(axis=0)", "C[j] = P[members].sum(axis=0)", "centroid as a sum"),
    ("cluster", "        if it >= max_iter:", "        if it > max_iter:", "k-means cap off by one"),
    ("cluster", "return np.argmax(np.asarray(C), axis=1)", "return np.argmin(np.asarray(C), axis=1)",
     "min pooling"),
    # Kron reduction (Section IV-A)
    ("kron", "    return L_oo - L_or[:, keep] @ Xs", "    return L_oo + L_or[:, keep] @ Xs",
     "Schur complement with the wrong sign"),
    ("kron", "    rhs = B[keep].toarray()", "    rhs = B[keep].toarray() * 0.5", "half of the coupling"),
    ("kron", "    keep = np.flatnonzero(touches[lab])", "    keep = np.arange(rest.size)",
     "unsampled components without samples kept in the solve"),
    ("kron", "    L_oo = L[omega][:, omega].toarray()", "    L_oo = np.diag(L[omega][:, omega].diagonal())",
     "sampled-block off-diagonal dropped"),
    # K-NN graphs (Section II)
    ("knn", "order = np.lexsort((cand, d2[a, cand]))[:K]", "order = np.lexsort((-cand, d2[a, cand]))[:K]",
     "ties to the higher index"),
    ("knn", "d2[np.arange(q.size), q] = np.inf", "d2[np.arange(q.size), q] = d2[np.arange(q.size), q]",
     "a point its own neighbour"),
    ("knn", "return float(np.mean(np.sqrt(np.asarray(d2, dtype=np.float64))))",
     "return float(np.sqrt(np.mean(np.sqrt(np.asarray(d2, dtype=np.float64)))))",
     "sigma^2 = mean distance"),
    ("knn", "w = np.exp(-np.asarray(d2, dtype=np.float64).ravel() / (sigma * sigma))",
     "w = np.exp(-np.sqrt(np.asarray(d2, dtype=np.float64).ravel()) / (sigma * sigma))",
     "kernel of the distance instead of its square"),
    ("knn", "    r = np.concatenate([rows, idx.ravel()])\n    c = np.concatenate([idx.ravel(), rows])",
     "    r = np.concatenate([rows, rows])\n    c = np.concatenate([idx.ravel(), idx.ravel()])",
     "directed graph (no union)"),
    ("knn", "vals = -Wc.data / np.sqrt(deg[Wc.row] * deg[Wc.col])", "vals = -Wc.data / deg[Wc.row]",
     "random-walk instead of symmetric normalisation"),
]

PIN_MODULES = (test_oracle_pins, test_oracle_approx_pins, test_oracle_cluster_pins,
               test_oracle_knn_pins, test_oracle_kron_pins)


def _pin_cases():
    """Every pin of the three suites as (name, callable, kwargs), fastest first
    (two slow pins are run last)."""
    slow = ("test_backward_dense_jacobian_and_adjoint_identity",
            "test_fista_beck_teboulle_lyapunov_energy_is_nonincreasing")
    cases = []
    for mod in PIN_MODULES:
        for name, fn in vars(mod).items():
            if not name.startswith("test_") or not inspect.isfunction(fn):
                continue
            marks = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
            if not marks:
                cases.append((name, fn, {}))
                continue
            assert len(marks) == 1, name
            names = [a.strip() for a in marks[0].args[0].split(",")]
            for v in marks[0].args[1]:
                v = v if len(names) > 1 else (v,)
                cases.append((name, fn, dict(zip(names, v))))
    cases.sort(key=lambda c: c[0] in slow)
    return cases


def _mutated_module(modname, old, new):
    real = importlib.import_module(f"oracle.{modname}")
    path = real.__file__
    src = open(path).read()
    assert src.count(old) == 1, f"mutation anchor not unique in oracle/{modname}.py: {old!r}"
    mod = types.ModuleType(real.__name__)
    mod.__file__ = path
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new), path, "exec"), mod.__dict__)
    return real, mod


@pytest.mark.parametrize("modname,old,new,what", MUTANTS, ids=[m[3] for m in MUTANTS])
def test_every_planted_oracle_mistake_fails_a_pin(monkeypatch, modname, old, new, what):
    real, mut = _mutated_module(modname, old, new)
    for name, obj in vars(mut).items():
        if inspect.isfunction(obj) and obj.__module__ == real.__name__:
            monkeypatch.setattr(real, name, obj)
    caught = None
    for name, fn, kw in _pin_cases():
        try:
            fn(**kw)
        except Exception as e:  # an assertion, or the mutant breaking an invariant outright
            caught = f"{name}{kw or ''}: {type(e).__name__}"
            break
    assert caught is not None, f"no pin catches the planted mistake: {what}"


def test_unmutated_oracle_passes_every_pin_in_process():
    # the same in-process runner on the real oracle: no pin fails, so a
    # failure above comes from the planted mistake
    assert oracle.frpcag.fista.__module__ == "oracle.frpcag"
    for name, fn, kw in _pin_cases():
        fn(**kw)
