"""Plant known mistakes in a copy of the oracle and check that the CPU pins
catch every one.

Runs on the CPU only: each entry replaces one expression of oracle/ in a
temporary copy of the repository and runs `pytest -m "not gpu"` there; a
mistake that no pin catches is reported as MISSED.  (Transposing grad v in
the tiring term is no mistake: the Eddington tensor is symmetric, so
P : grad v = P : grad v^T; it is not listed.)  Usage:
    python tests/plant_mistakes.py
"""
import os, shutil, subprocess, sys
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
M = [
 ("fldref.py", "return 0.5 * (Dl + Dr)", "return np.maximum(Dl, Dr)", "arith mean -> max"),
 ("fldref.py", "return 0.5 * (Dl + Dr)", "return np.sqrt(Dl * Dr)", "arith mean -> geometric"),
 ("fldref.py", "return 2.0 * Dl * Dr / (Dl + Dr)", "return Dl * Dr / (Dl + Dr)", "harmonic mean without its 2"),
 ("fldref.py", "return 2.0 * Dl * Dr / (Dl + Dr)", "return 0.5 * (Dl + Dr)", "harmonic -> arith"),
 ("fldref.py", "return (prob.gamma - 1.0) * e / (rho * prob.gas_const)", "return e / (rho * prob.gas_const)", "T without (gamma-1)"),
 ("fldref.py", "return (prob.gamma - 1.0) * e / (rho * prob.gas_const)", "return (prob.gamma - 1.0) * e / prob.gas_const", "T without rho"),
 ("fldref.py", "np.clip(k0 * rho ** a * T ** b, kmin, kmax)", "np.clip(k0 * rho ** a * T ** (b + 0.5), kmin, kmax)", "Kramers exponent -3 for -3.5"),
 ("fldref.py", "np.clip(k0 * rho ** a * T ** b, kmin, kmax)", "k0 * rho ** a * T ** b", "opacity without clip"),
 ("fldref.py", "np.clip(k0 * rho ** a * T ** b, kmin, kmax)", "np.clip(k0 * T ** b, kmin, kmax)", "opacity without rho"),
 ("fldref.py", "G = (shifted(-2) - 8.0 * shifted(-1) + 8.0 * shifted(1)", "G = (shifted(-2) + 8.0 * shifted(-1) - 8.0 * shifted(1)", "gradient sign"),
 ("fldref.py", "- shifted(2)) / (12.0 * prob.dx[d])", "- shifted(2)) / (6.0 * prob.dx[d])", "gradient 6 for 12"),
 ("fldref.py", "return (2.0 + R) / (6.0 + 3.0 * R + R * R)", "return (2.0 + R) / (6.0 + 3.0 * R)", "limiter denominator"),
 ("fldref.py", "R = gmag / (rho * kappa * E)", "R = gmag / (rho * kappa)", "R without E"),
 ("fldref.py", "D = prob.c * lam / (rho * kappa)", "D = lam / (rho * kappa)", "D without c"),
 ("fldref.py", "a = dt * _face_mean(D, Dr, prob.face_mean) / (prob.dx[d] ** 2)", "a = dt * _face_mean(D, Dr, prob.face_mean) / prob.dx[d]", "alpha with dx not dx^2"),
 ("fldref.py", "a = dt * _face_mean(D, Dr, prob.face_mean) / (prob.dx[d] ** 2)", "a = dt * _face_mean(D, Dr, prob.face_mean) / (prob.dx[prob.ndim - 1 - d] ** 2)", "alpha with the other axis' dx"),
 ("fldref.py", "            a[tuple(sl)] = 0.0", "            pass", "wall face not zeroed"),
 ("fldref.py", "mode = \"wrap\" if prob.bc[d] == PERIODIC else \"symmetric\"", "mode = \"wrap\" if prob.bc[d] == PERIODIC else \"reflect\"", "Neumann ghosts without the edge repeat"),
 ("fldref.py", "mode = \"wrap\" if prob.bc[d] == PERIODIC else \"symmetric\"", "mode = \"wrap\" if prob.bc[d] == PERIODIC else \"edge\"", "Neumann ghosts by edge copy"),
 ("fldref.py", "        Ax += flux\n", "        Ax -= flux\n", "flux sign"),
 ("fldref.py", "        Ax -= np.roll(flux, 1, axis=ax)", "        Ax -= np.roll(flux, -1, axis=ax)", "flux roll direction"),
 ("fldref.py", "vals += [a, a, -a, -a]", "vals += [a, a, -a, -0.5 * a]", "matrix asymmetric"),
 ("fldref.py", "beta = dt * prob.c * kappa * rho", "beta = dt * kappa * rho", "beta without c"),
 ("fldref.py", "a4 = beta * prob.a_rad * ((prob.gamma - 1.0) / (rho * prob.gas_const)) ** 4", "a4 = beta * prob.a_rad * (1.0 / (rho * prob.gas_const)) ** 4", "a4 without gamma-1"),
 ("fldref.py", "a4 = beta * prob.a_rad * ((prob.gamma - 1.0) / (rho * prob.gas_const)) ** 4", "a4 = beta * ((prob.gamma - 1.0) / (rho * prob.gas_const)) ** 4", "a4 without a_R"),
 ("fldref.py", "S = E_star + e\n", "S = E_star\n", "S without e"),
 ("fldref.py", "x = quartic_root(a4, 1.0 + beta, e + beta * S)", "x = quartic_root(a4, beta, e + beta * S)", "quartic linear coefficient without 1"),
 ("fldref.py", "return S - x, x", "return S - x, S - x", "exchange returns wrong e"),
 ("fldref.py", "low = 2.0 / (3.0 + np.sqrt(9.0 + 12.0 * R * R))", "low = 2.0 / (3.0 + np.sqrt(9.0 + 6.0 * R * R))", "Minerbo low branch 6 R^2"),
 ("fldref.py", "high = 1.0 / (1.0 + R + np.sqrt(1.0 + 2.0 * R))", "high = 1.0 / (1.0 + R + np.sqrt(1.0 + R))", "Minerbo high branch sqrt(1 + R)"),
 ("fldref.py", "return np.where(R <= 1.5, low, high)", "return np.where(R <= 1.0, low, high)", "Minerbo switch at R = 1"),
 ("fldref.py", "return lam + lam * lam * R * R", "return lam + lam * R * R", "Eddington factor lambda R^2"),
 ("explicit.py", "fr = [-lam * g for g in G]", "fr = [lam * g for g in G]", "radiation force sign"),
 ("explicit.py", "work = sum(v[d] * fr[d] for d in range(nd))", "work = sum(v[0] * fr[d] for d in range(nd))", "work with v_x only"),
 ("explicit.py", "t_ij = 0.5 * (3.0 * f - 1.0) * n[i] * n[j]", "t_ij = 0.5 * (3.0 * f - 1.0) * n[i] * n[i]", "Eddington tensor n_i n_i"),
 ("explicit.py", "                t_ij = t_ij + 0.5 * (1.0 - f)", "                t_ij = t_ij + (1.0 - f)", "Eddington tensor isotropic part without 1/2"),
 ("explicit.py", "tiring = tiring + t_ij * grads[j][i]", "tiring = tiring + t_ij * grads[j][j]", "tiring with d_j v_j in every entry"),
 ("explicit.py", "tiring = E * tiring", "tiring = tiring", "tiring without E"),
 ("unet_ref.py", "mh = m[k] / (1 - b1 ** t)", "mh = m[k]", "Adam without first-moment bias correction"),
 ("unet_ref.py", "vh = v[k] / (1 - b2 ** t)", "vh = v[k]", "Adam without second-moment bias correction"),
 ("unet_ref.py", "p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)", "p[k] = p[k] - lr * mh / np.sqrt(vh + eps)", "Adam eps inside sqrt"),
 ("unet_ref.py", "v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]", "v[k] = b2 * v[k] + (1 - b2) * np.abs(g[k])", "Adam v with |g|"),
 ("unet_ref.py", "f0 = lE - lE.mean()", "f0 = lE", "features: no mean removal"),
 ("unet_ref.py", "f1 = np.log(rhokappa_dx) / 4.0", "f1 = np.log(rhokappa_dx)", "features: f1 unscaled"),
 ("unet_ref.py", "f2 = np.log1p(alpha_x) / 4.0", "f2 = np.log(alpha_x + 1e-30) / 4.0", "features: log for log1p"),
 ("unet_ref.py", "return np.stack([f0, f1, f2, f3], axis=-1)[None]", "return np.stack([f0, f1, f3, f2], axis=-1)[None]", "features: x/y swapped"),
 ("fldref.py", "aw = 2.0 * dt * D[sl] / (prob.dx[d] ** 2)", "aw = dt * D[sl] / (prob.dx[d] ** 2)", "Dirichlet wall face a full cell away"),
 ("fldref.py", "rhs[sl] += aw * Ew", "rhs[sl] += aw", "Dirichlet rhs without E_w"),
 ("fldref.py", "Ep[tuple(sl)] = 2.0 * Ew - Ep[tuple(sl)]", "Ep[tuple(sl)] = Ew", "Dirichlet ghosts set to E_w"),
 ("fldref.py", "Ep[tuple(sl)] = 2.0 * Ew - Ep[tuple(sl)]", "pass", "Dirichlet ghosts mirrored"),
 ("fldref.py", "    return solve(alphas, E + rhs, prob, diag=diag, **kw)", "    return solve(alphas, E + rhs, prob, **kw)", "Dirichlet diagonal dropped"),
 ("fldref.py", "b = np.where(held, E_hold, E + rhs).ravel()", "b = np.where(held, E, E + rhs).ravel()", "held cells keep E^n"),
 ("fldref.py", "b = np.where(held, E_hold, E + rhs).ravel()", "b = np.where(held, E_hold, E).ravel()", "held step without the Dirichlet walls' rhs"),
 ("fldref.py", "A = (free_rows @ A + sp.diags(h.astype(np.float64))).tocsr()", "A = A.tocsr()", "held rows not replaced"),
 ("fldref.py", "A = (free_rows @ A + sp.diags(h.astype(np.float64))).tocsr()", "A = (free_rows @ A @ free_rows + sp.diags(h.astype(np.float64))).tocsr()", "free cells decoupled from the held values"),
 ("amr.py", "beta = (2.0 / 3.0) * dt * _mean(\n                            Df[J, I]", "beta = dt * _mean(\n                            Df[J, I]", "coarse-fine flux over one fine spacing"),
 ("amr.py", "beta = (2.0 / 3.0) * dt * _mean(\n                                D[l][J, I]", "beta = dt * _mean(\n                                D[l][J, I]", "hierarchy: coarse-fine flux over one fine spacing"),
 ("amr.py", "couple(me, c, beta, beta / 4.0)", "couple(me, c, beta, beta / 2.0)", "hierarchy: coarser side of an edge at 1/2"),
 ("amr.py", "child_mean(avg[l + 1])", "vals[l]", "hierarchy: covered cells keep their own values"),
 ("amr.py", "view.append(np.where(present[l], avg[l], inject(view[l - 1])))", "view.append(np.where(present[l], avg[l], inject(avg[l - 1]) * 0 + 1.0))", "hierarchy: outside a level's blocks a constant view"),
 ("amr.py", "couple(fidx[J, I], bidx[cb], beta, beta / 4.0)", "couple(fidx[J, I], bidx[cb], beta, beta / 2.0)", "base side of a block edge at 1/2"),
 ("amr.py", "cb = (JJ // 2, II // 2)", "cb = ((JJ // 2) % grid.ny, (I // 2) % grid.nx)", "coarse neighbour taken along the wrong axis"),
 ("amr.py", "base_view = np.where(ref, child_mean(fine_full), base)", "base_view = base", "covered base cells keep their own values"),
]
import tempfile
tmp = os.path.join(tempfile.gettempdir(), "fld_oracle_mutant")
res = []
for fname, old, new, label in M:
    if os.path.exists(tmp):
        shutil.rmtree(tmp)
    shutil.copytree(ROOT, tmp, ignore=shutil.ignore_patterns(".git", "_build", "_work", "gpurun_out", "__pycache__", "*.so"))
    p = os.path.join(tmp, "oracle", fname)
    s = open(p).read()
    assert s.count(old) == 1, (label, s.count(old))
    open(p, "w").write(s.replace(old, new))
    r = subprocess.run([sys.executable, "-m", "pytest", "tests", "-m", "not gpu", "-x", "-q", "-p", "no:cacheprovider",
                        "--deselect", "tests/test_abi.py"], cwd=tmp, capture_output=True, text=True)
    failed = [l for l in r.stdout.splitlines() if l.startswith("FAILED")]
    caught = r.returncode != 0
    res.append((label, caught, failed[0] if failed else r.stdout.splitlines()[-1]))
    print(("CAUGHT " if caught else "MISSED ") + label + " :: " + (failed[0][7:90] if failed else r.stdout.splitlines()[-1]), flush=True)
print(sum(c for _, c, _ in res), "of", len(res), "caught")
