"""Plausible mistakes planted in a copy of the oracle, one at a time, on the
CPU: a flipped sign, a dropped term, a transposed or shifted index, a wrong
normalisation.  Each one must make at least one pin of the oracle fail
(tests/test_oracle_mutants.py runs the pins against every mutant).

The oracle's own files are never changed: a C mutant is a patched copy of
oracle.c compiled into a temporary library that the oracle module is pointed
at; a Python mutant is a patched copy of the oracle module whose functions
replace the module's for that test session only.
"""
import atexit
import os
import shutil
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_DIR = os.path.join(os.path.dirname(HERE), "oracle")

# name: (file, text in the oracle, replacement)
MUTANTS = {
    # hopping term (eq. 4)
    "hop_projector_sign": ("c", "double sg = (dir == 0) ? -1.0 : 1.0;", "double sg = (dir == 0) ? 1.0 : -1.0;"),
    "hop_backward_link_not_daggered": ("c", "m3_dag(link(U, V, mu, m), u);", "memcpy(u, link(U, V, mu, m), sizeof(u));"),
    "hop_backward_link_at_n": ("c", "m3_dag(link(U, V, mu, m), u);", "m3_dag(link(U, V, mu, n), u);"),
    "hop_kappa_sign": ("c", "t[i] = s - kappa * h[i];", "t[i] = s + kappa * h[i];"),
    "site_index_x_y_swapped": ("c", "return c[0] + (long)L[0] * (c[1] + (long)L[1] * (c[2] + (long)L[2] * c[3]));",
                               "return c[1] + (long)L[1] * (c[0] + (long)L[0] * (c[2] + (long)L[2] * c[3]));"),
    # gamma matrices
    "gamma_y_sign": ("c", "if (k == 1) { s[0][1] = -I; s[1][0] = I; }", "if (k == 1) { s[0][1] = I; s[1][0] = -I; }"),
    # clover term
    "clover_quarter_not_eighth": ("c", "Fh[k] = (Q[k] - Qd[k]) / 8.0;", "Fh[k] = (Q[k] - Qd[k]) / 4.0;"),
    "clover_sign": ("c", "-= kappa * csw * gg[al][be] * Fh[3 * a + b];", "+= kappa * csw * gg[al][be] * Fh[3 * a + b];"),
    "clover_colour_transposed": ("c", "-= kappa * csw * gg[al][be] * Fh[3 * a + b];",
                                 "-= kappa * csw * gg[al][be] * Fh[3 * b + a];"),
    "clover_fourth_leaf_dropped": ("c", "m3_dag(link(U, V, mu, n), a);    m3_mul(t, a, t);\n"
                                        "    for (int k = 0; k < 9; k++) Q[k] += t[k];\n}",
                                   "m3_dag(link(U, V, mu, n), a);    m3_mul(t, a, t);\n}"),
    "clover_first_leaf_clockwise": ("c", "m3_dag(link(U, V, mu, n_pn), a); m3_mul(t, a, t);",
                                    "m3_mul(t, link(U, V, mu, n_pn), t);"),
    "clover_trace_subtracted": ("c", "for (int k = 0; k < 9; k++) Fh[k] = (Q[k] - Qd[k]) / 8.0;",
                                "for (int k = 0; k < 9; k++) Fh[k] = (Q[k] - Qd[k]) / 8.0;\n"
                                "            { cplx tr = (Fh[0] + Fh[4] + Fh[8]) / 3.0; Fh[0] -= tr; Fh[4] -= tr; Fh[8] -= tr; }"),
    "site_invert_elimination_sign": ("c", "for (int j = 0; j < 24; j++) a[r][j] -= f * a[col][j];",
                                     "for (int j = 0; j < 24; j++) a[r][j] += f * a[col][j];"),
    # inner product of the solver
    "vdot_not_conjugated": ("c", "cplx p = conj(a[i]) * b[i];", "cplx p = a[i] * b[i];"),
    # BiCGStab steps (readings of Algs. 1 and 2 shared by the oracle's solver)
    "bicgstab_beta_inverted": ("c", "cplx beta = (rho1 / rho) * (alpha / omega);",
                               "cplx beta = (rho1 / rho) / (alpha / omega);"),
    "bicgstab_alpha_without_rho": ("c", "alpha = rho1 / den;", "alpha = den;"),
    # link gradient
    "grad_hopping_sign": ("c", "Gl[3 * a + b] += kappa * s;", "Gl[3 * a + b] -= kappa * s;"),
    "grad_second_outer_product_dropped": ("c", " + z[3 * al + a] * conj(lam[mp * 12 + 3 * al + b]);", ";"),
    "grad_clover_quarter": ("c", "const double fac = kappa * csw / 8.0;", "const double fac = kappa * csw / 4.0;"),
    "grad_clover_hermitian_part": ("c", "N[3 * a + b] = M[3 * a + b] - conj(M[3 * b + a]);",
                                   "N[3 * a + b] = M[3 * a + b] + conj(M[3 * b + a]);"),
    # even-odd pieces (eqs. 6-9) and the Fourier solve
    "dhat_literal_eo_eo": ("py", "htilde(U, Finv, htilde(U, Finv, xe, 1), 0)", "htilde(U, Finv, htilde(U, Finv, xe, 0), 0)"),
    "bhat_sign": ("py", "restrict(fb, 0) + kappa * htilde", "restrict(fb, 0) - kappa * htilde"),
    "x_o_sign": ("py", "restrict(site_apply(Finv, b), 1) + kappa * htilde", "restrict(site_apply(Finv, b), 1) - kappa * htilde"),
    "parity_without_t": ("py", "return (x + y + z + t) & 1", "return (x + y + z) & 1"),
    "free_momentum_sin_sign": ("py", "- 2j * np.sin(p[mu])", "+ 2j * np.sin(p[mu])"),
    "dhat_sites_kappa_not_squared": ("c", "out[s * 12 + i] = xe[n * 12 + i] - kappa * kappa * a;",
                                     "out[s * 12 + i] = xe[n * 12 + i] - kappa * a;"),
    "htilde_sites_without_clover_inverse": ("c", "for (int j = 0; j < 12; j++) a += Fi[12 * i + j] * h[j];\n"
                                                 "            out[s * 12 + i] = a;",
                                            "a = h[i];\n            out[s * 12 + i] = a;"),
    "clover_sites_inverse_ignored": ("c", "        if (inverse) {\n            if (!invert12(F, Fi))",
                                     "        if (0) {\n            if (!invert12(F, Fi))"),
    # true residual of the full system
    "residual_zero": ("c", "r += creal(d) * creal(d) + cimag(d) * cimag(d);", "r += 0.0 * creal(d);"),
    "residual_drops_imag": ("c", "r += creal(d) * creal(d) + cimag(d) * cimag(d);", "r += creal(d) * creal(d);"),
    # storage format
    # more gamma matrices, hops, solver updates and the residual
    "gamma_x_sign": ("c", "if (k == 0) { s[0][1] = 1; s[1][0] = 1; }", "if (k == 0) { s[0][1] = -1; s[1][0] = -1; }"),
    "gamma_z_sign": ("c", "if (k == 2) { s[0][0] = 1; s[1][1] = -1; }", "if (k == 2) { s[0][0] = -1; s[1][1] = 1; }"),
    "gamma_t_sign": ("c", "g[0][0] = 1; g[1][1] = 1; g[2][2] = -1; g[3][3] = -1;",
                     "g[0][0] = -1; g[1][1] = -1; g[2][2] = 1; g[3][3] = 1;"),
    "gamma_spatial_i_swapped": ("c", "g[i][2 + j] = -I * s[i][j];\n                g[2 + i][j] = I * s[i][j];",
                                "g[i][2 + j] = I * s[i][j];\n                g[2 + i][j] = -I * s[i][j];"),
    "hop_forward_link_daggered": ("c", "memcpy(u, link(U, V, mu, n), sizeof(u));              /* U_mu(n)            */",
                                  "m3_dag(link(U, V, mu, n), u);"),
    "hop_directions_swapped": ("c", "long m = shifted(L, c, mu, dir == 0 ? +1 : -1);",
                               "long m = shifted(L, c, mu, dir == 0 ? -1 : +1);"),
    "bicgstab_x_update_drops_omega_s": ("c", "x[i] += alpha * p[i] + omega * s[i]; r[i] = s[i] - omega * t[i];",
                                        "x[i] += alpha * p[i]; r[i] = s[i] - omega * t[i];"),
    "residual_sign_of_D_x": ("c", "cplx d = b[n * 12 + i] - (a - kappa * h[i]);", "cplx d = b[n * 12 + i] + (a - kappa * h[i]);"),
    "residual_hop_sign": ("c", "cplx d = b[n * 12 + i] - (a - kappa * h[i]);", "cplx d = b[n * 12 + i] - (a + kappa * h[i]);"),
    "fp16_scale_per_spin": ("py", "sites = re.reshape(re.shape[:-3] + (24,))", "sites = re.reshape(re.shape[:-2] + (6,))"),
    "fp16_decode_without_scale": ("py", "dec = (h.astype(np.float32) * s).astype(np.float32).reshape(re.shape)",
                                  "dec = h.astype(np.float32).reshape(re.shape)"),
    "fp16_scale_from_sum": ("py", "s = np.abs(sites).max(axis=-1, keepdims=True).astype(np.float32)",
                            "s = np.abs(sites).sum(axis=-1, keepdims=True).astype(np.float32)"),
    "fp32_storage_not_rounded": ("py", "return np.asarray(psi, dtype=np.complex128).astype(np.complex64).astype(np.complex128)",
                                 "return np.asarray(psi, dtype=np.complex128).astype(np.complex128)"),
}


def patched(kind: str, find: str, repl: str) -> str:
    path = os.path.join(ORACLE_DIR, "oracle.c" if kind == "c" else "__init__.py")
    with open(path) as f:
        src = f.read()
    n = src.count(find)
    if n != 1:
        raise ValueError("mutation site found %d times in %s: %r" % (n, path, find))
    return src.replace(find, repl)


def install(name: str) -> None:
    """Point the already imported oracle module at the named mutant."""
    import oracle
    kind, find, repl = MUTANTS[name]
    src = patched(kind, find, repl)
    if kind == "c":
        d = tempfile.mkdtemp(prefix="oracle_mutant_")
        atexit.register(shutil.rmtree, d, True)
        c = os.path.join(d, "oracle.c")
        with open(c, "w") as f:
            f.write(src)
        oracle._SRC = c
        oracle._LIB = os.path.join(d, "liboracle.so")
        oracle._lib = None
        oracle.build(force=True)
    else:
        ns = {"__name__": "oracle_mutant", "__file__": os.path.join(ORACLE_DIR, "__init__.py")}
        exec(compile(src, "oracle_mutant(%s)" % name, "exec"), ns)
        for k, v in ns.items():
            if callable(v) and not k.startswith("__") and getattr(v, "__module__", None) == "oracle_mutant":
                setattr(oracle, k, v)
