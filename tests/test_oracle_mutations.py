"""The oracle's pins catch plausible mistakes (no GPU).

Each case plants one mistake in a private copy of the oracle, built from its
own source text with a single fragment replaced: a dropped term, a wrong sign
or index, a transposed operand, a missing step.  It then runs the pin tests
(the oracle checked against brute force, closed forms, the App. A toy model,
the rule of Eq. (eps), invariants and error bounds) against the copy and
requires at least one of them to fail.  The unaltered copy passes every pin,
so the failures come from the planted mistakes alone.  The package under
test itself is never modified.
"""
import os
import sys
import types

import pytest

import oracle as _real
import test_oracle_adjoint as _pins_adjoint
import test_oracle_pins as _pins
import test_oracle_ttm_grad as _pins_grad

_ROOT = os.path.dirname(os.path.abspath(_real.__file__))
_MODULES = ("tt", "ttm", "conventional", "adjoint", "ttm_grad")   # dependency order

# (case id, oracle module, fragment as written in the oracle, planted mistake)
MUTANTS = [
    # --- TT basics
    ("dense_transposed_carriage", "tt",
     "out = out @ core.reshape(core.shape[0], -1)",
     "out = out @ core.transpose(2, 1, 0).reshape(core.shape[2], -1)"),
    ("inner_wrong_axes", "tt",
     "env = np.tensordot(t, y, axes=([0, 1], [0, 1]))",
     "env = np.tensordot(t, y, axes=([0, 1], [2, 1]))"),
    ("inner3_drops_w", "tt",
     'env = np.einsum("bswx,bsy->wxy", t, b)',
     'env = np.einsum("bswx,bsy->wxy", np.abs(t), b)'),
    ("rank_rule_not_squared", "tt",
     "acc = acc + float(s[k]) * float(s[k])",
     "acc = acc + float(s[k])"),
    ("rank_rule_non_strict", "tt",
     "tails[k] < eps * total",
     "tails[k] <= eps * total"),
    ("rank_rule_tail_off_by_one", "tt",
     "return r, tails[r]",
     "return r, tails[r - 1]"),
    ("rank_rule_ignores_cap", "tt",
     "r = min(r, int(cap))",
     "r = r"),
    ("left_qr_transposed_r", "tt",
     "cores[i + 1] = np.tensordot(r, cores[i + 1], axes=(1, 0))",
     "cores[i + 1] = np.tensordot(r.T, cores[i + 1], axes=(1, 0))"),
    ("right_qr_untransposed_r", "tt",
     "cores[i - 1] = np.tensordot(cores[i - 1], r.T, axes=(2, 0))",
     "cores[i - 1] = np.tensordot(cores[i - 1], r, axes=(2, 0))"),
    ("round_drops_singular_values", "tt",
     "np.tensordot(cores[i - 1], u[:, :r] * s[:r], axes=(2, 0))",
     "np.tensordot(cores[i - 1], u[:, :r], axes=(2, 0))"),
    ("tt_sub_wrong_sign", "tt",
     "core = np.concatenate([c, -r], axis=2)",
     "core = np.concatenate([c, r], axis=2)"),
    # --- the TTM schedule of Sec. II.B
    ("contract_wrong_physical_index", "ttm",
     "out[:, eta, :] = a_core[:, eta, :] @ x_core[:, eta, :]",
     "out[:, eta, :] = a_core[:, eta, :] @ x_core[:, (eta + 1) % d, :]"),
    ("swap_legs_not_exchanged", "ttm",
     "mat = theta.transpose(0, 2, 1, 3).reshape(dl * dx, dp * dr)",
     "mat = theta.reshape(dl * dp, dx * dr)"),
    ("swap_drops_singular_values", "ttm",
     "x_new = (u[:, :r] * s[:r]).reshape(dl, dx, r)",
     "x_new = u[:, :r].reshape(dl, dx, r)"),
    ("swap_forced_discard_wrong", "ttm",
     "disc = float(np.sum(s[r:][::-1] ** 2)) if r < s.shape[0] else 0.0\n    return u, s, vt, r, disc",
     "disc = float(np.sum(s[r:][::-1])) if r < s.shape[0] else 0.0\n    return u, s, vt, r, disc"),
    ("chain_not_reversed", "ttm",
     "x = Bt[j]",
     "x = Bt[n - 1 - j]"),
    ("carriages_not_transposed", "ttm",
     "Bt = [np.ascontiguousarray(b.transpose(2, 1, 0)) for b in B]",
     "Bt = [np.ascontiguousarray(b[:, ::-1, :].transpose(2, 1, 0)) for b in B]"),
    ("gauge_moves_skipped", "ttm",
     "            _qr_move_right(Pi, p, res)",
     "            pass"),
    ("gauge_move_transposed_r", "ttm",
     "cores[p + 1] = np.tensordot(r, nxt, axes=(1, 0))",
     "cores[p + 1] = np.tensordot(r.T, nxt, axes=(1, 0))"),
    ("final_round_ignores_chi_out", "ttm",
     "r, disc = rank_rule(s, eps, chi_out)",
     "r, disc = rank_rule(s, eps, 0)"),
    ("final_round_drops_singular_values", "ttm",
     "np.tensordot(s[:r, None] * vt[:r], nxt, axes=(1, 0))",
     "np.tensordot(vt[:r], nxt, axes=(1, 0))"),
    ("swaps_capped_by_chi_out", "ttm",
     "swap(Pi[p], x, eps, chi_mid, take_forced())",
     "swap(Pi[p], x, eps, chi_out, take_forced())"),
    ("inputs_not_canonicalised", "ttm",
     "        A = left_orthogonalize(A)\n        B = left_orthogonalize(B)",
     "        A = [np.array(c) for c in A]\n        B = [np.array(c) for c in B]"),
    ("flops_merge_misses_a_leg", "ttm",
     "total += 2.0 * dl * dx * dm * dp * dr",
     "total += 2.0 * dl * dm * dp * dr"),
    ("flops_svd_without_back_transform", "ttm",
     "return 4.0 * m * n * n - (4.0 / 3.0) * n ** 3 + 4.0 * (m + n) * n * r",
     "return 4.0 * m * n * n - (4.0 / 3.0) * n ** 3"),
    ("flops_svd_sides_not_ordered", "ttm",
     "    if m < n:\n        m, n = n, m\n    return 4.0 * m",
     "    return 4.0 * m"),
    ("flops_wide_qr_as_tall", "ttm",
     "return 2.0 * n * m * m + (2.0 / 3.0) * m ** 3",
     "return 4.0 * m * n * n - (4.0 / 3.0) * n ** 3"),
    ("flops_gauge_move_product_not_recorded", "ttm",
     "    res.ops.append((\"gemm\", k, rr, nxt.shape[1] * nxt.shape[2]))\n    res.n_qr += 1",
     "    res.n_qr += 1"),
    ("centre_right_lq_drops_l", "ttm",
     "    x_new = x_new @ rf.T\n",
     "    x_new = x_new\n"),
    ("centre_right_lq_not_transposed", "ttm",
     "    p_new = q.T\n",
     "    p_new = q.T[:, ::-1]\n"),
    ("move_smaller_moves_the_larger", "ttm",
     "if max(c.shape[0] for c in A) < max(c.shape[0] for c in B):",
     "if max(c.shape[0] for c in A) > max(c.shape[0] for c in B):"),
    ("discards_not_recorded", "ttm",
     "            res.discards.append(disc)\n            res.n_swap += 1",
     "            res.discards.append(0.0)\n            res.n_swap += 1"),
    # --- the conventional product of Sec. II.A
    ("kron_wrong_physical_index", "conventional",
     "core[:, s, :] = np.kron(a[:, s, :], b[:, s, :])",
     "core[:, s, :] = np.kron(a[:, s, :], b[:, (s + 1) % d, :])"),
    ("local_core_wrong_order", "conventional",
     'np.einsum("casy,asx->csxy", t1, a)',
     'np.einsum("casy,asx->csyx", t1, a)'),
    ("right_env_reversed_physical_index", "conventional",
     'np.einsum("bsy,csay->cab", b, u2)',
     'np.einsum("bsy,csay->cab", b, u2[:, ::-1])'),
    ("splitmix_wrong_shift", "conventional",
     "z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK",
     "z = ((z ^ (z >> 28)) * 0x94D049BB133111EB) & _MASK"),
    # --- the gradient of <W, A*B>
    ("left_env_drops_terms", "adjoint",
     "nxt += np.tensordot(t, b[:, s, :], axes=(0, 0))",
     "nxt = np.tensordot(t, b[:, s, :], axes=(0, 0))"),
    ("right_env_wrong_physical_index", "adjoint",
     "t = np.tensordot(w[:, s, :], F, axes=(1, 0))",
     "t = np.tensordot(w[:, (s + 1) % w.shape[1], :], F, axes=(1, 0))"),
    ("grad_a_contracts_wrong_bond", "adjoint",
     "ga[:, s, :] = np.tensordot(ua, Fr, axes=([1, 2], [0, 2]))",
     "ga[:, s, :] = np.tensordot(ua, Fr, axes=([1, 2], [0, 1]))"),
    # --- reverse mode through the TTM product
    ("vjp_qr_mirrors_wrong_triangle", "ttm_grad",
     "X = np.tril(X) + np.tril(X, -1).T",
     "X = np.triu(X) + np.triu(X, 1).T"),
    ("vjp_svd_drops_direct_term", "ttm_grad",
     "    matbar = Zbar @ Vr.T\n",
     "    matbar = 0.0 * Zbar @ Vr.T\n"),
    ("vjp_svd_wrong_gap_sign", "ttm_grad",
     "F = 1.0 / (lam[None, :r] - lam[r:, None])",
     "F = 1.0 / (lam[r:, None] - lam[None, :r])"),
    ("vjp_svd_drops_null_space", "ttm_grad",
     "        Gbar = Gbar + (Nbar / lam[None, :r]) @ Vr.T",
     "        Gbar = Gbar"),
    ("vjp_merge_legs_not_exchanged", "ttm_grad",
     "tb = matbar.reshape(dl, dx, dp, dr).transpose(0, 2, 1, 3)",
     "tb = matbar.reshape(dl, dp, dx, dr)"),
    ("vjp_round_next_core_transposed", "ttm_grad",
     "            Pib[i + 1] = np.tensordot(Zt, nb, axes=(0, 0))",
     "            Pib[i + 1] = np.tensordot(Zt[::-1], nb, axes=(0, 0))"),
    ("grad_b_uses_wrong_factor", "adjoint",
     "ub = np.tensordot(t, a[:, s, :], axes=(0, 0))",
     "ub = np.tensordot(t, 2.0 * a[:, s, :], axes=(0, 0))"),
]

_counter = [0]


def _build(mutant=None):
    """A private copy of the oracle package, with one fragment replaced."""
    _counter[0] += 1
    name = "_oracle_copy_%d" % _counter[0]
    pkg = types.ModuleType(name)
    pkg.__path__ = []
    sys.modules[name] = pkg
    try:
        for mod in _MODULES:
            src = open(os.path.join(_ROOT, mod + ".py")).read()
            if mutant is not None and mutant[1] == mod:
                _, _, old, new = mutant
                assert src.count(old) == 1, "fragment not found once in oracle/%s.py: %r" % (mod, old)
                src = src.replace(old, new)
            m = types.ModuleType(name + "." + mod)
            m.__package__ = name
            m.__file__ = os.path.join(_ROOT, mod + ".py")
            sys.modules[m.__name__] = m
            exec(compile(src, m.__file__, "exec"), m.__dict__)
            setattr(pkg, mod, m)
        init = open(os.path.join(_ROOT, "__init__.py")).read()
        pkg.__package__ = name
        exec(compile(init, os.path.join(_ROOT, "__init__.py"), "exec"), pkg.__dict__)
    except BaseException:
        _drop(name)
        raise
    return pkg


def _drop(name):
    for key in [k for k in sys.modules if k == name or k.startswith(name + ".")]:
        del sys.modules[key]


def _pin_calls():
    """Every pin of the oracle as (label, zero-argument call)."""
    calls = []
    for mod in (_pins, _pins_adjoint, _pins_grad):
        for attr in sorted(vars(mod)):
            fn = getattr(mod, attr)
            if not (attr.startswith("test_") and callable(fn)):
                continue
            params = [m for m in getattr(fn, "pytestmark", []) if m.name == "parametrize"]
            if params:
                argname, values = params[0].args[0], params[0].args[1]
                names = [a.strip() for a in argname.split(",")]
                for v in values:
                    kw = dict(zip(names, v)) if len(names) > 1 else {names[0]: v}
                    calls.append(("%s[%s]" % (attr, v), lambda f=fn, kw=kw: f(**kw)))
            else:
                calls.append((attr, fn))
    return calls


def _run_pins(pkg, stop_at_first):
    """Run the pins with ``O`` bound to ``pkg``; return the labels that fail."""
    failed = []
    saved = (_pins.O, _pins_adjoint.O, _pins_grad.O)
    _pins.O = _pins_adjoint.O = _pins_grad.O = pkg
    try:
        for label, call in _pin_calls():
            try:
                call()
            except pytest.skip.Exception:
                continue
            except Exception:   # a wrong value, a wrong shape or a LAPACK error
                failed.append(label)
                if stop_at_first:
                    break
    finally:
        _pins.O, _pins_adjoint.O, _pins_grad.O = saved
    return failed


def test_unaltered_copy_passes_every_pin():
    pkg = _build()
    try:
        assert _run_pins(pkg, stop_at_first=False) == []
    finally:
        _drop(pkg.__name__)


@pytest.mark.parametrize("mutant", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(mutant):
    pkg = _build(mutant)
    try:
        failed = _run_pins(pkg, stop_at_first=True)
    finally:
        _drop(pkg.__name__)
    assert failed, "no pin catches the planted mistake %s" % mutant[0]
