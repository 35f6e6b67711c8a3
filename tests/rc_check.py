"""Near cutoff for the parity tests, taken from the oracle's own reading of the paper."""
from oracle import bem


def oracle_rc(ctx, V, T=None):
    """r_c from the oracle (bem.near_cutoff) for the mesh V, T (or a synth room as V); asserts
    that the library's default rule chose the same cutoff, so that the library's value is checked
    against an independent one rather than handed to the oracle."""
    if T is None:
        V, T = V.vertices, V.triangles
    rc = bem.near_cutoff(V, T)
    got = ctx.fmmbem_get_info().rc
    assert abs(got - rc) <= 1e-14 * rc, (got, rc)
    return rc
