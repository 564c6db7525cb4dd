"""Compositions of oracle steps that several GPU tests compare against
(test infrastructure: calls only the oracle)."""
import oracle as O


def oracle_trace(par, ct, L, shape, rotkeys, rlk, pts):
    """The bootstrapping-shaped operation trace, step by step on the oracle:
    per linear-transform level one hoisted group of baby-step rotations, the
    plaintext inner sums, the giant-step rotations, their sum and a rescale;
    between the two transform halves a chain of squarings with rescales.
    Returns (ct, L)."""
    def lin(ct, L):
        baby, giant = shape["baby"], shape["giant"]
        rotated = O.hrot_hoisted(par, ct, L, baby, [rotkeys[r] for r in baby])
        acc = None
        for g, rg in enumerate(giant):
            inner = O.pmult_sum(par, rotated, pts[g * len(baby):(g + 1) * len(baby)], L)
            out = O.hrot(par, inner, L, rg, rotkeys[rg])
            acc = out if acc is None else O.ct_add(par, acc, out, L)
        return O.rescale(par, acc, L), L - 1

    for _ in range(shape["levels"]):
        ct, L = lin(ct, L)
    for _ in range(shape["chain"]):
        ct = O.rescale(par, O.hmult(par, ct, ct, L, rlk), L)
        L -= 1
    for _ in range(shape["levels"]):
        ct, L = lin(ct, L)
    return ct, L


def oracle_job(par, job, keys):
    """The oracle result of one job of the mixed batch (see ckks_inputs.batch_jobs)."""
    L = job["L"]
    if job["op"] == "HMULT":
        return O.hmult(par, job["in0"], job["in1"], L, keys[job["key"]])
    if job["op"] == "HROT":
        return O.hrot(par, job["in0"], L, job["rot"], keys[job["key"]])
    return O.rescale(par, job["in0"], L)
