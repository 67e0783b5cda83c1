"""The FT-CCSD kernels E, S1 and S2 as lists of terms (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each entry restates one printed term of Appendix A (eqn:E, eqn:ccS1,
eqn:ccS2) in the paper's order and index letters:

    (coefficient, antisymmetriser, [factor, ...])

factor "F:pq"   thermal one-body integral f_pq
       "V:pqrs" thermal antisymmetrised integral <pq||rs>
       "s1:ia"  amplitude s_i^a        (stored as s1[i, a])
       "s2:ijab" amplitude s_ij^ab     (stored as s2[i, j, a, b])

The antisymmetriser acts on the output: "" none, "ij" = P(ij), "ab" = P(ab),
"ijab" = P(ij)P(ab), with P(pq) X = X - X(p<->q).  Letters i..n are hole
slots (weight sqrt(n_p)), letters a..f particle slots (weight sqrt(1-n_p)).
Every term holds exactly one integral factor, so each kernel is linear in the
thermal integrals.

Reading of the printed text (documented in the design notes):
  * the last term of eqn:ccS1 is printed with the summation label "jkcd" over
    <jk||bc> s_i^b s_j^c s_k^a; the summed letters are j, k, b, c.
"""

HOLE = "ijklmn"
PART = "abcdef"

# E(tau), eqn:E
E_TERMS = [
    (1.0, "", ["F:ia", "s1:ia"]),
    (0.25, "", ["V:ijab", "s2:ijab"]),
    (0.5, "", ["V:ijab", "s1:ia", "s1:jb"]),
]

# S_i^a(tau), eqn:ccS1
S1_TERMS = [
    (1.0, "", ["F:ai"]),
    (1.0, "", ["F:ab", "s1:ib"]),
    (-1.0, "", ["F:ji", "s1:ja"]),
    (1.0, "", ["V:jabi", "s1:jb"]),
    (1.0, "", ["F:jb", "s2:ijab"]),
    (0.5, "", ["V:ajbc", "s2:ijbc"]),
    (-0.5, "", ["V:jkib", "s2:jkab"]),
    (-1.0, "", ["F:jb", "s1:ib", "s1:ja"]),
    (1.0, "", ["V:jabc", "s1:jb", "s1:ic"]),
    (-1.0, "", ["V:jkbi", "s1:jb", "s1:ka"]),
    (-0.5, "", ["V:jkbc", "s1:ib", "s2:jkac"]),
    (-0.5, "", ["V:jkbc", "s1:ja", "s2:ikbc"]),
    (1.0, "", ["V:jkbc", "s1:jb", "s2:kica"]),
    (1.0, "", ["V:jkbc", "s1:ib", "s1:jc", "s1:ka"]),
]

# S_ij^ab(tau), eqn:ccS2
S2_TERMS = [
    (1.0, "", ["V:abij"]),
    (1.0, "ij", ["V:abcj", "s1:ic"]),
    (-1.0, "ab", ["V:kbij", "s1:ka"]),
    (1.0, "ab", ["F:bc", "s2:ijac"]),
    (-1.0, "ij", ["F:kj", "s2:ikab"]),
    (0.5, "", ["V:abcd", "s2:ijcd"]),
    (0.5, "", ["V:klij", "s2:klab"]),
    (1.0, "ijab", ["V:kbcj", "s2:ikac"]),
    (0.5, "ij", ["V:abcd", "s1:ic", "s1:jd"]),
    (0.5, "ab", ["V:klij", "s1:ka", "s1:lb"]),
    (-1.0, "ijab", ["V:akcj", "s1:ic", "s1:kb"]),
    (-1.0, "ij", ["F:kc", "s1:ic", "s2:kjab"]),
    (-1.0, "ab", ["F:kc", "s1:ka", "s2:ijcb"]),
    (1.0, "ab", ["V:kacd", "s1:kc", "s2:ijdb"]),
    (-1.0, "ij", ["V:klci", "s1:kc", "s2:ljab"]),
    (1.0, "ijab", ["V:akcd", "s1:ic", "s2:kjdb"]),
    (-1.0, "ijab", ["V:klic", "s1:ka", "s2:ljcb"]),
    (0.5, "ij", ["V:klcj", "s1:ic", "s2:klab"]),
    (-0.5, "ab", ["V:kbcd", "s1:ka", "s2:ijcd"]),
    (0.25, "", ["V:klcd", "s2:ijcd", "s2:klab"]),
    (0.5, "ijab", ["V:klcd", "s2:ikac", "s2:ljdb"]),
    (-0.5, "ab", ["V:klcd", "s2:klca", "s2:ijdb"]),
    (-0.5, "ij", ["V:klcd", "s2:kicd", "s2:ljab"]),
    (-0.5, "ijab", ["V:kbcd", "s1:ic", "s1:ka", "s1:jd"]),
    (0.5, "ijab", ["V:klcj", "s1:ic", "s1:ka", "s1:lb"]),
    (0.25, "ij", ["V:klcd", "s1:ic", "s1:jd", "s2:klab"]),
    (0.25, "ab", ["V:klcd", "s1:ka", "s1:lb", "s2:ijcd"]),
    (-1.0, "ijab", ["V:klcd", "s1:ic", "s1:ka", "s2:ljdb"]),
    (-1.0, "ij", ["V:klcd", "s1:kc", "s1:id", "s2:ljab"]),
    (-1.0, "ab", ["V:klcd", "s1:kc", "s1:la", "s2:ijdb"]),
    (0.25, "ijab", ["V:klcd", "s1:ic", "s1:ka", "s1:lb", "s1:jd"]),
]

OUT = {"E": "", "S1": "ia", "S2": "ijab"}
TERMS = {"E": E_TERMS, "S1": S1_TERMS, "S2": S2_TERMS}


def parse(factor: str):
    name, letters = factor.split(":")
    return name, letters


def slot_pattern(letters: str) -> str:
    """'o' for a hole letter, 'v' for a particle letter."""
    out = []
    for ch in letters:
        if ch in HOLE:
            out.append("o")
        elif ch in PART:
            out.append("v")
        else:
            raise ValueError(letters)
    return "".join(out)
