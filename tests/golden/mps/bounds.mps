* Bound types FX, negative UP, PL, BV, LO/UP; a second N row (ignored);
* RHS entries without a set name.
NAME BOUNDS
ROWS
 N  OBJ
 N  OTHER
 G  C1
 L  C2
COLUMNS
    A  OBJ  1.0  C1  1.0
    A  OTHER 5.0
    B  OBJ  -1.0  C1  1.0
    B  C2  1.0
    C  OBJ  2.0  C2  1.0
    D  OBJ  0.5  C1  -1.0
    E  OBJ  -2.0  C2  1.0
RHS
    C1  -2.0
    C2  10.0
BOUNDS
 FX BND A 1.5
 UP BND B -1.0
 PL BND C
 BV BND E
 LO BND D 0.25
 UP BND D 2.0
ENDATA
